// k_c2c_impl.hpp -- host dispatch over the instantiated lengths and tile
// shapes of k_c2c.
#pragma once

#include <type_traits>

#include "k_c2c.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

// Number of workgroups of `kernel` (nt threads, static LDS only) that can be
// resident on the whole device at once.
int resident_workgroups(const void *kernel, int nt);

// Tile-shape variants: 0 the default, 1 half the lines per tile (more
// workgroups per CU), 2 twice the lines (wider rows, one workgroup per CU),
// 3 twice the lines exchanged through the default LDS in two portions (wider
// rows, two workgroups per CU).
template <typename T, int N, bool CONTIG, int V>
struct C2CVariant {
    using D = C2CDefault<T, N, CONTIG>;
    static constexpr int VEC = D::VEC;
    static constexpr int LDS_BYTES_2W = (CONTIG ? 2 * D::W * (N + N / 8) : N * (2 * D::W + 16 / (2 * (int)sizeof(T)))) *
                                        2 * (int)sizeof(T);
    static constexpr bool multi = fft_npasses(N) > 1 && N >= 32;
    static constexpr bool has_half = multi && D::W / 2 >= VEC;
    static constexpr bool has_double = multi && LDS_BYTES_2W <= 150 * 1024;
    static constexpr bool has_split = multi && D::W * 2 <= 128 && (2 * D::NL / 2) % VEC == 0;
    // 4: four times the lines, 1024 threads, exchanged in two portions of 2W lines
    static constexpr bool has_quad = multi && LDS_BYTES_2W <= 150 * 1024 && D::TPL * 4 * D::W / (2 * D::NL) <= 1024 &&
                                     D::W * 4 <= 256;
    static constexpr int W = V == 1 && has_half ? D::W / 2
                             : ((V == 2 && has_double) || (V == 3 && has_split)) ? 2 * D::W
                             : (V == 4 && has_quad) ? 4 * D::W
                                                    : D::W;
    static constexpr int NL0 = (V == 2 && has_double) || (V == 3 && has_split) || (V == 4 && has_quad) ? 2 * D::NL
                                                                                                         : D::NL;
    static constexpr int NL = (W % NL0 == 0) ? NL0 : VEC;
    static constexpr int H = (V == 3 && has_split) || (V == 4 && has_quad) ? 2 : 1;
    using type = C2CCfg<T, N, CONTIG, W, NL, H>;
    static constexpr bool exists =
        V == 0 || (V == 1 && has_half) || (V == 2 && has_double) || (V == 3 && has_split) || (V == 4 && has_quad);
};

template <typename T, int N, bool CONTIG, int SIGN, int V>
static hipError_t c2c_launch_v(const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    using S = typename C2CVariant<T, N, CONTIG, V>::type;
    const void *fn = (const void *)&k_c2c<T, N, CONTIG, SIGN, S>;
    long g = a.ntiles;
    if (c.resident) {
        static const int resident = resident_workgroups(fn, S::NT);
        if (g > resident) g = resident;
    }
    if (g < 1) g = 1;
    PFFT_LAUNCH((k_c2c<T, N, CONTIG, SIGN, S>), dim3((unsigned)g), dim3(S::NT), 0, s, a, a.tiles);
    return hipGetLastError();
}

// Slot-group shapes of strided stages: NTT threads, NLM line pairs
// (complex64) or lines (complex128) per thread and slot, at most 12 points
// per thread (lengths of 16 or 24 take their alternative plans of 8 and 12),
// so a tile is as wide as the thread count allows (W = NLM * VEC * NTT / TPL
// lines); the LDS exchanges in the fewest slot-group portions whose rows fit
// WGS workgroups per CU.  Variants (tile_strided value in brackets):
//   9 (6):  512 threads, two workgroups per CU, lines of 1024 points and more
//   10 (7): 1024 threads, one workgroup per CU, lines of 1024 points and more
// (Wider tiles of this kind -- 1024 threads with one or two pairs per slot --
// measured 1.2-3x slower than the default shapes on lines of 256-768 points.)
template <typename T, int N, int NTT, int NLM, int WGS, int NMIN>
struct C2CSlotShape {
    using T2 = typename V2<T>::type;
    static constexpr int VEC = sizeof(T) == 4 ? 2 : 1;
    static constexpr int ESZ = 2 * (int)sizeof(T);
    static constexpr int ALT = (fft_points(N) > 12 && fft_p2_alt(N) != fft_p2(N)) ? 1 : 0;
    static constexpr int TPL = N / fft_points_a(N, ALT);
    static constexpr int SLOTS = TPL <= NTT ? NTT / TPL : 0;
    static constexpr int NL = NLM * VEC;
    static constexpr int W = SLOTS * NL;
    static constexpr int PADW = PFFT_STRIDED_PAD_BYTES / ESZ;
    static constexpr int CAP = 158 * 1024 / WGS - (TwiddleStage<T2, N>::on ? N * ESZ : 0);
    static constexpr int lds_bytes(int hs) { return N * (W / hs + PADW) * ESZ; }
    static constexpr int pick(int hs) { return hs > SLOTS ? 0 : (lds_bytes(hs) <= CAP ? hs : pick(hs * 2)); }
    static constexpr int HS = SLOTS > 0 ? pick(1) : 0;
    static constexpr bool exists = N >= NMIN && fft_npasses(N) > 1 && HS >= 1 && SLOTS % (HS > 0 ? HS : 1) == 0;
    using type = C2CCfg<T, N, false, exists ? W : VEC, exists ? NL : VEC, 1, ALT, exists ? HS : 1>;
};

template <typename T, int N, int ID>
struct C2CSlot;
template <typename T, int N>
struct C2CSlot<T, N, 9> : C2CSlotShape<T, N, 512, 1, 2, 1024> {};
template <typename T, int N>
struct C2CSlot<T, N, 10> : C2CSlotShape<T, N, 1024, 1, 1, 1024> {};

template <typename T, int N, int SIGN, int ID>
static hipError_t c2c_launch_slot(const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    using S = typename C2CSlot<T, N, ID>::type;
    (void)c;
    long g = a.ntiles < 1 ? 1 : a.ntiles;
    PFFT_LAUNCH((k_c2c<T, N, false, SIGN, S>), dim3((unsigned)g), dim3(S::NT), 0, s, a, a.tiles);
    return hipGetLastError();
}

// The alternative radix plan with the measured default tile shape of the
// mode (lines per tile and LDS portions of that shape, lines per thread
// chosen for at most 512 threads).
template <typename T, int N, bool CONTIG>
struct C2CAlt {
    static constexpr int VD = CONTIG ? 1 : (N >= 1024 ? 4 : 3);
    using Base = typename C2CVariant<T, N, CONTIG, C2CVariant<T, N, CONTIG, VD>::exists ? VD : 0>::type;
    static constexpr int W = Base::W, H = Base::H, VEC = Base::VEC;
    static constexpr int TPLA = N / fft_points_a(N, 1);
    static constexpr int nl_for(int nl) { return (TPLA * W / nl > 512 && nl < W) ? nl_for(nl * 2) : nl; }
    static constexpr int NL = nl_for(H * VEC);
    static constexpr bool exists =
        N >= 32 && fft_p2_alt(N) != fft_p2(N) && W % NL == 0 && TPLA * (W / NL) <= 512 && TPLA >= 1;
    using type = C2CCfg<T, N, CONTIG, W, exists ? NL : Base::NL, H, exists ? 1 : 0>;
};

template <typename T, int N, bool CONTIG, int SIGN>
static hipError_t c2c_launch_alt(const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    using S = typename C2CAlt<T, N, CONTIG>::type;
    (void)c;
    long g = a.ntiles < 1 ? 1 : a.ntiles;
    PFFT_LAUNCH((k_c2c<T, N, CONTIG, SIGN, S>), dim3((unsigned)g), dim3(S::NT), 0, s, a, a.tiles);
    return hipGetLastError();
}

// The stage of plans with buffers of 2^31 elements or more, with the
// measured default tile shape of the kernel's mode; strided lines of 1536
// points and more take the long-line shapes (512 threads at 1536, 1024
// beyond), as in the plan's rule.
template <typename T, int N, bool CONTIG>
struct C2CWideShape {
    static constexpr int V = C2CVariant<T, N, CONTIG, CONTIG ? 1 : 3>::exists ? (CONTIG ? 1 : 3) : 0;
    static constexpr int ID = N == 1536 ? 9 : 10;
    static constexpr bool use_long = !CONTIG && N >= 1536 && C2CSlot<T, N, ID>::exists;
    using type = typename std::conditional<use_long, typename C2CSlot<T, N, ID>::type,
                                           typename C2CVariant<T, N, CONTIG, V>::type>::type;
};

// The stage whose destination lines step the other way (XS): as above;
// contiguous-mode kernels take tile variant PFFT_XS_CONTIG_VARIANT.
#ifndef PFFT_XS_CONTIG_VARIANT
#define PFFT_XS_CONTIG_VARIANT 1
#endif
template <typename T, int N, bool CONTIG>
struct C2CXsShape {
    static constexpr int VC = PFFT_XS_CONTIG_VARIANT;
    static constexpr bool own = CONTIG && C2CVariant<T, N, true, VC>::exists;
    static constexpr int V = own ? VC : C2CWideShape<T, N, CONTIG>::V;
    using type = typename std::conditional<own, typename C2CVariant<T, N, true, VC>::type,
                                           typename C2CWideShape<T, N, CONTIG>::type>::type;
};

template <typename T, int N, bool CONTIG, int SIGN>
static hipError_t c2c_launch_xs(const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    using S = typename C2CXsShape<T, N, CONTIG>::type;
    (void)c;
    long g = a.ntiles < 1 ? 1 : a.ntiles;
    PFFT_LAUNCH((k_c2c<T, N, CONTIG, SIGN, S, true>), dim3((unsigned)g), dim3(S::NT), 0, s, a, a.tiles);
    return hipGetLastError();
}

// The stage of plans with buffers of 2^31 elements or more: 64-bit offsets,
// the same default tile shape, one tile per workgroup.
template <typename T, int N, bool CONTIG, int SIGN>
static hipError_t c2c_launch_wide(const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    using S = typename C2CWideShape<T, N, CONTIG>::type;
    (void)c;
    long g = a.ntiles < 1 ? 1 : a.ntiles;
    PFFT_LAUNCH((k_c2c<T, N, CONTIG, SIGN, S, false, long>), dim3((unsigned)g), dim3(S::NT), 0, s, a,
                       a.tiles);
    return hipGetLastError();
}

template <typename T, int N, bool CONTIG, int SIGN, int V>
static hipError_t c2c_launch_multi_v(const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                                     hipStream_t s)
{
    using S = typename C2CVariant<T, N, CONTIG, V>::type;
    const void *fn = (const void *)&k_c2c_multi<T, N, CONTIG, SIGN, S>;
    long g = nt;
    if (c.resident) {
        static const int resident = resident_workgroups(fn, S::NT);
        if (g > resident) g = resident;
    }
    if (g < 1) g = 1;
    PFFT_LAUNCH((k_c2c_multi<T, N, CONTIG, SIGN, S>), dim3((unsigned)g), dim3(S::NT), 0, s, args, tiles, nt);
    return hipGetLastError();
}

template <typename T, int N, bool CONTIG, int SIGN>
static hipError_t c2c_launch_multi_s(const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                                     hipStream_t s)
{
    switch (c.id) {
    case 1:
        if constexpr (C2CVariant<T, N, CONTIG, 1>::exists)
            return c2c_launch_multi_v<T, N, CONTIG, SIGN, 1>(c, args, tiles, nt, s);
        break;
    case 2:
        if constexpr (C2CVariant<T, N, CONTIG, 2>::exists)
            return c2c_launch_multi_v<T, N, CONTIG, SIGN, 2>(c, args, tiles, nt, s);
        break;
    case 3:
        if constexpr (C2CVariant<T, N, CONTIG, 3>::exists)
            return c2c_launch_multi_v<T, N, CONTIG, SIGN, 3>(c, args, tiles, nt, s);
        break;
    case 4:
        if constexpr (C2CVariant<T, N, CONTIG, 4>::exists)
            return c2c_launch_multi_v<T, N, CONTIG, SIGN, 4>(c, args, tiles, nt, s);
        break;
    default: break;
    }
    return c2c_launch_multi_v<T, N, CONTIG, SIGN, 0>(c, args, tiles, nt, s);
}

template <typename T, int N, bool CONTIG, int SIGN>
static hipError_t c2c_launch_s(const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    if (c.xside) return c2c_launch_xs<T, N, CONTIG, SIGN>(c, a, s);
    if (c.wide) return c2c_launch_wide<T, N, CONTIG, SIGN>(c, a, s);
    if (c.alt) {
        if constexpr (C2CAlt<T, N, CONTIG>::exists) return c2c_launch_alt<T, N, CONTIG, SIGN>(c, a, s);
    }
    switch (c.id) {
    case 9:
        if constexpr (!CONTIG && C2CSlot<T, N, 9>::exists) return c2c_launch_slot<T, N, SIGN, 9>(c, a, s);
        break;
    case 10:
        if constexpr (!CONTIG && C2CSlot<T, N, 10>::exists) return c2c_launch_slot<T, N, SIGN, 10>(c, a, s);
        break;
    case 1:
        if constexpr (C2CVariant<T, N, CONTIG, 1>::exists) return c2c_launch_v<T, N, CONTIG, SIGN, 1>(c, a, s);
        break;
    case 2:
        if constexpr (C2CVariant<T, N, CONTIG, 2>::exists) return c2c_launch_v<T, N, CONTIG, SIGN, 2>(c, a, s);
        break;
    case 3:
        if constexpr (C2CVariant<T, N, CONTIG, 3>::exists) return c2c_launch_v<T, N, CONTIG, SIGN, 3>(c, a, s);
        break;
    case 4:
        if constexpr (C2CVariant<T, N, CONTIG, 4>::exists) return c2c_launch_v<T, N, CONTIG, SIGN, 4>(c, a, s);
        break;
    default: break;
    }
    return c2c_launch_v<T, N, CONTIG, SIGN, 0>(c, a, s);
}

template <typename T, int N, int ID>
static bool c2c_slot_cfg(int variant, KernelConfig *c)
{
    if constexpr (C2CSlot<T, N, ID>::exists) {
        if (variant == ID) {
            c->W = C2CSlot<T, N, ID>::type::W;
            c->threads = C2CSlot<T, N, ID>::type::NT;
            c->id = ID;
            return true;
        }
    }
    return false;
}

template <typename T, int N, bool CONTIG>
static void c2c_cfg_mode(int variant, KernelConfig *c)
{
    int W, NT, id;
    if (variant == 8) {  // the alternative radix plan, where the length has one
        if constexpr (C2CAlt<T, N, CONTIG>::exists) {
            c->W = C2CAlt<T, N, CONTIG>::type::W;
            c->threads = C2CAlt<T, N, CONTIG>::type::NT;
            c->id = 8;
            c->alt = 1;
            return;
        }
        variant = CONTIG ? 1 : (N >= 1024 ? 4 : 3);
    }
    if (variant == 9 || variant == 10) {  // the slot-group shapes of strided stages
        if constexpr (!CONTIG) {
            if (c2c_slot_cfg<T, N, 9>(variant, c) || c2c_slot_cfg<T, N, 10>(variant, c)) return;
        }
        variant = CONTIG ? 1 : (N >= 1024 ? 4 : 3);
    }
    if (variant == 6) {  // the shape of the XS stage
        c->W = C2CXsShape<T, N, CONTIG>::type::W;
        c->threads = C2CXsShape<T, N, CONTIG>::type::NT;
        c->id = C2CXsShape<T, N, CONTIG>::V;
        c->xside = 1;
        return;
    }
    if (variant == 7) {  // the shape of the 64-bit-offset stage
        c->W = C2CWideShape<T, N, CONTIG>::type::W;
        c->threads = C2CWideShape<T, N, CONTIG>::type::NT;
        c->id = C2CWideShape<T, N, CONTIG>::V;
        c->wide = 1;
        return;
    }
    if (variant == 1 && C2CVariant<T, N, CONTIG, 1>::exists) {
        W = C2CVariant<T, N, CONTIG, 1>::type::W;
        NT = C2CVariant<T, N, CONTIG, 1>::type::NT;
        id = 1;
    } else if (variant == 2 && C2CVariant<T, N, CONTIG, 2>::exists) {
        W = C2CVariant<T, N, CONTIG, 2>::type::W;
        NT = C2CVariant<T, N, CONTIG, 2>::type::NT;
        id = 2;
    } else if (variant == 3 && C2CVariant<T, N, CONTIG, 3>::exists) {
        W = C2CVariant<T, N, CONTIG, 3>::type::W;
        NT = C2CVariant<T, N, CONTIG, 3>::type::NT;
        id = 3;
    } else if (variant == 4 && C2CVariant<T, N, CONTIG, 4>::exists) {
        W = C2CVariant<T, N, CONTIG, 4>::type::W;
        NT = C2CVariant<T, N, CONTIG, 4>::type::NT;
        id = 4;
    } else {
        W = C2CVariant<T, N, CONTIG, 0>::type::W;
        NT = C2CVariant<T, N, CONTIG, 0>::type::NT;
        id = 0;
    }
    c->W = W;
    c->threads = NT;
    c->id = id;
}

template <typename T, int N>
static void c2c_cfg_n(int contig, int variant, KernelConfig *c)
{
    if (contig)
        c2c_cfg_mode<T, N, true>(variant, c);
    else
        c2c_cfg_mode<T, N, false>(variant, c);
}

#define PFFT_FOR_EACH_N(X)                                                                          \
    X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(3) X(6) X(12) X(24) \
        X(48) X(96) X(192) X(384) X(768) X(1536) X(3072)

template <typename T>
static int c2c_config_t(int N, int contig, int variant, KernelConfig *cfg)
{
    switch (N) {
#define PFFT_CASE(n)                           \
    case n:                                    \
        c2c_cfg_n<T, n>(contig, variant, cfg); \
        return 0;
        PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
    default:
        return -1;
    }
}

// One translation unit per (precision, mode, sign) instantiates the kernels of
// every length for that combination (keeps parallel builds short).
template <typename T, bool CONTIG, int SIGN>
static hipError_t c2c_launch_ms(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    switch (N) {
#define PFFT_CASE(n) \
    case n:          \
        return c2c_launch_s<T, n, CONTIG, SIGN>(c, a, s);
        PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
    default:
        return hipErrorInvalidValue;
    }
}

template <typename T, bool CONTIG, int SIGN>
static hipError_t c2c_launch_multi_ms(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                                      hipStream_t s)
{
    switch (N) {
#define PFFT_CASE(n) \
    case n:          \
        return c2c_launch_multi_s<T, n, CONTIG, SIGN>(c, args, tiles, nt, s);
        PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t c2c_f32_c_fwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s);
hipError_t c2c_multi_f32_c_fwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s);
hipError_t c2c_f32_c_bwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s);
hipError_t c2c_multi_f32_c_bwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s);
hipError_t c2c_f32_s_fwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s);
hipError_t c2c_multi_f32_s_fwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s);
hipError_t c2c_f32_s_bwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s);
hipError_t c2c_multi_f32_s_bwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s);
hipError_t c2c_f64_c_fwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s);
hipError_t c2c_multi_f64_c_fwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s);
hipError_t c2c_f64_c_bwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s);
hipError_t c2c_multi_f64_c_bwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s);
hipError_t c2c_f64_s_fwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s);
hipError_t c2c_multi_f64_s_fwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s);
hipError_t c2c_f64_s_bwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s);
hipError_t c2c_multi_f64_s_bwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s);

}  // namespace pfft
