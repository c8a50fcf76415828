// k_real.hip -- real-to-complex and complex-to-real stage kernels along the
// last axis (the half spectrum k = 0..N/2 of a real line, footnote of Sec. 2).
//
// A real line of even length N = 2M is read as M complex points
// z_n = x_{2n} + i x_{2n+1}; one M-point complex transform Z and a pairing of
// bins k and M-k then give the N/2+1 output bins:
//   X_k = (Z_k + conj Z_{M-k}) / 2 - (i/2) e^{-2 pi i k/N} (Z_k - conj Z_{M-k}).
// The complex-to-real kernel inverts this: with imag(X_0) = imag(X_M) = 0,
//   Z'_k = (X_k + conj X_{M-k}) + i e^{+2 pi i k/N} (X_k - conj X_{M-k}),
// an M-point inverse transform of Z' gives x_{2n} + i x_{2n+1}, i.e. the sum
// over the Hermitian extension of X (unnormalised).
// Flags turn them into each other's adjoints: SF_DOUBLE_INTERIOR doubles the
// r2c output bins 0 < k < M; SF_HALVE_INTERIOR halves the c2r input bins.
#include <type_traits>

#include "fft_device.hpp"
#include "k_c2c_impl.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

template <typename T2, int M>
struct RealLds {
    static constexpr int LINE = M + M / 8 + 2;
    __device__ static __forceinline__ int idx(int w, int k) { return w * LINE + k + (k >> 3); }
};

// S: the launch shape of the M-point transform (a contiguous-mode C2CCfg).
// Off: element offsets (long in the plans with buffers of 2^31 elements or more).
template <typename T, int NR, int KIND, class S, typename Off = int>
struct RealStage {
    using T2 = typename V2<T>::type;
    static constexpr int M = NR / 2;
    static constexpr int P = S::P, TPL = S::TPL, NL = S::NL, SLOTS = S::SLOTS, W = S::W;
    using LT = LdsTile<T2, M, W, true>;
    using RL = RealLds<T2, M>;
    static constexpr int LDS_N = (LT::SIZE > W * RL::LINE) ? LT::SIZE : W * RL::LINE;
    // the M-point table and the first M entries of the N-point table, staged
    // in LDS once per workgroup where they are small
    static constexpr bool TW_LDS = TwiddleStage<T2, M>::on;
    static constexpr int TW_N = TW_LDS ? 2 * M : 1;

    __device__ static __forceinline__ void stage_twiddles(const StageArgs &a, T2 *twl, const T2 *&tw, const T2 *&tw2)
    {
        tw = (const T2 *)a.twiddle;    // M-point table
        tw2 = (const T2 *)a.twiddle2;  // N-point table
        if constexpr (TW_LDS) {
            for (int i = threadIdx.x; i < M; i += S::NT) {
                twl[i] = tw[i];
                twl[M + i] = tw2[i];
            }
            __syncthreads();
            tw = twl;
            tw2 = twl + M;
        }
    }

    // One tile of the stage (arguments a, tile t), with the twiddle tables of
    // ta staged in twl: with SF_LATE_TWIDDLES while the tile's loads are in
    // flight in complex-to-real stages and in single-precision real-to-complex
    // stages, else before them (double-precision real-to-complex stages
    // measured faster that way).
    static constexpr bool LATE_OK = KIND == KIND_C2R || sizeof(T) == 4;
    __device__ static __forceinline__ void run(const StageArgs &a, const Tile &t, T2 *lds, T2 *twl,
                                               const StageArgs &ta)
    {
        const T2 *tw = nullptr, *tw2 = nullptr;
        const bool late_tw = LATE_OK && (ta.flags & SF_LATE_TWIDDLES);
        if (!late_tw) stage_twiddles(ta, twl, tw, tw2);
        const int count = t.count;
        const int tid = threadIdx.x;
        const int jt = tid % TPL;
        const int slot = tid / TPL;
        int wl[NL];
        bool valid[NL];
#pragma unroll
        for (int l = 0; l < NL; l++) {
            wl[l] = slot + l * SLOTS;
            valid[l] = wl[l] < count;
        }
        const T scale = (T)a.scale;
        T2 v[NL][P];

        if constexpr (KIND == KIND_R2C) {
            // real side: pairs (2n, 2n+1) of real positions, n = jt + m*TPL
            SideAddr<P, Off> rs;
            rs.init(a.side[0], t, 0, 2 * jt, 2 * TPL, NR, true);
            const T *__restrict__ in = (const T *)a.src;
            if (count == W) {
                // whole real lines, each byte read once: streaming loads
#pragma unroll
                for (int l = 0; l < NL; l++)
#pragma unroll
                    for (int m = 0; m < P; m++)
                        v[l][m] = load_stream((const T2 *)(in + rs.off[m] + wl[l] * rs.stride[m]));
            } else {
#pragma unroll
                for (int l = 0; l < NL; l++)
#pragma unroll
                    for (int m = 0; m < P; m++)
                        v[l][m] = valid[l] ? *(const T2 *)(in + rs.off[m] + wl[l] * rs.stride[m]) : c_zero<T2>();
            }
            if (late_tw) stage_twiddles(ta, twl, tw, tw2);
            fft_passes<T2, M, W, true, -1, NL, 1, 0>(v, wl, jt, lds, tw);
            __syncthreads();
#pragma unroll
            for (int l = 0; l < NL; l++)
#pragma unroll
                for (int m = 0; m < P; m++) lds[RL::idx(wl[l], jt + m * TPL)] = v[l][m];
            __syncthreads();
            SideAddr<P, Off> cs;
            cs.init(a.side[1], t, 1, jt, TPL, M + 1, true);
            T2 *__restrict__ out = (T2 *)a.dst;
            const bool dbl = (a.flags & SF_DOUBLE_INTERIOR) != 0;
            // whole destination lines (the half spectrum stays in its block):
            // streaming stores
            const bool stream = a.side[1].R == 0;
#pragma unroll
            for (int l = 0; l < NL; l++) {
                if (!valid[l]) continue;
#pragma unroll
                for (int m = 0; m < P; m++) {
                    const int k = jt + m * TPL;
                    const T2 zk = lds[RL::idx(wl[l], k)];
                    T2 zc = lds[RL::idx(wl[l], k == 0 ? 0 : M - k)];
                    zc.y = -zc.y;
                    const T2 e = c_scale(c_add(zk, zc), (T)0.5);
                    T2 d = c_sub(zk, zc);  // (Z_k - conj Z_{M-k})
                    T2 o;                  // -(i/2) d
                    o.x = d.y * (T)0.5;
                    o.y = -d.x * (T)0.5;
                    T2 x = c_add(e, c_mul(tw2[k], o));
                    T f = scale;
                    if (dbl && k > 0) f *= (T)2;
                    T2 *q = out + cs.off[m] + wl[l] * cs.stride[m];
                    if (stream)
                        store_stream(q, c_scale(x, f));
                    else
                        *q = c_scale(x, f);
                }
                if (jt == 0) {
                    // bin M: E_0 - O_0 = Re Z_0 - Im Z_0
                    const T2 z0 = lds[RL::idx(wl[l], 0)];
                    const Side &sd = a.side[1];
                    const int2 pc = sd.pos[M];
                    const long na = sd.na[pc.x];
                    const long base = sd.rank_off[t.rank[1] + pc.x * sd.R];
                    const long addr = base + ((long)(t.O[1] + wl[l]) * na + pc.y) * t.E[1] + t.I[1];
                    T2 x;
                    x.x = (z0.x - z0.y) * scale;
                    x.y = (T)0;
                    out[addr] = x;
                }
            }
        } else {
            // complex side: bins k = jt + m*TPL and bin M, through LDS
            const T2 *__restrict__ in = (const T2 *)a.src;
            SideAddr<P, Off> cs;
            cs.init(a.side[0], t, 0, jt, TPL, M + 1, true);
            const bool half = (a.flags & SF_HALVE_INTERIOR) != 0;
            // all loads first (a full tile without predicates), then the LDS
            // writes, so the loads are in flight together
            if (count == W) {
#pragma unroll
                for (int l = 0; l < NL; l++)
#pragma unroll
                    for (int m = 0; m < P; m++) v[l][m] = load_stream(in + cs.off[m] + wl[l] * cs.stride[m]);
            } else {
#pragma unroll
                for (int l = 0; l < NL; l++)
#pragma unroll
                    for (int m = 0; m < P; m++)
                        v[l][m] = valid[l] ? in[cs.off[m] + wl[l] * cs.stride[m]] : c_zero<T2>();
            }
            T2 xm[NL];
            if (jt == 0) {
                const Side &sd = a.side[0];
                const int2 pc = sd.pos[M];
                const long na = sd.na[pc.x];
                const long base = sd.rank_off[t.rank[0] + pc.x * sd.R];
#pragma unroll
                for (int l = 0; l < NL; l++) {
                    const long addr = base + ((long)(t.O[0] + wl[l]) * na + pc.y) * t.E[0] + t.I[0];
                    xm[l] = valid[l] ? in[addr] : c_zero<T2>();
                }
            }
            if (late_tw) stage_twiddles(ta, twl, tw, tw2);
#pragma unroll
            for (int l = 0; l < NL; l++) {
#pragma unroll
                for (int m = 0; m < P; m++) {
                    const int k = jt + m * TPL;
                    T2 x = v[l][m];
                    if (k == 0) x.y = (T)0;
                    if (half && k > 0) x = c_scale(x, (T)0.5);
                    lds[RL::idx(wl[l], k)] = x;
                }
                if (jt == 0) {
                    T2 x = xm[l];
                    x.y = (T)0;
                    lds[RL::idx(wl[l], M)] = x;
                }
            }
            __syncthreads();
#pragma unroll
            for (int l = 0; l < NL; l++)
#pragma unroll
                for (int m = 0; m < P; m++) {
                    const int k = jt + m * TPL;
                    const T2 xk = lds[RL::idx(wl[l], k)];
                    T2 xc = lds[RL::idx(wl[l], M - k)];
                    xc.y = -xc.y;
                    const T2 s = c_add(xk, xc);
                    const T2 d = c_sub(xk, xc);
                    T2 w = tw2[k];
                    w.y = -w.y;             // e^{+2 pi i k / N}
                    const T2 wd = c_mul(w, d);
                    T2 z;                   // s + i * wd
                    z.x = s.x - wd.y;
                    z.y = s.y + wd.x;
                    v[l][m] = z;
                }
            __syncthreads();
            fft_passes<T2, M, W, true, 1, NL, 1, 0>(v, wl, jt, lds, tw);
            SideAddr<P, Off> rs;
            rs.init(a.side[1], t, 1, 2 * jt, 2 * TPL, NR, true);
            T *__restrict__ out = (T *)a.dst;
            if (count == W && a.side[1].R == 0) {
                // whole real lines in the destination: streaming stores
#pragma unroll
                for (int l = 0; l < NL; l++)
#pragma unroll
                    for (int m = 0; m < P; m++)
                        store_stream((T2 *)(out + rs.off[m] + wl[l] * rs.stride[m]), c_scale(v[l][m], scale));
            } else {
#pragma unroll
                for (int l = 0; l < NL; l++)
#pragma unroll
                    for (int m = 0; m < P; m++)
                        if (valid[l]) *(T2 *)(out + rs.off[m] + wl[l] * rs.stride[m]) = c_scale(v[l][m], scale);
            }
        }
    }
};

template <typename T, int NR, int KIND, class S, typename Off = int>
__global__ __launch_bounds__(S::NT) void k_real(StageArgs a, const Tile *__restrict__ tiles)
{
    using R = RealStage<T, NR, KIND, S, Off>;
    using T2 = typename R::T2;
    __shared__ T2 lds[R::LDS_N];
    __shared__ T2 twl[R::TW_N];
    R::run(a, tiles[blockIdx.x], lds, twl, a);
}

// The same stage over the tiles of several transforms in one launch (a
// batch): each tile carries the index of its transform's arguments in bits
// 8..31 of its flags; the members share the length, so the twiddle tables of
// the first member serve all.
template <typename T, int NR, int KIND, class S>
__global__ __launch_bounds__(S::NT) void k_real_multi(const StageArgs *__restrict__ args,
                                                      const Tile *__restrict__ tiles)
{
    using R = RealStage<T, NR, KIND, S, int>;
    using T2 = typename R::T2;
    __shared__ T2 lds[R::LDS_N];
    __shared__ T2 twl[R::TW_N];
    const Tile &t = tiles[blockIdx.x];
    R::run(args[t.flags >> 8], t, lds, twl, args[0]);
}

#define PFFT_FOR_EACH_NR(X)                                                                             \
    X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(8192) X(6) X(12) X(24) X(48) X(96) \
        X(192) X(384) X(768) X(1536) X(3072) X(6144)

// Launch shapes: variant 1 (half the lines per tile) where it exists, else
// the default; variant 2 a quarter of the default lines, one line per slot
// (more, smaller workgroups per CU).  (Two lines per slot in quarter-width
// tiles measured no faster than the better of these for either kind.)
template <typename T, int NR>
struct RealQuarter {
    using D = C2CDefault<T, NR / 2, true>;
    static constexpr int W = D::W / 4 >= 1 ? D::W / 4 : 1;
    static constexpr bool exists = D::W >= 4 && D::TPL * W <= 1024;
    using type = C2CCfg<T, NR / 2, true, W, 1>;
};
template <typename T, int NR>
struct RealShape {
    static constexpr bool half = C2CVariant<T, NR / 2, true, 1>::exists;
    template <int V>
    using type = typename std::conditional<V == 2 && RealQuarter<T, NR>::exists, typename RealQuarter<T, NR>::type,
                                           typename C2CVariant<T, NR / 2, true, (V == 1 && half) ? 1 : 0>::type>::type;
};

template <typename T>
static int real_config_t(int NR, int variant, KernelConfig *cfg)
{
    // variant 7: the 64-bit-offset kernel with the default shape (1)
    const int v = (variant == 1 || variant == 7) ? 1 : variant == 2 ? 2 : 0;
    cfg->wide = variant == 7;
    switch (NR) {
#define PFFT_CASE(n)                                                                              \
    case n:                                                                                       \
        cfg->W = v == 2 ? RealShape<T, n>::template type<2>::W                                      \
                        : (v ? RealShape<T, n>::template type<1>::W : RealShape<T, n>::template type<0>::W);   \
        cfg->threads = v == 2 ? RealShape<T, n>::template type<2>::NT                               \
                        : (v ? RealShape<T, n>::template type<1>::NT : RealShape<T, n>::template type<0>::NT); \
        cfg->id = v;                                                                              \
        return 0;
        PFFT_FOR_EACH_NR(PFFT_CASE)
#undef PFFT_CASE
    default:
        return -1;
    }
}

template <typename T, int NR, int V, typename Off = int>
static hipError_t real_launch_v(int kind, const StageArgs &a, hipStream_t s)
{
    using S = typename RealShape<T, NR>::template type<V>;
    dim3 grid((unsigned)a.ntiles);
    if (kind == KIND_R2C)
        PFFT_LAUNCH((k_real<T, NR, KIND_R2C, S, Off>), grid, dim3(S::NT), 0, s, a, a.tiles);
    else
        PFFT_LAUNCH((k_real<T, NR, KIND_C2R, S, Off>), grid, dim3(S::NT), 0, s, a, a.tiles);
    return hipGetLastError();
}

template <typename T, int NR, int V>
static hipError_t real_launch_multi_v(int kind, const StageArgs *args, const Tile *tiles, long nt, hipStream_t s)
{
    using S = typename RealShape<T, NR>::template type<V>;
    dim3 grid((unsigned)(nt < 1 ? 1 : nt));
    if (kind == KIND_R2C)
        PFFT_LAUNCH((k_real_multi<T, NR, KIND_R2C, S>), grid, dim3(S::NT), 0, s, args, tiles);
    else
        PFFT_LAUNCH((k_real_multi<T, NR, KIND_C2R, S>), grid, dim3(S::NT), 0, s, args, tiles);
    return hipGetLastError();
}

template <typename T>
static hipError_t real_launch_multi_t(int NR, int kind, int variant, const StageArgs *args, const Tile *tiles, long nt,
                                      hipStream_t s)
{
    switch (NR) {
#define PFFT_CASE(n)                                                                               \
    case n:                                                                                        \
        return variant == 1   ? real_launch_multi_v<T, n, 1>(kind, args, tiles, nt, s)            \
               : variant == 2 ? real_launch_multi_v<T, n, 2>(kind, args, tiles, nt, s)            \
                              : real_launch_multi_v<T, n, 0>(kind, args, tiles, nt, s);
        PFFT_FOR_EACH_NR(PFFT_CASE)
#undef PFFT_CASE
    default:
        return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t real_launch_t(int NR, int kind, int variant, int wide, const StageArgs &a, hipStream_t s)
{
    switch (NR) {
#define PFFT_CASE(n)                                                                      \
    case n:                                                                               \
        return wide ? real_launch_v<T, n, 1, long>(kind, a, s)                            \
                    : (variant == 1   ? real_launch_v<T, n, 1>(kind, a, s)                  \
                       : variant == 2 ? real_launch_v<T, n, 2>(kind, a, s)                  \
                                      : real_launch_v<T, n, 0>(kind, a, s));
        PFFT_FOR_EACH_NR(PFFT_CASE)
#undef PFFT_CASE
    default:
        return hipErrorInvalidValue;
    }
}

int real_config(int prec, int N, int kind, int variant, KernelConfig *cfg)
{
    (void)kind;
    return prec == 0 ? real_config_t<float>(N, variant, cfg) : real_config_t<double>(N, variant, cfg);
}

hipError_t real_launch_multi(int prec, int N, int kind, const KernelConfig &cfg, const StageArgs *args,
                             const Tile *tiles, long nt, hipStream_t s)
{
    return prec == 0 ? real_launch_multi_t<float>(N, kind, cfg.id, args, tiles, nt, s)
                     : real_launch_multi_t<double>(N, kind, cfg.id, args, tiles, nt, s);
}

hipError_t real_launch(int prec, int N, int kind, const KernelConfig &cfg, const StageArgs &a, hipStream_t s)
{
    return prec == 0 ? real_launch_t<float>(N, kind, cfg.id, cfg.wide, a, s)
                     : real_launch_t<double>(N, kind, cfg.id, cfg.wide, a, s);
}

}  // namespace pfft
