// k_c2c.hpp -- the complex partial-transform stage kernel (one template,
// instantiated per precision in k_c2c_f32.hip / k_c2c_f64.hip).
//
// A workgroup transforms tiles of up to W lines of N points along the
// transform axis.  Each line is read from the source layout's rank blocks
// (a line along an axis split over a grid direction is read from every rank
// of that direction's subgroup: the subarray gather of the exchange) and
// written to the destination layout's blocks, so a redistribution followed by
// a partial transform costs one read and one write of the data.
//
// Strided tiles (transform axis is not the last axis): the tile's lines are
// adjacent in memory, so lanes run across lines and every point of the tile
// is a coalesced row of W elements; fp32 lanes move two lines per 16-byte
// access.  Contiguous tiles (last axis): lanes run along the line.
//
// A workgroup walks the tile list with a stride of gridDim.x: launched with
// one workgroup per tile it runs one tile; launched with the number of
// workgroups the device holds at once it loops (a persistent grid).
#pragma once

#include "fft_device.hpp"

namespace pfft {

template <typename T, int N, bool CONTIG, int W_, int NL_, int H_ = 1, int ALT_ = 0, int HS_ = 1>
struct C2CCfg {
    static constexpr int ALT = ALT_;                                 // alternative radix plan
    static constexpr int HS = HS_;                                   // LDS portions over slot groups
    static constexpr int P = fft_points_a(N, ALT_);
    static constexpr int TPL = N / P;                                // threads per line slot
    static constexpr int VEC = (!CONTIG && sizeof(T) == 4) ? 2 : 1;  // lines per access
    static constexpr int W = W_;                                     // lines per tile
    static constexpr int NL = NL_;                                   // lines per thread
    static constexpr int SLOTS = W / NL;                             // line slots per pass
    static constexpr int NT = TPL * SLOTS;                           // threads per workgroup
    static constexpr int H = H_;                                     // LDS portions per exchange
    static constexpr int WL = W / (H * HS_);                         // lines held in LDS at once
    static_assert(W % NL == 0 && NL % VEC == 0, "tile shape");
    static_assert(NL % H == 0 && W % H == 0 && (NL / H) % VEC == 0, "LDS portions");
    static_assert(HS_ == 1 || (H_ == 1 && !CONTIG && SLOTS % HS_ == 0), "slot-group portions");
    static_assert(NT <= 1024, "workgroup too large");
};

// Default launch shape per (precision, N, mode): about 64-74 KB of LDS per
// workgroup (two workgroups per CU), at most 512 threads.
template <typename T, int N, bool CONTIG>
struct C2CDefault {
    static constexpr int VEC = (!CONTIG && sizeof(T) == 4) ? 2 : 1;
    static constexpr int ESZ = 2 * (int)sizeof(T);
    static constexpr int TPL = N / fft_points(N);
    static constexpr int W0 = (fft_npasses(N) > 1) ? (64 * 1024) / (N * ESZ) : 128;
    static constexpr int floor_pow2(int x) { return x < 2 ? 1 : 2 * floor_pow2(x / 2); }
    static constexpr int W1 = floor_pow2(W0 > 64 && fft_npasses(N) > 1 ? 64 : W0);
    static constexpr int W = W1 < VEC ? VEC : W1;
    static constexpr int nl_for(int nl) { return (TPL * W / nl > 512 && nl < W) ? nl_for(nl * 2) : nl; }
    static constexpr int NL = nl_for(VEC);
    using type = C2CCfg<T, N, CONTIG, W, NL>;
};

// STREAM: strided tiles may use streaming loads / stores (SF_LOAD_NT,
// SF_STORE_NT); without it those paths are not generated.  XS: the
// destination's lines step the other way (a stage into or out of a layout
// with another storage order: lines adjacent on one side, each line
// contiguous on the other); loads keep the kernel's mode, stores go point by
// point to line w at O + w (strided kernels) or I + w (contiguous kernels).
template <typename T, int N, bool CONTIG, int SIGN, class S, bool STREAM = true, bool XS = false,
          typename Off = int>
struct C2CWorker {
    using T2 = typename V2<T>::type;
    using T4 = typename V2<T>::quad;
    static constexpr int P = S::P, TPL = S::TPL, VEC = S::VEC, NL = S::NL, SLOTS = S::SLOTS, W = S::W;
    using LT = LdsTile<T2, N, S::WL, CONTIG>;
    // XS stages with line portions stage their stores through the LDS tile
    static constexpr bool XS_STAGED = XS && S::HS == 1;
    static constexpr int LDS_SIZE = (fft_npasses_a(N, S::ALT) > 1 || XS_STAGED) ? LT::SIZE : 1;

    int jt, slot;
    int wl[NL];
    // with portions over slot groups: the thread's group and its lines
    // numbered inside the group (the LDS rows it uses)
    static constexpr int SPG = SLOTS / S::HS;
    int grp = 0;
    int wg[S::HS > 1 ? NL : 1];

    // Make the thread geometry opaque to the optimiser once per tile, so the
    // per-position LDS offsets and twiddle indices are recomputed instead of
    // being hoisted out of the tile loop into (many) live registers.
    __device__ __forceinline__ void refresh()
    {
        asm volatile("" : "+v"(jt));
#pragma unroll
        for (int l = 0; l < NL; l++) asm volatile("" : "+v"(wl[l]));
        if constexpr (S::HS > 1) {
#pragma unroll
            for (int l = 0; l < NL; l++) asm volatile("" : "+v"(wg[l]));
        }
    }

    __device__ __forceinline__ void init_geometry()
    {
        const int tid = threadIdx.x;
        if constexpr (CONTIG) {
            jt = tid % TPL;
            slot = tid / TPL;
        } else {
            slot = tid % SLOTS;
            jt = tid / SLOTS;
        }
#pragma unroll
        for (int l = 0; l < NL; l++) {
            if constexpr (CONTIG)
                wl[l] = slot + l * SLOTS;
            else
                wl[l] = (slot + (l / VEC) * SLOTS) * VEC + (l % VEC);
        }
        if constexpr (S::HS > 1) {
            grp = slot / SPG;
#pragma unroll
            for (int l = 0; l < NL; l++) wg[l] = (slot % SPG + (l / VEC) * SPG) * VEC + (l % VEC);
        }
    }

    // Element offset of each of this thread's lines from line 0 of the tile
    // (strided mode; stride 1 between lines of a run, ostr between runs).
    __device__ __forceinline__ void line_offsets(const Tile &t, int s, int (&lo)[NL]) const
    {
        if (t.run == 0) {
#pragma unroll
            for (int l = 0; l < NL; l++) lo[l] = wl[l];
            return;
        }
        const unsigned run = (unsigned)t.run, b0 = (unsigned)t.b0;
        const int ostr = t.ostr[s];
#pragma unroll
        for (int l = 0; l < NL; l++) {
            const unsigned q = b0 + (unsigned)wl[l];
            const unsigned k = q / run;
            lo[l] = (int)(q - k * run) + (int)k * ostr;
        }
    }

    // Element offset of line l at position m.
    __device__ __forceinline__ static Off at(const SideAddr<P, Off> &sa, const int (&lo)[NL], const int (&wl_)[NL],
                                             int l, int m)
    {
        if constexpr (CONTIG)
            return sa.off[m] + wl_[l] * sa.stride[m];
        else
            return sa.off[m] + lo[l];
    }

    // Compute both sides' addresses of tile `ti` and issue its loads.  A full
    // tile whose addresses are even on both sides (Tile flag bit 0) takes the
    // unpredicated path; others are predicated line by line.
    __device__ __forceinline__ void load(const StageArgs &a, const Tile &t, T2 (&v)[NL][P], SideAddr<P, Off> &dst,
                                         int &count) const
    {
        count = t.count;
        const bool fast = (t.count == W) && (VEC == 1 || (t.flags & 1));
        if (!fast) count = -count;  // sign marks the predicated path for process()
        SideAddr<P, Off> src;
        src.init(a.side[0], t, 0, jt, TPL, N, CONTIG);
        dst.init(a.side[1], t, 1, jt, TPL, N, XS ? !CONTIG : CONTIG);
        const T2 *__restrict__ in = (const T2 *)a.src;
        int lo[NL];
        if constexpr (!CONTIG) line_offsets(t, 0, lo);
        if (fast && CONTIG) {
            // lines along the last axis (whole, or gathered in pieces):
            // streaming loads where the stage asks for them (always in the
            // multi-transform kernel)
            const bool nt = !STREAM || (a.flags & SF_LOAD_NT) != 0;
#pragma unroll
            for (int l = 0; l < NL; l++)
#pragma unroll
                for (int m = 0; m < P; m++) {
                    const T2 *p2 = in + src.off[m] + wl[l] * src.stride[m];
                    v[l][m] = nt ? load_stream(p2) : *p2;
                }
        } else if (fast) {
            // rows of adjacent lines; streaming loads where the stage asks for them
            const bool nt = STREAM && (a.flags & SF_LOAD_NT) != 0;
#pragma unroll
            for (int l = 0; l < NL; l += VEC)
#pragma unroll
                for (int m = 0; m < P; m++) {
                    if constexpr (VEC == 2) {
                        const T4 *p4 = (const T4 *)(in + at(src, lo, wl, l, m));
                        T4 q = nt ? load_stream(p4) : *p4;
                        v[l][m].x = q.x;
                        v[l][m].y = q.y;
                        v[l + 1][m].x = q.z;
                        v[l + 1][m].y = q.w;
                    } else {
                        const T2 *p2 = in + at(src, lo, wl, l, m);
                        v[l][m] = nt ? load_stream(p2) : *p2;
                    }
                }
        } else {
            const int cnt = t.count;
#pragma unroll
            for (int l = 0; l < NL; l++) {
                const bool ok = wl[l] < cnt;
#pragma unroll
                for (int m = 0; m < P; m++) v[l][m] = ok ? in[at(src, lo, wl, l, m)] : c_zero<T2>();
            }
        }
    }

    // Store of an XS stage through the LDS tile, one portion of WL lines at a
    // time: the transformed lines are written in the kernel's LDS layout and
    // read back in the destination's order, so the stores coalesce.  A
    // contiguous-mode kernel (destination lines adjacent, point j of line w at
    // off(j) + w) stores with lanes across the lines of the portion; a
    // strided-mode kernel (destination lines contiguous) stores with up to 64
    // lanes along a line.
    __device__ __forceinline__ void xs_store_staged(const StageArgs &a, const Tile &t, T2 (&v)[NL][P], int cnt,
                                                    T2 *lds) const
    {
        constexpr int H = S::H, WL = S::WL, NT = S::NT, NLH = NL / H;
        T2 *__restrict__ out = (T2 *)a.dst;
        const int tid = threadIdx.x;
        if constexpr (CONTIG) {
            static_assert(NT % WL == 0 && (N * WL) % NT == 0, "staged store geometry");
            constexpr int SJ = NT / WL;           // threads per line position set
            constexpr int NV = N * WL / NT;       // points per thread and portion
            const int sw = tid % WL, sj = tid / WL;
            SideAddr<NV, Off> sd;
            sd.init(a.side[1], t, 1, sj, SJ, N, false);
#pragma unroll
            for (int h = 0; h < H; h++) {
                __syncthreads();
#pragma unroll
                for (int l = h * NLH; l < (h + 1) * NLH; l++)
#pragma unroll
                    for (int m = 0; m < P; m++) lds[LT::idx(wl[l] - h * WL, jt + m * TPL)] = v[l][m];
                __syncthreads();
                const int w = h * WL + sw;
                if (w < cnt) {
#pragma unroll
                    for (int k = 0; k < NV; k++) out[sd.off[k] + (Off)w] = lds[LT::idx(sw, sj + k * SJ)];
                }
            }
        } else {
            constexpr int SJ = (N % 64 == 0) ? 64 : (N % 32 == 0) ? 32 : (N % 16 == 0) ? 16 : (N % 8 == 0) ? 8 : 1;
            constexpr int LP = NT / SJ;            // lines stored per pass
            constexpr int NV = N / SJ;             // points per thread and line
            static_assert(NT % SJ == 0, "staged store geometry");
            const int sj = tid % SJ, sw = tid / SJ;
            SideAddr<NV, Off> sd;
            sd.init(a.side[1], t, 1, sj, SJ, N, true);
#pragma unroll
            for (int h = 0; h < H; h++) {
                __syncthreads();
#pragma unroll
                for (int l = h * NLH; l < (h + 1) * NLH; l++)
#pragma unroll
                    for (int m = 0; m < P; m++) lds[LT::idx(wl[l] - h * WL, jt + m * TPL)] = v[l][m];
                __syncthreads();
#pragma unroll
                for (int wloc = sw; wloc < WL; wloc += LP) {
                    const int w = h * WL + wloc;
                    if (w < cnt) {
#pragma unroll
                        for (int k = 0; k < NV; k++) out[sd.off[k] + (Off)w * sd.stride[k]] = lds[LT::idx(wloc, sj + k * SJ)];
                    }
                }
            }
        }
        __syncthreads();  // the LDS reads are done before any later use of the tile
    }

    // Transform the registers of one tile (LDS-staged passes), scale, store.
    __device__ __forceinline__ void process(const StageArgs &a, const Tile &t, T2 (&v)[NL][P],
                                            const SideAddr<P, Off> &dst, int count, T2 *lds, const T2 *tw) const
    {
        if constexpr (fft_npasses_a(N, S::ALT) > 1) __syncthreads();  // the previous tile's last LDS reads are done
        if constexpr (S::HS > 1)
            fft_passes<T2, N, S::WL, CONTIG, SIGN, NL, 1, 0, S::ALT, S::HS>(v, wg, jt, lds, tw, grp);
        else
            fft_passes<T2, N, S::WL, CONTIG, SIGN, NL, S::H, 0, S::ALT>(v, wl, jt, lds, tw);
        const T scale = (T)a.scale;
        if (scale != (T)1) {
#pragma unroll
            for (int l = 0; l < NL; l++)
#pragma unroll
                for (int m = 0; m < P; m++) v[l][m] = c_scale(v[l][m], scale);
        }
        T2 *__restrict__ out = (T2 *)a.dst;
        if constexpr (XS_STAGED) {
            xs_store_staged(a, t, v, count > 0 ? count : -count, lds);
            return;
        }
        if constexpr (XS) {
            // line w of the destination at dst.off[m] + w * dst.stride[m]
            const int cnt = count > 0 ? count : -count;
#pragma unroll
            for (int l = 0; l < NL; l++) {
                const bool ok = wl[l] < cnt;
#pragma unroll
                for (int m = 0; m < P; m++)
                    if (ok) out[dst.off[m] + wl[l] * dst.stride[m]] = v[l][m];
            }
            return;
        }
        // Whole destination lines along the last axis are written with
        // streaming stores where the stage asks for them (always in the
        // multi-transform kernel); rows of strided tiles and line segments
        // scattered over several blocks with ordinary stores.
        const bool stream = CONTIG && a.side[1].R == 0 && (!STREAM || (a.flags & SF_STORE_NT) != 0);
        int lo[NL];
        if constexpr (!CONTIG) line_offsets(t, 1, lo);
        if (count > 0 && stream) {
#pragma unroll
            for (int l = 0; l < NL; l++)
#pragma unroll
                for (int m = 0; m < P; m++) store_stream(out + dst.off[m] + wl[l] * dst.stride[m], v[l][m]);
        } else if (count > 0) {
            const bool nt = STREAM && (a.flags & SF_STORE_NT) != 0;
#pragma unroll
            for (int l = 0; l < NL; l += VEC)
#pragma unroll
                for (int m = 0; m < P; m++) {
                    if constexpr (VEC == 2) {
                        T4 q;
                        q.x = v[l][m].x;
                        q.y = v[l][m].y;
                        q.z = v[l + 1][m].x;
                        q.w = v[l + 1][m].y;
                        T4 *p4 = (T4 *)(out + at(dst, lo, wl, l, m));
                        if (nt)
                            store_stream(p4, q);
                        else
                            *p4 = q;
                    } else {
                        T2 *p2 = out + at(dst, lo, wl, l, m);
                        if (nt)
                            store_stream(p2, v[l][m]);
                        else
                            *p2 = v[l][m];
                    }
                }
        } else {
            const int cnt = -count;
#pragma unroll
            for (int l = 0; l < NL; l++) {
                const bool ok = wl[l] < cnt;
#pragma unroll
                for (int m = 0; m < P; m++)
                    if (ok) out[at(dst, lo, wl, l, m)] = v[l][m];
            }
        }
    }
};

// Occupancy target of a tile shape: two workgroups per CU when their LDS fits
// (which caps VGPRs at 128 for 512-thread workgroups); the 64-bit-offset
// kernels of the largest plans leave the compiler their extra registers.
template <class S, typename Off = int>
constexpr int c2c_waves_per_eu()
{
    return (S::NT == 512 && (S::H > 1 || S::HS > 1) && sizeof(Off) == 4) ? 4 : 1;
}

// Twiddle table of the stage staged in LDS once per workgroup (the passes
// then read twiddles with LDS instead of vector-memory instructions).
#ifndef PFFT_TWIDDLES_IN_LDS
#define PFFT_TWIDDLES_IN_LDS 1
#endif
template <typename T2, int N>
struct TwiddleStage {
    static constexpr bool on = PFFT_TWIDDLES_IN_LDS && fft_npasses(N) > 1 && N * sizeof(T2) <= 8192;
    static constexpr int SIZE = on ? N : 1;
    __device__ static __forceinline__ const T2 *stage(T2 *buf, const void *tw)
    {
        if constexpr (on) {
            const T2 *g = (const T2 *)tw;
            for (int i = threadIdx.x; i < N; i += blockDim.x) buf[i] = g[i];
            __syncthreads();
            return buf;
        } else {
            (void)buf;
            return (const T2 *)tw;
        }
    }
};

// `tiles` is a.tiles passed as a restrict-qualified argument: tile records
// are then known to be unchanged by the kernel's stores and can be read
// through the scalar cache.
template <typename T, int N, bool CONTIG, int SIGN, class S, bool XS = false, typename Off = int>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(c2c_waves_per_eu<S, Off>()))) void k_c2c(
    StageArgs a, const Tile *__restrict__ tiles)
{
    using Wk = C2CWorker<T, N, CONTIG, SIGN, S, true, XS, Off>;
    using T2 = typename Wk::T2;
    constexpr int NL = S::NL, P = S::P;
    __shared__ T2 lds[Wk::LDS_SIZE];
    __shared__ T2 twl[TwiddleStage<T2, N>::SIZE];
    // SF_LATE_TWIDDLES: the twiddle table is staged while the first tile's
    // loads are in flight (single-precision contiguous stages measured faster
    // staging it first in every case)
    constexpr bool late_ok = !CONTIG || sizeof(T) == 8;
    const bool late_tw = late_ok && (a.flags & SF_LATE_TWIDDLES);
    const T2 *tw = late_tw ? nullptr : TwiddleStage<T2, N>::stage(twl, a.twiddle);
    Wk wk;
    wk.init_geometry();
    const long G = gridDim.x, nt = a.ntiles;
    T2 v[NL][P];
    SideAddr<P, Off> d;
    int c;
    // SF_XCD_ORDER with one tile per workgroup: workgroup b runs on XCD
    // b % 8, which takes the contiguous range x*q + min(x, r) + [0, q + (x < r))
    // of the nt = 8q + r tiles (a bijection of the tile indices)
    const bool xcd = !CONTIG && (a.flags & SF_XCD_ORDER) && G == nt;
    for (long ti0 = blockIdx.x; ti0 < nt; ti0 += G) {
        long ti = ti0;
        if (xcd) {
            const long q = nt / 8, r = nt % 8, x = ti0 % 8, k = ti0 / 8;
            ti = x * q + (x < r ? x : r) + k;
        }
        wk.refresh();
        // (contiguous stages measured faster with the tile read through the
        // vector path)
        const Tile &t = CONTIG ? a.tiles[ti] : tiles[ti];
        wk.load(a, t, v, d, c);
        if (late_tw && ti0 == blockIdx.x) tw = TwiddleStage<T2, N>::stage(twl, a.twiddle);
        wk.process(a, t, v, d, c, lds, tw);
    }
}

// The same stage for tiles of several transforms in one launch: each tile
// carries the index of its transform's arguments in bits 8..31 of its flags.
// Every transform of one launch has lines of N points in one precision, so
// they share one twiddle table (e^{-2 pi i m / N}), staged from the first
// transform's copy.
template <typename T, int N, bool CONTIG, int SIGN, class S>
__global__ __launch_bounds__(S::NT) __attribute__((amdgpu_waves_per_eu(c2c_waves_per_eu<S>()))) void k_c2c_multi(
    const StageArgs *__restrict__ args, const Tile *__restrict__ tiles, long nt)
{
    using Wk = C2CWorker<T, N, CONTIG, SIGN, S, false>;
    using T2 = typename Wk::T2;
    constexpr int NL = S::NL, P = S::P;
    __shared__ T2 lds[Wk::LDS_SIZE];
    __shared__ T2 twl[TwiddleStage<T2, N>::SIZE];
    const T2 *tw = TwiddleStage<T2, N>::stage(twl, args[0].twiddle);
    Wk wk;
    wk.init_geometry();
    const long G = gridDim.x;
    T2 v[NL][P];
    SideAddr<P> d;
    int c;
    for (long ti = blockIdx.x; ti < nt; ti += G) {
        const Tile &t = tiles[ti];
        const StageArgs &a = args[(unsigned)t.flags >> 8];
        wk.refresh();
        wk.load(a, t, v, d, c);
        wk.process(a, t, v, d, c, lds, tw);
    }
}

}  // namespace pfft
