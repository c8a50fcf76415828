// k_r2r.hpp -- real-to-real partial transforms: the cosine and sine
// transforms of type II and their inverses of type III, along any axis of a
// layout, with the same gather/scatter addressing as the complex stages (so a
// redistribution is fused into the load or the store as for the FFT).  The
// method carries such "similar" transforms unchanged (Sec. 1 and the
// conclusions); the definitions, unnormalised:
//   type II cosine:  Y_k = 2 sum_j x_j cos(pi (2j+1) k / 2N)
//   type III cosine: Y_k = x_0 + 2 sum_{j>=1} x_j cos(pi j (2k+1) / 2N)
//   type II sine:    Y_k = 2 sum_j x_j sin(pi (2j+1) (k+1) / 2N)
//   type III sine:   Y_k = (-1)^k x_{N-1} + 2 sum_{j<N-1} x_j sin(pi (j+1) (2k+1) / 2N)
//
// Each line goes through one complex FFT (Makhoul's reordering):
//   type II:  v_n = x_{p(n)} with p(n) = 2n for n < ceil(N/2), 2(N-1-n)+1
//             after; V = FFT_N(v); Y_k = 2 Re(e^{-i pi k/2N} V_k).
//   type III: V_k = e^{+i pi k/2N} (X_k - i X_{N-k}) / 2 (X_N = 0);
//             v = unnormalised inverse FFT_N of V; y_{p(n)} = 2 Re v_n.
//   sine:     type II of x_j (-1)^j, output reversed; type III of the
//             reversed input, output times (-1)^k.
// For even N >= 4 the real sequence v is packed as z_n = v_{2n} + i v_{2n+1}
// and transformed at half length M = N/2, with the usual pairing of bins k
// and M-k (as in the real-to-complex stage):
//   V_k = (Z_k + conj Z_{M-k})/2 - (i/2) e^{-2 pi i k/N} (Z_k - conj Z_{M-k}),
//   Y_k = 2 Re(w_k V_k), Y_{N-k} = -2 Im(w_k V_k), w_k = e^{-i pi k/2N};
// and backwards Z'_k = (V_k + conj V_{M-k}) + i e^{2 pi i k/N} (V_k - conj V_{M-k}),
// whose unnormalised inverse FFT_M is v_{2n} + i v_{2n+1}.
// The lines of a tile are staged as real values in LDS twice (reordering in,
// reordering out), so global accesses stay in natural order.
#pragma once

#include <type_traits>

#include "fft_device.hpp"
#include "k_c2c_impl.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

// Launch shape: the tile width of the complex stage's variant V (one LDS
// portion), at most 512 threads.  (Two LDS portions measured slower here and
// round differently: the compiler contracts multiply-adds differently in that
// instantiation.)
template <typename T, int N, bool CONTIG, int V>
struct R2RCfg {
    using D = C2CDefault<T, N, CONTIG>;
    using B = C2CVariant<T, N, CONTIG, V>;
    static constexpr int P = fft_points(N);
    static constexpr int TPL = N / P;
    static constexpr int H = 1;
    static constexpr int W = (B::exists && B::H == 1) ? B::W : D::W;
    static constexpr int WL = W;
    static constexpr int nl_for(int nl) { return (TPL * W / nl > 512 && nl < W) ? nl_for(nl * 2) : nl; }
    static constexpr int NL = nl_for(1);
    static constexpr int SLOTS = W / NL;
    static constexpr int NT = TPL * SLOTS;
};

// Row pieces of a strided real tile (N rows of W adjacent lines): Q reals
// (16 bytes) per piece, CPR pieces per row; thread `tid` moves piece
// tid % CPR of rows tid / CPR + i * TPR, i < RPT.  Used for full tiles whose
// line 0 starts at a multiple of Q elements at every row on both sides (tile
// flag FLAG: bit 1 for 4-byte reals, bit 0 for 8-byte reals).
template <typename T, int N, int W, int NT, bool CONTIG>
struct R2RRows {
    static constexpr int Q = 16 / (int)sizeof(T);
    static constexpr int CPR = W / Q > 0 ? W / Q : 1;
    static constexpr int TPR = NT / CPR > 0 ? NT / CPR : 1;
    static constexpr int RPT = N / TPR > 0 ? N / TPR : 1;
    static constexpr bool on = !CONTIG && W % Q == 0 && NT % CPR == 0 && N % TPR == 0 && RPT <= 32;
    static constexpr int FLAG = sizeof(T) == 4 ? 2 : 1;
    using V = typename V2<T>::type;  // replaced below for 4-byte reals
    __device__ static __forceinline__ T get(const V &v, int e) { return e == 0 ? v.x : v.y; }
    __device__ static __forceinline__ void set(V &v, int e, T x) { (e == 0 ? v.x : v.y) = x; }
    __device__ static __forceinline__ V load_nt(const V *p) { return load_stream(p); }
    __device__ static __forceinline__ void store_nt(V *p, V v) { store_stream(p, v); }
};
template <int N, int W, int NT, bool CONTIG>
struct R2RRows<float, N, W, NT, CONTIG> {
    static constexpr int Q = 4;
    static constexpr int CPR = W / Q > 0 ? W / Q : 1;
    static constexpr int TPR = NT / CPR > 0 ? NT / CPR : 1;
    static constexpr int RPT = N / TPR > 0 ? N / TPR : 1;
    static constexpr bool on = !CONTIG && W % Q == 0 && NT % CPR == 0 && N % TPR == 0 && RPT <= 32;
    static constexpr int FLAG = 2;
    using V = float4;
    __device__ static __forceinline__ float get(const V &v, int e)
    {
        return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
    }
    __device__ static __forceinline__ void set(V &v, int e, float x)
    {
        if (e == 0) v.x = x;
        else if (e == 1) v.y = x;
        else if (e == 2) v.z = x;
        else v.w = x;
    }
    typedef float f4 __attribute__((ext_vector_type(4)));
    __device__ static __forceinline__ V load_nt(const V *p)
    {
        const f4 t = __builtin_nontemporal_load((const f4 *)p);
        V v;
        v.x = t.x;
        v.y = t.y;
        v.z = t.z;
        v.w = t.w;
        return v;
    }
    __device__ static __forceinline__ void store_nt(V *p, V v)
    {
        const f4 t = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(t, (f4 *)p);
    }
};

// Line pieces of a contiguous real tile (W lines of N adjacent reals): Q
// reals (16 bytes) per piece, CPL pieces per line; thread `tid` moves piece
// tid % CPL of lines tid / CPL + i * LG, i < LPT.  Used for full tiles whose
// aligned groups of Q positions are adjacent and start at a multiple of Q
// elements in every line on both sides (tile flag FLAG).
template <typename T, int N, int W, int NT, bool CONTIG>
struct R2RLines {
    using RW = R2RRows<T, N, W, NT, false>;  // piece type and accessors
    using V = typename RW::V;
    static constexpr int Q = RW::Q;
    static constexpr int CPL = N / Q > 0 ? N / Q : 1;
    static constexpr int LG = NT / CPL > 0 ? NT / CPL : 1;
    static constexpr int LPT = W / LG > 0 ? W / LG : 1;
    static constexpr bool on = CONTIG && N % Q == 0 && CPL <= NT && NT % CPL == 0 && W % LG == 0 && LPT <= 32;
    static constexpr int FLAG = RW::FLAG;
};

// Tile of workgroup b when the device hands workgroups to its 8 XCDs in turn
// (b to XCD b % 8): each XCD takes one contiguous range of tiles, in order, so
// neighbouring tiles that share cache lines meet in the same L2.  (A bijection
// of 0..n-1 for any n, so only the traffic depends on the dispatch order.)
// Strided real tiles of 16 lines have 64-byte rows: two tiles share every
// 128-byte line, which round-robin order fetched twice from two L2s.
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    constexpr int X = 8;
    const int q = n / X, r = n % X, x = b % X, k = b / X;
    return x * q + (x < r ? x : r) + k;
}

template <typename T, int N, bool CONTIG, class S>
__global__ __launch_bounds__(S::NT) void k_r2r(StageArgs a, const Tile *__restrict__ tiles)
{
    using T2 = typename V2<T>::type;
    constexpr int P = S::P, TPL = S::TPL, NL = S::NL, W = S::W, SLOTS = S::SLOTS;
    constexpr int H = S::H, WL = S::WL;
    using LT = LdsTile<T2, N, WL, CONTIG>;
    constexpr int RLINE = N + 1, RROW = W + 1;  // real staging (aliases the exchange LDS)
    constexpr int STAGE = CONTIG ? W * RLINE : N * RROW;
    constexpr int LDS_N = LT::SIZE > (STAGE + 1) / 2 ? LT::SIZE : (STAGE + 1) / 2;
    constexpr bool TQL = N * sizeof(T2) <= 8192;  // quarter-wave twiddles staged in LDS when small
    __shared__ T2 lds[LDS_N];
    __shared__ T2 twl[TwiddleStage<T2, N>::SIZE];
    __shared__ T2 tql[TQL ? N : 1];
    if constexpr (TQL)
        for (int i = threadIdx.x; i < N; i += blockDim.x) tql[i] = ((const T2 *)a.twiddle2)[i];
    const T2 *tw = TwiddleStage<T2, N>::stage(twl, a.twiddle);  // tql is first read after the barrier below
    T *rl = (T *)lds;
    auto ridx = [](int w, int j) { return CONTIG ? w * RLINE + j : j * RROW + w; };

    const int tid = threadIdx.x;
    const int jt = CONTIG ? tid % TPL : tid / SLOTS;
    const int slot = CONTIG ? tid / TPL : tid % SLOTS;
    int wl[NL];
#pragma unroll
    for (int l = 0; l < NL; l++) wl[l] = slot + l * SLOTS;
    const Tile &t = tiles[blockIdx.x];
    const int count = t.count;
    const bool inverse = (a.flags & SF_R2R_INVERSE) != 0;
    const bool sine = (a.flags & SF_R2R_SINE) != 0;
    const bool adj = (a.flags & SF_R2R_ADJOINT) != 0;
    const int special = sine ? N - 1 : 0;  // the element types II and III weigh differently
    constexpr int h = (N + 1) / 2;

    // 1. the tile's lines, natural order, into LDS (all loads first)
    SideAddr<P> src;
    src.init(a.side[0], t, 0, jt, TPL, N, CONTIG);
    const T *__restrict__ in = (const T *)a.src;
    T xr[NL][P];
    if (count == W) {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) xr[l][m] = in[src.off[m] + wl[l] * src.stride[m]];
    } else {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) xr[l][m] = wl[l] < count ? in[src.off[m] + wl[l] * src.stride[m]] : (T)0;
    }
#pragma unroll
    for (int l = 0; l < NL; l++)
#pragma unroll
        for (int m = 0; m < P; m++) rl[ridx(wl[l], jt + m * TPL)] = xr[l][m];
    __syncthreads();

    // 2. the complex FFT input, point k = jt + m*TPL of each line
    const T2 *tq = TQL ? (const T2 *)tql : (const T2 *)a.twiddle2;  // e^{-i pi k / 2N}
    T2 v[NL][P];
#pragma unroll
    for (int l = 0; l < NL; l++)
#pragma unroll
        for (int m = 0; m < P; m++) {
            const int k = jt + m * TPL;
            if (!inverse) {
                const int p = k < h ? 2 * k : 2 * (N - 1 - k) + 1;
                T x = rl[ridx(wl[l], p)];
                if (sine && (p & 1)) x = -x;
                v[l][m].x = x;
                v[l][m].y = (T)0;
            } else {
                const int jk = sine ? N - 1 - k : k;
                const int jn = sine ? k - 1 : N - k;
                T xk = rl[ridx(wl[l], jk)];
                T xn = k == 0 ? (T)0 : rl[ridx(wl[l], jn)];
                if (adj && jk == special) xk *= (T)2;
                if (adj && k > 0 && jn == special) xn *= (T)2;
                const T2 w = tq[k];
                // e^{+i pi k/2N} (xk - i xn) / 2, with the fused multiply-adds
                // spelled out (the same rounding in every launch shape)
                v[l][m].x = (T)0.5 * fma(w.x, xk, -(w.y * xn));
                v[l][m].y = (T)-0.5 * fma(w.x, xn, w.y * xk);
            }
        }
    __syncthreads();

    // 3. the N-point transform (forward for type II, inverse for type III)
    if (inverse)
        fft_passes<T2, N, WL, CONTIG, 1, NL, H, 0>(v, wl, jt, lds, tw);
    else
        fft_passes<T2, N, WL, CONTIG, -1, NL, H, 0>(v, wl, jt, lds, tw);
    __syncthreads();

    // 4. outputs reordered through LDS, then stored in natural order
    const T scale = (T)a.scale;
#pragma unroll
    for (int l = 0; l < NL; l++)
#pragma unroll
        for (int m = 0; m < P; m++) {
            const int k = jt + m * TPL;
            if (!inverse) {
                const T2 w = tq[k];
                T y = (T)2 * fma(w.x, v[l][m].x, -(w.y * v[l][m].y)) * scale;
                const int q = sine ? N - 1 - k : k;
                if (adj && q == special) y *= (T)0.5;
                rl[ridx(wl[l], q)] = y;
            } else {
                const int q = k < h ? 2 * k : 2 * (N - 1 - k) + 1;
                T y = (T)2 * v[l][m].x * scale;
                if (sine && (q & 1)) y = -y;
                rl[ridx(wl[l], q)] = y;
            }
        }
    __syncthreads();
    SideAddr<P> dst;
    dst.init(a.side[1], t, 1, jt, TPL, N, CONTIG);
    T *__restrict__ out = (T *)a.dst;
#pragma unroll
    for (int l = 0; l < NL; l++)
#pragma unroll
        for (int m = 0; m < P; m++)
            if (wl[l] < count) out[dst.off[m] + wl[l] * dst.stride[m]] = rl[ridx(wl[l], jt + m * TPL)];
}

// Half-length stage of N = 2M points: S is the launch shape of the M-point
// transform; each thread also loads and stores 2P of the line's N reals.
template <typename T, int M, bool CONTIG, class S>
__global__ __launch_bounds__(S::NT) void k_r2r_half(StageArgs a, const Tile *__restrict__ tiles)
{
    using T2 = typename V2<T>::type;
    constexpr int N = 2 * M;
    constexpr int P = S::P, TPL = S::TPL, NL = S::NL, W = S::W, SLOTS = S::SLOTS;
    using LT = LdsTile<T2, M, W, CONTIG>;
    constexpr int RLINE = N + 1, RROW = W + 1;  // real staging (aliases the exchange LDS)
    constexpr int STAGE = CONTIG ? W * RLINE : N * RROW;
    constexpr int LDS_N = LT::SIZE > (STAGE + 1) / 2 ? LT::SIZE : (STAGE + 1) / 2;
    // The M-point twiddles and the post table are staged in LDS when small;
    // on contiguous tiles only when that costs no workgroup per CU (160 KB of
    // LDS per CU), since those stages gain more from tiles in flight (strided
    // stages measured the other way round).
    constexpr int LDS_CU = 160 * 1024;
    constexpr int B_BASE = LDS_N * (int)sizeof(T2);
    constexpr int B_TW = M * (int)sizeof(T2), B_PT = 2 * (M + 1) * (int)sizeof(T2);
    constexpr bool TWL = TwiddleStage<T2, M>::on && (!CONTIG || LDS_CU / (B_BASE + B_TW) == LDS_CU / B_BASE);
    constexpr int B_T = B_BASE + (TWL ? B_TW : 0);
    constexpr bool PT = B_PT <= 8192 && (!CONTIG || LDS_CU / (B_T + B_PT) == LDS_CU / B_T);
    __shared__ T2 lds[LDS_N];
    __shared__ T2 twl[TWL ? M : 1];
    __shared__ T2 ptl[PT ? 2 * (M + 1) : 1];
    // (both are first read after the barrier that ends step 1)
    if constexpr (TWL)
        for (int i = threadIdx.x; i < M; i += blockDim.x) twl[i] = ((const T2 *)a.twiddle)[i];
    if constexpr (PT)
        for (int i = threadIdx.x; i < 2 * (M + 1); i += blockDim.x) ptl[i] = ((const T2 *)a.twiddle2)[i];
    const T2 *tw = TWL ? (const T2 *)twl : (const T2 *)a.twiddle;
    const T2 *te = PT ? (const T2 *)ptl : (const T2 *)a.twiddle2;  // e^{-2 pi i k/N}, k <= M
    const T2 *tq = te + (M + 1);                                     // e^{-i pi k/2N}, k <= M
    T *rl = (T *)lds;
    auto ridx = [](int w, int j) { return CONTIG ? w * RLINE + j : j * RROW + w; };

    const int tid = threadIdx.x;
    const int jt = CONTIG ? tid % TPL : tid / SLOTS;
    const int slot = CONTIG ? tid / TPL : tid % SLOTS;
    int wl[NL];
#pragma unroll
    for (int l = 0; l < NL; l++) wl[l] = slot + l * SLOTS;
    const Tile &t = tiles[CONTIG ? (int)blockIdx.x : xcd_tile(blockIdx.x, (int)a.ntiles)];
    const int count = t.count;
    const bool inverse = (a.flags & SF_R2R_INVERSE) != 0;
    const bool sine = (a.flags & SF_R2R_SINE) != 0;
    const bool adj = (a.flags & SF_R2R_ADJOINT) != 0;
    const int special = sine ? N - 1 : 0;
    constexpr int h = M;  // ceil(N/2)

    // 1. the tile's lines, natural order, into LDS (all loads first); the
    // adjoint of type II doubles the special input element of type III
    const T *__restrict__ in = (const T *)a.src;
    const bool dbl = adj && inverse;
    using RW = R2RRows<T, N, W, S::NT, CONTIG>;
    using RC = R2RLines<T, N, W, S::NT, CONTIG>;
    const bool wide = RW::on && count == W && (t.flags & RW::FLAG);
    const bool wide_c = RC::on && count == W && (t.flags & RC::FLAG);
    if (wide_c) {
        // contiguous tile, full and aligned: 16-byte pieces of each line
        const int q = tid % RC::CPL, r0 = tid / RC::CPL;
        SideAddr<1> ws;
        ws.init(a.side[0], t, 0, q * RC::Q, 1, N, true);
        typename RC::V xv[RC::LPT];
#pragma unroll
        for (int i = 0; i < RC::LPT; i++)  // each byte read once: streaming loads
            xv[i] = RW::load_nt((const typename RC::V *)(in + ws.off[0] + (r0 + i * RC::LG) * ws.stride[0]));
#pragma unroll
        for (int i = 0; i < RC::LPT; i++)
#pragma unroll
            for (int e = 0; e < RC::Q; e++) {
                const int j = q * RC::Q + e;
                const T x = RW::get(xv[i], e);
                rl[ridx(r0 + i * RC::LG, j)] = (dbl && j == special) ? (T)2 * x : x;
            }
    } else if (wide) {
        // strided tile, full and aligned: rows of W reals in 16-byte pieces
        // (any thread may move any piece: the staging decouples the loads
        // from the transform's point ownership)
        const int q = tid % RW::CPR, r0 = tid / RW::CPR;
        SideAddr<RW::RPT> ws;
        ws.init(a.side[0], t, 0, r0, RW::TPR, N, false);
        typename RW::V xv[RW::RPT];
#pragma unroll
        for (int i = 0; i < RW::RPT; i++) xv[i] = *(const typename RW::V *)(in + ws.off[i] + q * RW::Q);
#pragma unroll
        for (int i = 0; i < RW::RPT; i++) {
            const int j = r0 + i * RW::TPR;
#pragma unroll
            for (int e = 0; e < RW::Q; e++) {
                const T x = RW::get(xv[i], e);
                rl[ridx(q * RW::Q + e, j)] = (dbl && j == special) ? (T)2 * x : x;
            }
        }
    } else {
        SideAddr<2 * P> src;
        src.init(a.side[0], t, 0, jt, TPL, N, CONTIG);
        T xr[NL][2 * P];
        if (count == W) {
#pragma unroll
            for (int l = 0; l < NL; l++)
#pragma unroll
                for (int m = 0; m < 2 * P; m++) xr[l][m] = in[src.off[m] + wl[l] * src.stride[m]];
        } else {
#pragma unroll
            for (int l = 0; l < NL; l++)
#pragma unroll
                for (int m = 0; m < 2 * P; m++)
                    xr[l][m] = wl[l] < count ? in[src.off[m] + wl[l] * src.stride[m]] : (T)0;
        }
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < 2 * P; m++) {
                const int j = jt + m * TPL;
                rl[ridx(wl[l], j)] = (dbl && j == special) ? (T)2 * xr[l][m] : xr[l][m];
            }
    }
    __syncthreads();

    // 2. the M-point input, point k = jt + m*TPL of each line
    T2 v[NL][P];
    if (!inverse) {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int n = jt + m * TPL;
                const int p0 = 2 * n < h ? 4 * n : 2 * (N - 1 - 2 * n) + 1;
                const int p1 = 2 * n + 1 < h ? 4 * n + 2 : 2 * (N - 2 - 2 * n) + 1;
                T x0 = rl[ridx(wl[l], p0)], x1 = rl[ridx(wl[l], p1)];
                if (sine && (p0 & 1)) x0 = -x0;
                if (sine && (p1 & 1)) x1 = -x1;
                v[l][m].x = x0;
                v[l][m].y = x1;
            }
    } else {
        // X in the type III input order (the sine transform reads it reversed)
        auto X = [&](int w, int j) { return rl[ridx(w, sine ? N - 1 - j : j)]; };
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int k = jt + m * TPL;
                const int kc = M - k;  // 1..M
                // V_k = e^{+i pi k/2N} (X_k - i X_{N-k}) / 2 and the same at M-k
                const T xk = X(wl[l], k), xnk = k == 0 ? (T)0 : X(wl[l], N - k);
                const T xc = X(wl[l], kc), xnc = X(wl[l], N - kc);
                const T2 qk = tq[k], qc = tq[kc];
                T2 vk, vc;
                vk.x = (T)0.5 * fma(qk.x, xk, -(qk.y * xnk));
                vk.y = (T)-0.5 * fma(qk.x, xnk, qk.y * xk);
                vc.x = (T)0.5 * fma(qc.x, xc, -(qc.y * xnc));
                vc.y = (T)-0.5 * fma(qc.x, xnc, qc.y * xc);
                // Z'_k = (V_k + conj V_c) + i e^{+2 pi i k/N} (V_k - conj V_c)
                const T2 s = {vk.x + vc.x, vk.y - vc.y};
                const T2 d = {vk.x - vc.x, vk.y + vc.y};
                const T2 e = te[k];  // e^{-2 pi i k/N}; its conjugate here
                const T2 ed = {fma(e.x, d.x, e.y * d.y), fma(e.x, d.y, -(e.y * d.x))};
                v[l][m].x = s.x - ed.y;
                v[l][m].y = s.y + ed.x;
            }
    }
    __syncthreads();

    // 3. the M-point transform
    if (inverse)
        fft_passes<T2, M, W, CONTIG, 1, NL, 1, 0>(v, wl, jt, lds, tw);
    else
        fft_passes<T2, M, W, CONTIG, -1, NL, 1, 0>(v, wl, jt, lds, tw);
    __syncthreads();

    // 4. outputs into registers (type II pairs bins k and M-k through LDS)
    const T scale = (T)a.scale;
    T yr[NL][2 * P];
    int yq[2 * P];  // output position of yr[.][m] (the same for every line)
    if (!inverse) {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) lds[LT::idx(wl[l], jt + m * TPL)] = v[l][m];
        __syncthreads();
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int k = jt + m * TPL;
                const T2 zk = v[l][m];
                T2 zc = lds[LT::idx(wl[l], k == 0 ? 0 : M - k)];
                zc.y = -zc.y;
                // X_k = (Z_k + conj Z_c)/2 - (i/2) e^{-2 pi i k/N} (Z_k - conj Z_c)
                const T2 sm = {(T)0.5 * (zk.x + zc.x), (T)0.5 * (zk.y + zc.y)};
                const T2 df = {(T)0.5 * (zk.x - zc.x), (T)0.5 * (zk.y - zc.y)};
                const T2 e = te[k];
                const T2 ed = {fma(e.x, df.x, -(e.y * df.y)), fma(e.x, df.y, e.y * df.x)};
                const T2 xk = {sm.x + ed.y, sm.y - ed.x};
                const T2 q = tq[k];
                const T2 wx = {fma(q.x, xk.x, -(q.y * xk.y)), fma(q.x, xk.y, q.y * xk.x)};
                // Y_k = 2 Re(w_k X_k); Y_{N-k} = -2 Im(w_k X_k) (k > 0); bin M from Z_0 (k = 0)
                T y0 = (T)2 * wx.x * scale;
                T y1;
                int q1;
                if (k == 0) {
                    const T xm = zk.x - zk.y;  // X_M (real)
                    y1 = (T)2 * tq[M].x * xm * scale;
                    q1 = M;
                } else {
                    y1 = (T)-2 * wx.y * scale;
                    q1 = N - k;
                }
                int q0 = k;
                if (sine) {
                    q0 = N - 1 - q0;
                    q1 = N - 1 - q1;
                }
                if (adj && q0 == special) y0 *= (T)0.5;
                if (adj && q1 == special) y1 *= (T)0.5;
                yr[l][2 * m] = y0;
                yr[l][2 * m + 1] = y1;
                if (l == 0) {
                    yq[2 * m] = q0;
                    yq[2 * m + 1] = q1;
                }
            }
    } else {
#pragma unroll
        for (int m = 0; m < P; m++) {
            const int n = jt + m * TPL;
            yq[2 * m] = 2 * n < h ? 4 * n : 2 * (N - 1 - 2 * n) + 1;
            yq[2 * m + 1] = 2 * n + 1 < h ? 4 * n + 2 : 2 * (N - 2 - 2 * n) + 1;
        }
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                T y0 = (T)2 * v[l][m].x * scale, y1 = (T)2 * v[l][m].y * scale;
                if (sine && (yq[2 * m] & 1)) y0 = -y0;
                if (sine && (yq[2 * m + 1] & 1)) y1 = -y1;
                yr[l][2 * m] = y0;
                yr[l][2 * m + 1] = y1;
            }
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < NL; l++)
#pragma unroll
        for (int m = 0; m < 2 * P; m++) rl[ridx(wl[l], yq[m])] = yr[l][m];
    __syncthreads();

    // 5. natural-order stores
    T *__restrict__ out = (T *)a.dst;
    if (wide_c) {
        const int q = tid % RC::CPL, r0 = tid / RC::CPL;
        SideAddr<1> wd;
        wd.init(a.side[1], t, 1, q * RC::Q, 1, N, true);
#pragma unroll
        for (int i = 0; i < RC::LPT; i++) {
            typename RC::V y;
#pragma unroll
            for (int e = 0; e < RC::Q; e++) RW::set(y, e, rl[ridx(r0 + i * RC::LG, q * RC::Q + e)]);
            typename RC::V *o = (typename RC::V *)(out + wd.off[0] + (r0 + i * RC::LG) * wd.stride[0]);
            if (a.side[1].R == 0)
                RW::store_nt(o, y);  // whole destination lines: streaming stores
            else
                *o = y;
        }
        return;
    }
    if (wide) {
        const int q = tid % RW::CPR, r0 = tid / RW::CPR;
        SideAddr<RW::RPT> wd;
        wd.init(a.side[1], t, 1, r0, RW::TPR, N, false);
#pragma unroll
        for (int i = 0; i < RW::RPT; i++) {
            typename RW::V y;
#pragma unroll
            for (int e = 0; e < RW::Q; e++) RW::set(y, e, rl[ridx(q * RW::Q + e, r0 + i * RW::TPR)]);
            *(typename RW::V *)(out + wd.off[i] + q * RW::Q) = y;
        }
        return;
    }
    SideAddr<2 * P> dst;
    dst.init(a.side[1], t, 1, jt, TPL, N, CONTIG);
#pragma unroll
    for (int l = 0; l < NL; l++)
#pragma unroll
        for (int m = 0; m < 2 * P; m++)
            if (wl[l] < count) out[dst.off[m] + wl[l] * dst.stride[m]] = rl[ridx(wl[l], jt + m * TPL)];
}

// Strided half-length stage with the reordering folded into the row
// addresses: each thread owns RV adjacent lines (one 16-byte piece of every
// row it touches), loads the rows its points need directly, keeps the lines in
// registers through the M-point transform and stores its output rows
// directly; the LDS serves only the transform's exchanges and the pairing of
// bins k and M-k (no staging of the lines).  SL groups of RV lines per tile.
template <typename T, int M, int SL>
struct R2RRowsCfg {
    using T2 = typename V2<T>::type;
    static constexpr int RV = 16 / (int)sizeof(T);
    static constexpr int P = fft_points(M);
    static constexpr int TPL = M / P;
    static constexpr int NL = RV;
    static constexpr int W = SL * RV;
    static constexpr int NT = TPL * SL;
    using LT = LdsTile<T2, M, W, false>;
    static constexpr bool exists = P <= 12 && NT >= 64 && NT <= 1024 && LT::SIZE * (int)sizeof(T2) <= 150 * 1024;
};

// Element e of a 16-byte row piece (four floats or two doubles).
__device__ __forceinline__ float piece_get(const float4 &q, int e)
{
    return e == 0 ? q.x : e == 1 ? q.y : e == 2 ? q.z : q.w;
}
__device__ __forceinline__ double piece_get(const double2 &q, int e) { return e == 0 ? q.x : q.y; }

template <typename T, int M, int SL, bool INV>
__global__ __launch_bounds__((R2RRowsCfg<T, M, SL>::NT)) void k_r2r_rows(StageArgs a, const Tile *__restrict__ tiles)
{
    using C = R2RRowsCfg<T, M, SL>;
    using T2 = typename C::T2;
    using LT = typename C::LT;
    using RVec = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    constexpr int N = 2 * M, P = C::P, TPL = C::TPL, NL = C::NL, RV = C::RV, W = C::W;
    constexpr int FLAG = sizeof(T) == 4 ? 2 : 1;  // rows 16-byte aligned on both sides
    constexpr bool PT = 2 * (M + 1) * (int)sizeof(T2) <= 8192;
    __shared__ T2 lds[LT::SIZE];
    __shared__ T2 twl[TwiddleStage<T2, M>::SIZE];
    __shared__ T2 ptl[PT ? 2 * (M + 1) : 1];
    if constexpr (PT)
        for (int i = threadIdx.x; i < 2 * (M + 1); i += blockDim.x) ptl[i] = ((const T2 *)a.twiddle2)[i];
    const T2 *tw = TwiddleStage<T2, M>::stage(twl, a.twiddle);
    if constexpr (PT) __syncthreads();
    const T2 *te = PT ? (const T2 *)ptl : (const T2 *)a.twiddle2;  // e^{-2 pi i k/N}, k <= M
    const T2 *tq = te + (M + 1);                                     // e^{-i pi k/2N}, k <= M

    const int tid = threadIdx.x;
    const int slot = tid % SL, jt = tid / SL;
    int wl[NL];
#pragma unroll
    for (int l = 0; l < NL; l++) wl[l] = slot * RV + l;
    const Tile &t = tiles[xcd_tile(blockIdx.x, (int)a.ntiles)];
    const int count = t.count;
    const bool vec = count == W && (t.flags & FLAG);
    constexpr bool inverse = INV;  // type III (the launch picks the kernel by SF_R2R_INVERSE)
    const bool sine = (a.flags & SF_R2R_SINE) != 0;
    const bool adj = (a.flags & SF_R2R_ADJOINT) != 0;
    const bool dbl = adj && inverse;
    const int special = sine ? N - 1 : 0;
    const T scale = (T)a.scale;
    const T *__restrict__ in = (const T *)a.src;
    T *__restrict__ out = (T *)a.dst;
    // type II order: element v_i of the reordered line is x_{p(i)}
    auto p_of = [](int i) { return i < M ? 2 * i : 2 * (N - 1 - i) + 1; };

    // 1. the rows the thread's points need, directly
    int pos[2 * P];
#pragma unroll
    for (int m = 0; m < P; m++) {
        const int k = jt + m * TPL;
        if constexpr (!inverse) {
            pos[2 * m] = p_of(2 * k);
            pos[2 * m + 1] = p_of(2 * k + 1);
        } else {
            // X_k and X_{N-k} (X_M for k = 0) in the type III input order
            const int j1 = k == 0 ? M : N - k;
            pos[2 * m] = sine ? N - 1 - k : k;
            pos[2 * m + 1] = sine ? N - 1 - j1 : j1;
        }
    }
    T x[2 * P][RV];
    {
        SideAddr<2 * P> src;
        src.init_pos(a.side[0], t, 0, pos, false);
        if (vec) {
#pragma unroll
            for (int i = 0; i < 2 * P; i++) {
                const RVec q = *(const RVec *)(in + src.off[i] + slot * RV);
#pragma unroll
                for (int e = 0; e < RV; e++) x[i][e] = piece_get(q, e);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 2 * P; i++)
#pragma unroll
                for (int e = 0; e < RV; e++) x[i][e] = wl[e] < count ? in[src.off[i] + wl[e]] : (T)0;
        }
    }

    // 2. the M-point input
    T2 v[NL][P];
    if constexpr (!inverse) {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                T x0 = x[2 * m][l], x1 = x[2 * m + 1][l];
                if (sine && (pos[2 * m] & 1)) x0 = -x0;
                if (sine && (pos[2 * m + 1] & 1)) x1 = -x1;
                v[l][m].x = x0;
                v[l][m].y = x1;
            }
    } else {
        // V_k = e^{+i pi k/2N} (X_k - i X_{N-k}) / 2 (the adjoint of type II
        // doubles X_0); V_{M-k} comes from the thread that owns M-k (V_M,
        // owned by nobody, from X_M by the thread of k = 0)
        T2 vm[NL];
#pragma unroll
        for (int l = 0; l < NL; l++) vm[l] = T2{(T)0, (T)0};
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int k = jt + m * TPL;
                T xk = x[2 * m][l];
                if (dbl && k == 0) xk *= (T)2;
                const T xnk = k == 0 ? (T)0 : x[2 * m + 1][l];
                const T2 qk = tq[k];
                v[l][m].x = (T)0.5 * fma(qk.x, xk, -(qk.y * xnk));
                v[l][m].y = (T)-0.5 * fma(qk.x, xnk, qk.y * xk);
                if (m == 0) {
                    const T xc = x[1][l];  // X_M where k = 0
                    const T2 qc = tq[M];
                    vm[l].x = (T)0.5 * fma(qc.x, xc, -(qc.y * xc));
                    vm[l].y = (T)-0.5 * fma(qc.x, xc, qc.y * xc);
                }
                lds[LT::idx(wl[l], k)] = v[l][m];
            }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int k = jt + m * TPL;
                const T2 vk = v[l][m];
                // (a value select: an LDS load for every k, V_M where k = 0)
                T2 vc = lds[LT::idx(wl[l], k == 0 ? M - 1 : M - k)];
                if (k == 0) vc = vm[l];
                // Z'_k = (V_k + conj V_c) + i e^{+2 pi i k/N} (V_k - conj V_c)
                const T2 sm = {vk.x + vc.x, vk.y - vc.y};
                const T2 d = {vk.x - vc.x, vk.y + vc.y};
                const T2 e = te[k];
                const T2 ed = {fma(e.x, d.x, e.y * d.y), fma(e.x, d.y, -(e.y * d.x))};
                v[l][m].x = sm.x - ed.y;
                v[l][m].y = sm.y + ed.x;
            }
        __syncthreads();
    }

    // 3. the M-point transform
    if constexpr (inverse)
        fft_passes<T2, M, W, false, 1, NL, 1, 0>(v, wl, jt, lds, tw);
    else
        fft_passes<T2, M, W, false, -1, NL, 1, 0>(v, wl, jt, lds, tw);
    __syncthreads();

    // 4. outputs (type II pairs bins k and M-k through LDS), by row
    if constexpr (!inverse) {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) lds[LT::idx(wl[l], jt + m * TPL)] = v[l][m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < P; m++) {
            const int k = jt + m * TPL;
            int q0 = k, q1 = k == 0 ? M : N - k;
            if (sine) {
                q0 = N - 1 - q0;
                q1 = N - 1 - q1;
            }
            pos[2 * m] = q0;
            pos[2 * m + 1] = q1;
        }
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int k = jt + m * TPL;
                const T2 zk = v[l][m];
                T2 zc = lds[LT::idx(wl[l], k == 0 ? 0 : M - k)];
                zc.y = -zc.y;
                // X_k = (Z_k + conj Z_c)/2 - (i/2) e^{-2 pi i k/N} (Z_k - conj Z_c)
                const T2 sm = {(T)0.5 * (zk.x + zc.x), (T)0.5 * (zk.y + zc.y)};
                const T2 df = {(T)0.5 * (zk.x - zc.x), (T)0.5 * (zk.y - zc.y)};
                const T2 e = te[k];
                const T2 ed = {fma(e.x, df.x, -(e.y * df.y)), fma(e.x, df.y, e.y * df.x)};
                const T2 xk = {sm.x + ed.y, sm.y - ed.x};
                const T2 q = tq[k];
                const T2 wx = {fma(q.x, xk.x, -(q.y * xk.y)), fma(q.x, xk.y, q.y * xk.x)};
                // Y_k = 2 Re(w_k X_k); Y_{N-k} = -2 Im(w_k X_k) (k > 0); bin M from Z_0 (k = 0)
                T y0 = (T)2 * wx.x * scale;
                T y1 = k == 0 ? (T)2 * tq[M].x * (zk.x - zk.y) * scale : (T)-2 * wx.y * scale;
                if (adj && pos[2 * m] == special) y0 *= (T)0.5;
                if (adj && pos[2 * m + 1] == special) y1 *= (T)0.5;
                x[2 * m][l] = y0;
                x[2 * m + 1][l] = y1;
            }
    } else {
#pragma unroll
        for (int m = 0; m < P; m++) {
            const int n = jt + m * TPL;
            pos[2 * m] = p_of(2 * n);
            pos[2 * m + 1] = p_of(2 * n + 1);
        }
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) {
                T y0 = (T)2 * v[l][m].x * scale, y1 = (T)2 * v[l][m].y * scale;
                if (sine && (pos[2 * m] & 1)) y0 = -y0;
                if (sine && (pos[2 * m + 1] & 1)) y1 = -y1;
                x[2 * m][l] = y0;
                x[2 * m + 1][l] = y1;
            }
    }
    SideAddr<2 * P> dst;
    dst.init_pos(a.side[1], t, 1, pos, false);
    if (vec) {
#pragma unroll
        for (int i = 0; i < 2 * P; i++) {
            RVec q;
            if constexpr (RV == 4)
                q = make_float4(x[i][0], x[i][1], x[i][2], x[i][3]);
            else
                q = make_double2(x[i][0], x[i][1]);
            *(RVec *)(out + dst.off[i] + slot * RV) = q;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 2 * P; i++)
#pragma unroll
            for (int e = 0; e < RV; e++)
                if (wl[e] < count) out[dst.off[i] + wl[e]] = x[i][e];
    }
}

template <typename T, int M>
static bool r2r_rows_cfg(int variant, KernelConfig *cfg)
{
    if (variant == 11) {
        if constexpr (R2RRowsCfg<T, M, 8>::exists) {
            cfg->W = R2RRowsCfg<T, M, 8>::W;
            cfg->threads = R2RRowsCfg<T, M, 8>::NT;
            cfg->id = 11;
            cfg->resident = 0;
            return true;
        }
    }
    if (variant == 12) {
        if constexpr (R2RRowsCfg<T, M, 4>::exists) {
            cfg->W = R2RRowsCfg<T, M, 4>::W;
            cfg->threads = R2RRowsCfg<T, M, 4>::NT;
            cfg->id = 12;
            cfg->resident = 0;
            return true;
        }
    }
    return false;
}

template <typename T, int M, int SL>
static hipError_t r2r_rows_launch_sl(const StageArgs &a, hipStream_t s)
{
    const dim3 grid((unsigned)a.ntiles), block(R2RRowsCfg<T, M, SL>::NT);
    if (a.flags & SF_R2R_INVERSE)
        PFFT_LAUNCH((k_r2r_rows<T, M, SL, true>), grid, block, 0, s, a, a.tiles);
    else
        PFFT_LAUNCH((k_r2r_rows<T, M, SL, false>), grid, block, 0, s, a, a.tiles);
    return hipGetLastError();
}

template <typename T, int M>
static bool r2r_rows_launch(int variant, const StageArgs &a, hipStream_t s, hipError_t *e)
{
    if (variant == 11) {
        if constexpr (R2RRowsCfg<T, M, 8>::exists) {
            *e = r2r_rows_launch_sl<T, M, 8>(a, s);
            return true;
        }
    }
    if (variant == 12) {
        if constexpr (R2RRowsCfg<T, M, 4>::exists) {
            *e = r2r_rows_launch_sl<T, M, 4>(a, s);
            return true;
        }
    }
    return false;
}

template <typename T, int N, bool CONTIG, int V>
static void r2r_shape(KernelConfig *cfg)
{
    using S = R2RCfg<T, N, CONTIG, V>;
    cfg->W = S::W;
    cfg->threads = S::NT;
    cfg->id = V;
    cfg->resident = 0;
}

template <typename T, int N, bool CONTIG, int V>
static hipError_t r2r_launch_full(const StageArgs &a, hipStream_t s)
{
    using S = R2RCfg<T, N, CONTIG, V>;
    PFFT_LAUNCH((k_r2r<T, N, CONTIG, S>), dim3((unsigned)a.ntiles), dim3(S::NT), 0, s, a, a.tiles);
    return hipGetLastError();
}

template <typename T, int M, bool CONTIG, int V>
static hipError_t r2r_launch_half(const StageArgs &a, hipStream_t s)
{
    using S = R2RCfg<T, M, CONTIG, V>;
    PFFT_LAUNCH((k_r2r_half<T, M, CONTIG, S>), dim3((unsigned)a.ntiles), dim3(S::NT), 0, s, a, a.tiles);
    return hipGetLastError();
}

inline bool half_length_supported(int M)
{
    switch (M) {
#define PFFT_CASE(n) \
    case n:          \
        return true;
        PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
    default:
        return false;
    }
}

inline bool r2r_half_length_impl(int N) { return N >= 4 && N % 2 == 0 && half_length_supported(N / 2); }

// variants: 0 the default tile, 1 half as many lines (as the complex
// stages'); others use the default.  Even lengths use the half-length kernel
// (tile shapes of the N/2-point transform), lengths 2 and 3 the full one.
template <typename T>
static int r2r_config_t(int N, int contig, int variant, KernelConfig *cfg)
{
    const int v = variant == 1 ? 1 : 0;
    if (r2r_half_length_impl(N)) {
        switch (N / 2) {
#define PFFT_CASE(n)                                                                          \
    case n:                                                                                   \
        if (contig)                                                                           \
            (v == 1 ? r2r_shape<T, n, true, 1> : r2r_shape<T, n, true, 0>)(cfg);             \
        else if (!r2r_rows_cfg<T, n>(variant, cfg))                                           \
            (v == 1 ? r2r_shape<T, n, false, 1> : r2r_shape<T, n, false, 0>)(cfg);           \
        return 0;
            PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
        }
        return -1;
    }
    if (N == 2) {
        (contig ? (v == 1 ? r2r_shape<T, 2, true, 1> : r2r_shape<T, 2, true, 0>)
                : (v == 1 ? r2r_shape<T, 2, false, 1> : r2r_shape<T, 2, false, 0>))(cfg);
        return 0;
    }
    if (N == 3) {
        (contig ? (v == 1 ? r2r_shape<T, 3, true, 1> : r2r_shape<T, 3, true, 0>)
                : (v == 1 ? r2r_shape<T, 3, false, 1> : r2r_shape<T, 3, false, 0>))(cfg);
        return 0;
    }
    return -1;
}

template <typename T>
static hipError_t r2r_launch_t(int N, int contig, int variant, const StageArgs &a, hipStream_t s)
{
    if (r2r_half_length_impl(N)) {
        switch (N / 2) {
#define PFFT_CASE(n)                                                                                          \
    case n:                                                                                                   \
        if (contig)                                                                                           \
            return variant == 1 ? r2r_launch_half<T, n, true, 1>(a, s) : r2r_launch_half<T, n, true, 0>(a, s); \
        {                                                                                                      \
            hipError_t e_ = hipSuccess;                                                                        \
            if (r2r_rows_launch<T, n>(variant, a, s, &e_)) return e_;                                          \
        }                                                                                                      \
        return variant == 1 ? r2r_launch_half<T, n, false, 1>(a, s) : r2r_launch_half<T, n, false, 0>(a, s);
            PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
        }
        return hipErrorInvalidValue;
    }
    if (N == 2)
        return contig ? (variant == 1 ? r2r_launch_full<T, 2, true, 1>(a, s) : r2r_launch_full<T, 2, true, 0>(a, s))
                      : (variant == 1 ? r2r_launch_full<T, 2, false, 1>(a, s) : r2r_launch_full<T, 2, false, 0>(a, s));
    if (N == 3)
        return contig ? (variant == 1 ? r2r_launch_full<T, 3, true, 1>(a, s) : r2r_launch_full<T, 3, true, 0>(a, s))
                      : (variant == 1 ? r2r_launch_full<T, 3, false, 1>(a, s) : r2r_launch_full<T, 3, false, 0>(a, s));
    return hipErrorInvalidValue;
}

}  // namespace pfft
