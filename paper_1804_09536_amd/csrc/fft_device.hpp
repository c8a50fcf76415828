// fft_device.hpp -- device building blocks of libpfft's stage kernels for
// gfx950: complex arithmetic, radix-2^k butterflies, the LDS-staged Stockham
// passes, and the index arithmetic that reads a line from whichever virtual
// ranks' blocks hold it (the subarray gather of the exchange, Sec. 3.2.2,
// done by address computation instead of a separate copy).
#pragma once

#include <hip/hip_runtime.h>

#include "pfft_internal.hpp"

namespace pfft {

template <typename T>
struct V2;
template <>
struct V2<float> {
    using type = float2;
    using quad = float4;
};
template <>
struct V2<double> {
    using type = double2;
    using quad = double4;
};

template <typename T2>
__device__ __forceinline__ T2 c_add(T2 a, T2 b)
{
    T2 r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename T2>
__device__ __forceinline__ T2 c_sub(T2 a, T2 b)
{
    T2 r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename T2>
__device__ __forceinline__ T2 c_mul(T2 a, T2 b)
{
    T2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename T2, typename T>
__device__ __forceinline__ T2 c_scale(T2 a, T s)
{
    T2 r;
    r.x = a.x * s;
    r.y = a.y * s;
    return r;
}
template <typename T2>
__device__ __forceinline__ T2 c_zero()
{
    T2 r;
    r.x = 0;
    r.y = 0;
    return r;
}

// Streaming (non-temporal) store of a complex value or a pair of them: the
// data is not read again by this kernel, so it need not occupy the caches.
template <typename V>
__device__ __forceinline__ void store_stream(V *p, V v)
{
    using E = decltype(v.x);
    if constexpr (sizeof(V) == 2 * sizeof(E)) {
        typedef E n2 __attribute__((ext_vector_type(2)));
        n2 t = {v.x, v.y};
        __builtin_nontemporal_store(t, (n2 *)p);
    } else {
        typedef E n4 __attribute__((ext_vector_type(4)));
        n4 t = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(t, (n4 *)p);
    }
}

// Streaming (non-temporal) load of one complex value or a pair of them.
template <typename V>
__device__ __forceinline__ V load_stream(const V *p)
{
    using E = decltype(p->x);
    V v;
    if constexpr (sizeof(V) == 2 * sizeof(E)) {
        typedef E n2 __attribute__((ext_vector_type(2)));
        n2 t = __builtin_nontemporal_load((const n2 *)p);
        v.x = t.x;
        v.y = t.y;
    } else {
        typedef E n4 __attribute__((ext_vector_type(4)));
        n4 t = __builtin_nontemporal_load((const n4 *)p);
        v.x = t.x;
        v.y = t.y;
        v.z = t.z;
        v.w = t.w;
    }
    return v;
}

// ---------------------------------------------------------------------------
// Radix-R DFT in registers, R = 1, 2, 4, 8, 16:  a_s <- sum_r a_r w^{SIGN r s},
// w = e^{2 pi i / R}.  Built by even/odd splitting; multiplications by the
// exact roots 1, -1, +-i are done by sign changes and swaps.

// cos(2 pi k / 16) and sin(2 pi k / 16), k = 0..7
#define PFFT_C1 0.92387953251128675613
#define PFFT_S1 0.38268343236508977173
#define PFFT_H 0.70710678118654752440

template <int R, int SIGN, int S, typename T2>
__device__ __forceinline__ T2 root_mul(T2 x)
{
    using T = decltype(x.x);
    constexpr int k = (16 / R) * S;  // exponent in units of 2 pi / 16, 0 <= k < 8
    static_assert(k >= 0 && k < 8, "root index");
    T2 r;
    if constexpr (k == 0) {
        return x;
    } else if constexpr (k == 4) {  // w = SIGN * i
        if constexpr (SIGN > 0) {
            r.x = -x.y;
            r.y = x.x;
        } else {
            r.x = x.y;
            r.y = -x.x;
        }
        return r;
    } else if constexpr (k == 2) {  // w = (1 + SIGN i) / sqrt 2
        const T h = (T)PFFT_H;
        if constexpr (SIGN > 0) {
            r.x = (x.x - x.y) * h;
            r.y = (x.y + x.x) * h;
        } else {
            r.x = (x.x + x.y) * h;
            r.y = (x.y - x.x) * h;
        }
        return r;
    } else if constexpr (k == 6) {  // w = (-1 + SIGN i) / sqrt 2
        const T h = (T)PFFT_H;
        if constexpr (SIGN > 0) {
            r.x = (-x.x - x.y) * h;
            r.y = (-x.y + x.x) * h;
        } else {
            r.x = (-x.x + x.y) * h;
            r.y = (-x.y - x.x) * h;
        }
        return r;
    } else {
        // k = 1, 3, 5, 7
        constexpr double cs[8] = {1.0, PFFT_C1, PFFT_H, PFFT_S1, 0.0, -PFFT_S1, -PFFT_H, -PFFT_C1};
        constexpr double sn[8] = {0.0, PFFT_S1, PFFT_H, PFFT_C1, 1.0, PFFT_C1, PFFT_H, PFFT_S1};
        T2 w;
        w.x = (T)cs[k];
        w.y = (T)(SIGN * sn[k]);
        return c_mul(x, w);
    }
}

template <int R, int SIGN, int S, typename T2>
__device__ __forceinline__ void radix_combine(T2 *a, const T2 *e, const T2 *o)
{
    if constexpr (S < R / 2) {
        T2 t = root_mul<R, SIGN, S>(o[S]);
        a[S] = c_add(e[S], t);
        a[S + R / 2] = c_sub(e[S], t);
        radix_combine<R, SIGN, S + 1>(a, e, o);
    }
}

template <int R, int SIGN, typename T2>
__device__ __forceinline__ void dft_regs(T2 *a)
{
    if constexpr (R == 1) {
        return;
    } else if constexpr (R == 2) {
        T2 t = a[0];
        a[0] = c_add(t, a[1]);
        a[1] = c_sub(t, a[1]);
    } else if constexpr (R == 3) {
        using T = decltype(a[0].x);
        const T s3 = (T)(SIGN * 0.86602540378443864676);  // SIGN * sqrt(3)/2
        const T2 p = c_add(a[1], a[2]);
        const T2 m = c_sub(a[1], a[2]);
        T2 t;
        t.x = a[0].x - (T)0.5 * p.x;
        t.y = a[0].y - (T)0.5 * p.y;
        T2 u;  // i * s3 * m
        u.x = -s3 * m.y;
        u.y = s3 * m.x;
        a[0] = c_add(a[0], p);
        a[1] = c_add(t, u);
        a[2] = c_sub(t, u);
    } else {
        constexpr int H = R / 2;
        T2 e[H], o[H];
#pragma unroll
        for (int i = 0; i < H; i++) {
            e[i] = a[2 * i];
            o[i] = a[2 * i + 1];
        }
        dft_regs<H, SIGN>(e);
        dft_regs<H, SIGN>(o);
        radix_combine<R, SIGN, 0>(a, e, o);
    }
}

// ---------------------------------------------------------------------------
// Radix plan of an N-point line, N = 2^a or 3 * 2^a (2 <= N <= 4096 / 6144).
// Each thread of a line owns P points; every pass has a radix dividing P.
// Radix-3 lengths run the power-of-two passes first and one radix-3 pass
// last, so the span L of every pass is a power of two.

__host__ __device__ constexpr bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

__host__ __device__ constexpr int pow2_part(int N) { return is_pow2(N) ? N : N / 3; }

__host__ __device__ constexpr int fft_points_pow2(int N) { return N <= 16 ? N : (N <= 512 ? 8 : 16); }

// Points per thread of the power-of-two passes (the largest radix).  For
// 3 * 2^a lengths the three-fold points per thread would double the
// registers of the power-of-two plan, so the power-of-two part is halved
// there: 12 points per thread up to 768 (one more LDS exchange, half the
// registers: 384^3 -16 %), 24 from 1536 on (whose 16-line tiles measured
// slower with the extra exchanges).
__host__ __device__ constexpr int fft_p2(int N)
{
    if (is_pow2(N)) return fft_points_pow2(N);
    const int N2 = N / 3;
    return N2 <= 8 ? N2 : (N2 <= 256 ? 4 : 8);
}

// The alternative radix plan of a length (a result-neutral tuning choice):
// the other power-of-two part, 16 instead of 8 points per thread (or 8
// instead of 16 from 1024 on) for powers of two from 32, 8 instead of 4 (or
// 4 instead of 8) for 3 * 2^a from 48; other lengths have none.
__host__ __device__ constexpr int fft_p2_alt(int N)
{
    if (is_pow2(N)) return N < 32 ? fft_p2(N) : (fft_p2(N) == 8 ? 16 : 8);
    return N / 3 <= 8 ? fft_p2(N) : (fft_p2(N) == 4 ? 8 : 4);
}
__host__ __device__ constexpr int fft_p2a(int N, int ALT) { return ALT ? fft_p2_alt(N) : fft_p2(N); }

__host__ __device__ constexpr int fft_points_a(int N, int ALT) { return is_pow2(N) ? fft_p2a(N, ALT) : 3 * fft_p2a(N, ALT); }
__host__ __device__ constexpr int fft_points(int N) { return fft_points_a(N, 0); }

__host__ __device__ constexpr int fft_npasses_a(int N, int ALT)
{
    int n = 0, rem = pow2_part(N);
    const int P = fft_p2a(N, ALT);
    while (rem > 1) {
        rem = rem >= P ? rem / P : 1;
        n++;
    }
    return is_pow2(N) ? n : n + 1;
}
__host__ __device__ constexpr int fft_npasses(int N) { return fft_npasses_a(N, 0); }

__host__ __device__ constexpr int fft_radix_a(int N, int ALT, int pass)
{
    if (!is_pow2(N) && pass == fft_npasses_a(N, ALT) - 1) return 3;
    int P = fft_p2a(N, ALT), rem = pow2_part(N);
    for (int i = 0; i < pass; i++) rem = rem >= P ? rem / P : 1;
    return rem >= P ? P : rem;
}

__host__ __device__ constexpr int fft_span_a(int N, int ALT, int pass)  // L = product of radices before `pass`
{
    int L = 1;
    for (int i = 0; i < pass; i++) L *= fft_radix_a(N, ALT, i);
    return L;
}

__host__ __device__ constexpr bool fft_supported(int N)
{
    return N >= 2 && (is_pow2(N) ? N <= 4096 : (N % 3 == 0 && is_pow2(N / 3) && N <= 6144));
}

// Butterflies of one pass on the P registers of one line slot.  Register m
// holds position jt + m*TPL of the line on entry (for every pass) and, after
// the butterflies, output (b, s) of butterfly b sits in register b + s*(P/R).
template <typename T2, int N, int P, int R, int L, int SIGN>
__device__ __forceinline__ void pass_butterflies(T2 (&v)[P], int jt, const T2 *__restrict__ tw)
{
    constexpr int TPL = N / P;
    constexpr int NB = P / R;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        T2 x[R];
#pragma unroll
        for (int r = 0; r < R; r++) x[r] = v[b + r * NB];
        if constexpr (L > 1) {
            const int q = jt + b * TPL;
            const int k = q & (L - 1);
#pragma unroll
            for (int r = 1; r < R; r++) {
                T2 w = tw[r * k * (N / (L * R))];
                if constexpr (SIGN > 0) w.y = -w.y;
                x[r] = c_mul(x[r], w);
            }
        }
        dft_regs<R, SIGN>(x);
#pragma unroll
        for (int s = 0; s < R; s++) v[b + s * NB] = x[s];
    }
}

// Position in the line of output (b, s) of a pass.
template <int N, int P, int R, int L>
__device__ __forceinline__ int pass_out_index(int jt, int b, int s)
{
    constexpr int TPL = N / P;
    const int q = jt + b * TPL;
    return (q / L) * (L * R) + s * L + (q & (L - 1));
}

// LDS addressing of a tile of W lines of N points.
//  strided tiles: point-major, lines contiguous, rows padded by 16 bytes;
//  contiguous tiles: line-major, one pad element after every 8 points.
#ifndef PFFT_STRIDED_PAD_BYTES
#define PFFT_STRIDED_PAD_BYTES 16
#endif
template <typename T2, int N, int W, bool CONTIG>
struct LdsTile {
    static constexpr int PADW = PFFT_STRIDED_PAD_BYTES / (int)sizeof(T2);
    static constexpr int ROW = W + PADW;
    static constexpr int LINE = N + N / 8;
    static constexpr int SIZE = CONTIG ? W * LINE : N * ROW;
    __device__ static __forceinline__ int idx(int w, int j)
    {
        if constexpr (CONTIG)
            return w * LINE + j + (j >> 3);
        else
            return j * ROW + w;
    }
};

// Run all passes of an N-point transform on the register sets of NL line
// slots (lines w_l of the tile), staging through LDS between passes.  On
// entry register m of slot l holds point jt + m*TPL of line w_l; on exit the
// transform's output point jt + m*TPL.  The LDS holds WL lines: with H > 1
// portions, slots [h*NL/H, (h+1)*NL/H) (lines [h*WL, (h+1)*WL)) exchange in
// turn, so a tile of H*WL lines needs the LDS of WL lines.
// ALT selects the alternative radix plan (fft_p2_alt).  With HS > 1
// portions over line slots instead (H = 1): the slots of the tile form HS
// groups, the thread's slot group is `grp`, and wl holds the thread's lines
// numbered inside its group (the LDS then holds WL = W / HS lines); group h
// exchanges in turn h, every line of its threads at once.
template <typename T2, int N, int WL, bool CONTIG, int SIGN, int NL, int H, int PASS, int ALT = 0, int HS = 1>
__device__ __forceinline__ void fft_passes(T2 (&v)[NL][fft_points_a(N, ALT)], const int (&wl)[NL], int jt, T2 *lds,
                                           const T2 *__restrict__ tw, int grp = 0)
{
    constexpr int P = fft_points_a(N, ALT);
    constexpr int NP = fft_npasses_a(N, ALT);
    constexpr int R = fft_radix_a(N, ALT, PASS);
    constexpr int L = fft_span_a(N, ALT, PASS);
    constexpr int TPL = N / P;
    constexpr int NLH = NL / H;
    static_assert(NL % H == 0, "portions must split the line slots evenly");
    static_assert(HS == 1 || H == 1, "portions over lines or over slots, not both");
    using LT = LdsTile<T2, N, WL, CONTIG>;
#pragma unroll
    for (int l = 0; l < NL; l++) pass_butterflies<T2, N, P, R, L, SIGN>(v[l], jt, tw);
    if constexpr (PASS + 1 < NP && HS > 1) {
        for (int h = 0; h < HS; h++) {
            if (PASS > 0 || h > 0) __syncthreads();
            if (grp == h) {
#pragma unroll
                for (int l = 0; l < NL; l++)
#pragma unroll
                    for (int b = 0; b < P / R; b++)
#pragma unroll
                        for (int s = 0; s < R; s++)
                            lds[LT::idx(wl[l], pass_out_index<N, P, R, L>(jt, b, s))] = v[l][b + s * (P / R)];
            }
            __syncthreads();
            if (grp == h) {
#pragma unroll
                for (int l = 0; l < NL; l++)
#pragma unroll
                    for (int m = 0; m < P; m++) v[l][m] = lds[LT::idx(wl[l], jt + m * TPL)];
            }
        }
        fft_passes<T2, N, WL, CONTIG, SIGN, NL, H, PASS + 1, ALT, HS>(v, wl, jt, lds, tw, grp);
    } else if constexpr (PASS + 1 < NP) {
#pragma unroll
        for (int h = 0; h < H; h++) {
            if (PASS > 0 || h > 0) __syncthreads();
#pragma unroll
            for (int l = h * NLH; l < (h + 1) * NLH; l++) {
#pragma unroll
                for (int b = 0; b < P / R; b++)
#pragma unroll
                    for (int s = 0; s < R; s++)
                        lds[LT::idx(wl[l] - h * WL, pass_out_index<N, P, R, L>(jt, b, s))] = v[l][b + s * (P / R)];
            }
            __syncthreads();
#pragma unroll
            for (int l = h * NLH; l < (h + 1) * NLH; l++)
#pragma unroll
                for (int m = 0; m < P; m++) v[l][m] = lds[LT::idx(wl[l] - h * WL, jt + m * TPL)];
        }
        fft_passes<T2, N, WL, CONTIG, SIGN, NL, H, PASS + 1, ALT, HS>(v, wl, jt, lds, tw, grp);
    }
}

// ---------------------------------------------------------------------------
// Addressing of one side of a stage for the P positions a thread owns.
// Offsets are 32-bit (Off = int) where every buffer of the plan has fewer than
// 2^31 elements, 64-bit (Off = long) in the kernels of larger plans.
template <int P, typename Off = int>
struct SideAddr {
    Off off[P];     // element offset of position m in line 0 of the tile
    Off stride[P];  // distance between consecutive lines of the tile

    __device__ __forceinline__ void init(const Side &sd, const Tile &t, int s, int jt, int TPL, int N, bool contig)
    {
        const int rank = t.rank[s];
        const long O = t.O[s], E = t.E[s], I = t.I[s];
        if (sd.ublock > 0) {
            // every block has the same shape: block index and offsets by arithmetic
            const int un = sd.un;
#pragma unroll
            for (int m = 0; m < P; m++) {
                int j = jt + m * TPL;
                if (j >= N) j = N - 1;
                const int c = (unsigned)j / (unsigned)un;
                const int loc = j - c * un;
                const long base = (long)(rank + c * sd.R) * sd.ublock;
                off[m] = (Off)(base + (O * un + loc) * E + I);
                stride[m] = contig ? (Off)(un * E) : (Off)1;
            }
            return;
        }
        // table lookups in three rounds (every position's block first, then
        // the blocks' extents and offsets) so each round's loads are in flight
        // together instead of one dependent chain per position
        int2 pc[P];
#pragma unroll
        for (int m = 0; m < P; m++) {
            int j = jt + m * TPL;
            if (j >= N) j = N - 1;  // callers mask positions past the end
            pc[m] = sd.pos[j];
        }
        long na[P], base[P];
#pragma unroll
        for (int m = 0; m < P; m++) {
            na[m] = sd.na[pc[m].x];
            base[m] = sd.rank_off[rank + pc[m].x * sd.R];
        }
#pragma unroll
        for (int m = 0; m < P; m++) {
            off[m] = (Off)(base[m] + (O * na[m] + pc[m].y) * E + I);
            stride[m] = contig ? (Off)(na[m] * E) : (Off)1;
        }
    }

    // The same for explicit positions pos[m] (each in [0, N)).
    __device__ __forceinline__ void init_pos(const Side &sd, const Tile &t, int s, const int (&pos)[P], bool contig)
    {
        const int rank = t.rank[s];
        const long O = t.O[s], E = t.E[s], I = t.I[s];
        if (sd.ublock > 0) {
            const int un = sd.un;
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int j = pos[m];
                const int c = (unsigned)j / (unsigned)un;
                const int loc = j - c * un;
                const long base = (long)(rank + c * sd.R) * sd.ublock;
                off[m] = (Off)(base + (O * un + loc) * E + I);
                stride[m] = contig ? (Off)(un * E) : (Off)1;
            }
            return;
        }
        int2 pc[P];
#pragma unroll
        for (int m = 0; m < P; m++) pc[m] = sd.pos[pos[m]];
        long na[P], base[P];
#pragma unroll
        for (int m = 0; m < P; m++) {
            na[m] = sd.na[pc[m].x];
            base[m] = sd.rank_off[rank + pc[m].x * sd.R];
        }
#pragma unroll
        for (int m = 0; m < P; m++) {
            off[m] = (Off)(base[m] + (O * na[m] + pc[m].y) * E + I);
            stride[m] = contig ? (Off)(na[m] * E) : (Off)1;
        }
    }
};

}  // namespace pfft
