// k_mixed.hip -- partial transforms of lengths without a register-resident
// Stockham plan (factors 5, 7 and other primes, lengths past the radix-2/3
// kernels), for every layout: the gather/scatter addressing is that of the
// Stockham stage kernels, so the redistributions fuse the same way.
//
// One workgroup per tile of W lines.  The lines are staged in LDS and
// transformed there by a mixed-radix Stockham autosort (Sec. 2's partial
// transform, Eqs. 1-2): radix-4 and radix-2 passes for the power-of-two
// part, then radix 3, 5 and 7 butterflies in registers, then any other prime
// factor p by a direct p-point sum per butterfly.  A pass of radix R on a
// line of L points with span S (the product of the earlier radices) takes,
// for every q < L/R, the inputs x_r = A[q + r L/R], multiplies x_r by
// w^{r (q mod S)} with w = e^{sign 2 pi i / (S R)}, forms the R-point DFT
// y_s, and writes y_s to B[(q div S) S R + s S + (q mod S)].
//
// Lines whose largest prime factor exceeds kBluesteinPrime go through
// Bluestein's chirp-z identity jk = (j^2 + k^2 - (k - j)^2) / 2:
//   y_k = a_k sum_j (x_j a_j) conj(a_{k-j}),   a_m = e^{sign pi i m^2 / N},
// a linear convolution of length 2N-1 evaluated as a cyclic one of a
// 7-smooth length M >= 2N-1: forward M-point transform, pointwise product
// with V = DFT_M(v) (v_m = conj(a_m) for |m| < N, wrapped mod M; tabulated
// by the plan for sign -1, the sign +1 table is conj(V[(M-k) mod M])),
// inverse M-point transform, then a_k / M.
//
// KIND_C2C: N complex points -> N bins.  KIND_R2C: N real points -> N/2+1
// bins.  KIND_C2R: N/2+1 bins (Hermitian extension, imaginary parts of bins
// 0 and N/2 ignored) -> N real points.
#include "fft_device.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

constexpr int kMixedThreads = 256;
constexpr int kMixedMaxLds = 160 * 1024;

// cos / sin (2 pi k / 5) and (2 pi k / 7)
#define PFFT_C51 0.30901699437494742410
#define PFFT_S51 0.95105651629515357212
#define PFFT_C52 -0.80901699437494742410
#define PFFT_S52 0.58778525229247312917
#define PFFT_C71 0.62348980185873353053
#define PFFT_S71 0.78183148246802980871
#define PFFT_C72 -0.22252093395631440429
#define PFFT_S72 0.97492791218182360702
#define PFFT_C73 -0.90096886790241912624
#define PFFT_S73 0.43388373911755812048

// Element (line w, position j) of a tile on side s; the tile's flag bit 2+s
// says whether its lines step in I (adjacent lines) or in O (contiguous lines).
__device__ __forceinline__ long mixed_addr(const Side &sd, const Tile &t, int s, int w, int j)
{
    const bool istep = (t.flags >> (2 + s)) & 1;
    const int2 pc = sd.pos[j];
    const long na = sd.na[pc.x];
    const long base = sd.rank_off[t.rank[s] + pc.x * sd.R];
    const long O = t.O[s] + (istep ? 0 : w), I = t.I[s] + (istep ? w : 0);
    return base + (O * na + pc.y) * t.E[s] + I;
}

// Odd prime R-point DFT from cosine/sine constants, pairing x_r with x_{R-r}:
//   y_0 = sum x_r,  y_s = x_0 + sum_r c_{rs} (x_r + x_{R-r}) + i sg sum_r s_{rs} (x_r - x_{R-r})
// for 1 <= s <= (R-1)/2, and y_{R-s} with the sine terms negated.
template <int R, typename T2, typename T>
__device__ __forceinline__ void dft_odd(T2 *x, T sg)
{
    constexpr int H = (R - 1) / 2;
    // cos(2 pi m / R), sin(2 pi m / R) for m = 1..H
    constexpr double C[4] = {1.0, R == 3 ? -0.5 : R == 5 ? PFFT_C51 : PFFT_C71, R == 5 ? PFFT_C52 : PFFT_C72, PFFT_C73};
    constexpr double S[4] = {0.0, R == 3 ? 0.86602540378443864676 : R == 5 ? PFFT_S51 : PFFT_S71,
                             R == 5 ? PFFT_S52 : PFFT_S72, PFFT_S73};
    T2 p[H + 1], m[H + 1];
    T2 y0 = x[0];
#pragma unroll
    for (int r = 1; r <= H; r++) {
        p[r] = c_add(x[r], x[R - r]);
        m[r] = c_sub(x[r], x[R - r]);
        y0 = c_add(y0, p[r]);
    }
    T2 y[R];
#pragma unroll
    for (int s = 1; s <= H; s++) {
        T2 re = x[0], im = c_zero<T2>();
#pragma unroll
        for (int r = 1; r <= H; r++) {
            const int k = (r * s) % R;  // angle index; cos symmetric, sin odd about R/2
            const int kk = k <= H ? k : R - k;
            const T c = (T)C[kk], sn = (T)(k <= H ? S[kk] : -S[kk]);
            re.x += c * p[r].x;
            re.y += c * p[r].y;
            im.x += sn * m[r].x;
            im.y += sn * m[r].y;
        }
        // i * sg * im
        T2 t;
        t.x = -sg * im.y;
        t.y = sg * im.x;
        y[s] = c_add(re, t);
        y[R - s] = c_sub(re, t);
    }
    x[0] = y0;
#pragma unroll
    for (int s = 1; s < R; s++) x[s] = y[s];
}

// One Stockham pass of radix R over the count lines of length L held at
// src (line stride L), result to dst.  tw: e^{-2 pi i t / TW}, t < TW, with
// L | TW.  sign: direction of the transform.
template <typename T, int R>
__device__ void pass_fixed(const typename V2<T>::type *src, typename V2<T>::type *dst, int count, int L, int S,
                           const typename V2<T>::type *__restrict__ tw, int TW, int sign)
{
    using T2 = typename V2<T>::type;
    const int Q = L / R, per = count * Q;
    const int step = TW / (S * R);  // table stride of w = e^{-2 pi i / (S R)}
    const T sg = (T)sign;
    for (int e = threadIdx.x; e < per; e += kMixedThreads) {
        const int w = e / Q, q = e - w * Q;
        const T2 *in = src + (long)w * L;
        T2 *out = dst + (long)w * L;
        const int k = q % S;
        T2 x[R];
#pragma unroll
        for (int r = 0; r < R; r++) {
            x[r] = in[q + r * Q];
            if (r > 0 && k > 0) {
                T2 f = tw[(long)r * k * step % TW];
                f.y *= -sg;  // table holds e^{-...}; sign +1 wants the conjugate
                x[r] = c_mul(x[r], f);
            }
        }
        if constexpr (R == 2) {
            const T2 a0 = x[0];
            x[0] = c_add(a0, x[1]);
            x[1] = c_sub(a0, x[1]);
        } else if constexpr (R == 4) {
            const T2 s02 = c_add(x[0], x[2]), d02 = c_sub(x[0], x[2]);
            const T2 s13 = c_add(x[1], x[3]), d13 = c_sub(x[1], x[3]);
            T2 t;  // sg * i * d13
            t.x = -sg * d13.y;
            t.y = sg * d13.x;
            x[0] = c_add(s02, s13);
            x[2] = c_sub(s02, s13);
            x[1] = c_add(d02, t);
            x[3] = c_sub(d02, t);
        } else {
            dft_odd<R>(x, sg);
        }
        const int base = (q / S) * S * R + k;
#pragma unroll
        for (int s = 0; s < R; s++) out[base + s * S] = x[s];
    }
}

// A pass of any prime radix R by the direct R-point sum (w^{rs} from the
// table: e^{sign 2 pi i r s / R} = tw[(r s mod R) TW / R] conjugated as needed).
template <typename T>
__device__ void pass_generic(const typename V2<T>::type *src, typename V2<T>::type *dst, int count, int L, int S,
                             int R, const typename V2<T>::type *__restrict__ tw, int TW, int sign)
{
    using T2 = typename V2<T>::type;
    const int Q = L / R, per = count * Q;
    const int step = TW / (S * R), rstep = TW / R;
    const T sg = (T)sign;
    for (int e = threadIdx.x; e < per; e += kMixedThreads) {
        const int w = e / Q, q = e - w * Q;
        const T2 *in = src + (long)w * L;
        T2 *out = dst + (long)w * L;
        const int k = q % S;
        const int base = (q / S) * S * R + k;
        for (int s = 0; s < R; s++) {
            T2 acc = c_zero<T2>();
            for (int r = 0; r < R; r++) {
                T2 x = in[q + r * Q];
                if (r > 0 && k > 0) {
                    T2 f = tw[(long)r * k * step % TW];
                    f.y *= -sg;
                    x = c_mul(x, f);
                }
                T2 f = tw[(long)((r * s) % R) * rstep];
                f.y *= -sg;
                const T2 p = c_mul(x, f);
                acc.x += p.x;
                acc.y += p.y;
            }
            out[base + s * S] = acc;
        }
    }
}

// Smallest radix of the pass plan of the remaining length n: 4, 2, 3, 5,
// 7, then the smallest prime factor.
__host__ __device__ inline int mixed_next_radix(int n)
{
    if (n % 4 == 0) return 4;
    if (n % 2 == 0) return 2;
    for (int f = 3; f * f <= n; f += 2)
        if (n % f == 0) return f;
    return n;
}

// Transform `count` lines of length L in place between buffers a and b (the
// result ends in *res), with the table tw of TW entries (L | TW).
template <typename T>
__device__ void mixed_transform(typename V2<T>::type *a, typename V2<T>::type *b, typename V2<T>::type **res,
                                int count, int L, const typename V2<T>::type *__restrict__ tw, int TW, int sign)
{
    using T2 = typename V2<T>::type;
    T2 *src = a, *dst = b;
    int rem = L, S = 1;
    while (rem > 1) {
        const int R = mixed_next_radix(rem);
        switch (R) {
        case 2: pass_fixed<T, 2>(src, dst, count, L, S, tw, TW, sign); break;
        case 3: pass_fixed<T, 3>(src, dst, count, L, S, tw, TW, sign); break;
        case 4: pass_fixed<T, 4>(src, dst, count, L, S, tw, TW, sign); break;
        case 5: pass_fixed<T, 5>(src, dst, count, L, S, tw, TW, sign); break;
        case 7: pass_fixed<T, 7>(src, dst, count, L, S, tw, TW, sign); break;
        default: pass_generic<T>(src, dst, count, L, S, R, tw, TW, sign); break;
        }
        __syncthreads();
        T2 *t = src;
        src = dst;
        dst = t;
        S *= R;
        rem /= R;
    }
    *res = src;
}

template <typename T, int KIND>
__global__ __launch_bounds__(kMixedThreads) void k_mixed(StageArgs a, const Tile *__restrict__ tiles, int sign, int W)
{
    using T2 = typename V2<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    const int M = a.M;                           // Bluestein length (0: direct)
    const int L = M > 0 ? M : N;                 // transform length in LDS
    const int H = N / 2 + 1;
    const int nin = KIND == KIND_C2R ? H : N;    // positions read per line
    const int nout = KIND == KIND_R2C ? H : N;   // positions written per line
    T2 *bufa = (T2 *)smem;
    T2 *bufb = bufa + (long)W * L;
    const Tile &t = tiles[blockIdx.x];
    const int count = t.count;
    const T2 *__restrict__ tw = (const T2 *)a.twiddle;      // L entries e^{-2 pi i t / L}
    const T2 *__restrict__ chirp = (const T2 *)a.twiddle2;  // N entries e^{-pi i m^2 / N}
    const T2 *__restrict__ vhat = (const T2 *)a.twiddle3;   // M entries, sign -1
    const T sg = (T)sign;
    const bool halve = (a.flags & SF_HALVE_INTERIOR) != 0;
    // load (and zero the Bluestein padding / the C2R extension); where the
    // source lines are adjacent (step in I) consecutive threads take
    // consecutive lines, else consecutive positions of a line
    const bool in_across = (t.flags >> 2) & 1;
    for (int e = threadIdx.x; e < count * L; e += kMixedThreads) {
        const int w = in_across ? e % count : e / L, j = in_across ? e / count : e - (e / L) * L;
        T2 x = c_zero<T2>();
        if (KIND == KIND_C2R ? j < H : j < N) {
            const long ad = mixed_addr(a.side[0], t, 0, w, j);
            if constexpr (KIND == KIND_R2C) {
                x.x = ((const T *)a.src)[ad];
            } else {
                x = ((const T2 *)a.src)[ad];
            }
            if constexpr (KIND == KIND_C2R) {
                if (j == 0 || 2 * j == N) x.y = (T)0;
                if (halve && j > 0 && 2 * j < N) x = c_scale(x, (T)0.5);
            }
            if (M > 0 && KIND != KIND_C2R) {
                T2 c = chirp[j];
                c.y *= -sg;
                x = c_mul(x, c);
            }
        }
        bufa[(long)w * L + j] = x;
    }
    __syncthreads();
    if constexpr (KIND == KIND_C2R) {
        // Hermitian extension: bin N-j = conj(bin j) for 0 < j < N-j, then the chirp
        for (int e = threadIdx.x; e < count * N; e += kMixedThreads) {
            const int w = e / N, j = e - w * N;
            if (j >= H) {
                T2 x = bufa[(long)w * L + (N - j)];
                x.y = -x.y;
                bufa[(long)w * L + j] = x;
            }
        }
        __syncthreads();
        if (M > 0) {
            for (int e = threadIdx.x; e < count * N; e += kMixedThreads) {
                const int w = e / N, j = e - w * N;
                T2 c = chirp[j];
                c.y *= -sg;
                bufa[(long)w * L + j] = c_mul(bufa[(long)w * L + j], c);
            }
            __syncthreads();
        }
    }
    T2 *res;
    if (M == 0) {
        mixed_transform<T>(bufa, bufb, &res, count, L, tw, L, sign);
    } else {
        mixed_transform<T>(bufa, bufb, &res, count, L, tw, L, -1);
        for (int e = threadIdx.x; e < count * L; e += kMixedThreads) {
            const int w = e / L, k = e - w * L;
            T2 v = vhat[sign < 0 ? k : (k == 0 ? 0 : L - k)];
            if (sign > 0) v.y = -v.y;
            res[(long)w * L + k] = c_mul(res[(long)w * L + k], v);
        }
        __syncthreads();
        T2 *other = res == bufa ? bufb : bufa;
        mixed_transform<T>(res, other, &res, count, L, tw, L, +1);
    }
    const T scale = (T)a.scale * (M > 0 ? (T)1 / (T)M : (T)1);
    const bool dbl = (a.flags & SF_DOUBLE_INTERIOR) != 0;
    const bool out_across = (t.flags >> 3) & 1;
    for (int e = threadIdx.x; e < count * nout; e += kMixedThreads) {
        const int w = out_across ? e % count : e / nout, k = out_across ? e / count : e - (e / nout) * nout;
        T2 y = res[(long)w * L + k];
        if (M > 0) {
            T2 c = chirp[k];
            c.y *= -sg;
            y = c_mul(y, c);
        }
        const long ad = mixed_addr(a.side[1], t, 1, w, k);
        if constexpr (KIND == KIND_C2R) {
            ((T *)a.dst)[ad] = y.x * scale;
        } else {
            T f = scale;
            if (KIND == KIND_R2C && dbl && k > 0 && 2 * k < N) f *= (T)2;
            ((T2 *)a.dst)[ad] = c_scale(y, f);
        }
    }
}

// Dynamic LDS above 64 KB has to be allowed per kernel once.
static int mixed_prepare()
{
    static const int rc = [] {
        const void *fns[6] = {(const void *)&k_mixed<float, KIND_C2C>,  (const void *)&k_mixed<float, KIND_R2C>,
                              (const void *)&k_mixed<float, KIND_C2R>,  (const void *)&k_mixed<double, KIND_C2C>,
                              (const void *)&k_mixed<double, KIND_R2C>, (const void *)&k_mixed<double, KIND_C2R>};
        for (const void *f : fns)
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMixedMaxLds) != hipSuccess)
                return -1;
        return 0;
    }();
    return rc;
}

int mixed_largest_prime(int n)
{
    int p = 1;
    for (int f = 2; f * f <= n; f++)
        while (n % f == 0) {
            p = f;
            n /= f;
        }
    return n > 1 ? (n > p ? n : p) : p;
}

int mixed_bluestein_length(int N)
{
    if (N < 2 || mixed_largest_prime(N) <= kBluesteinPrime) return 0;
    for (long m = 2L * N - 1;; m++) {
        long r = m;
        for (int f : {2, 3, 5, 7})
            while (r % f == 0) r /= f;
        if (r == 1) return m > (1L << 30) ? -1 : (int)m;
    }
}

static size_t mixed_lds(int prec, int L, int W) { return (size_t)(prec == 0 ? 8 : 16) * 2 * (size_t)W * (size_t)L; }

int mixed_config(int prec, int N, int kind, KernelConfig *cfg)
{
    (void)kind;
    if (N < 1) return -1;
    const int M = mixed_bluestein_length(N);
    if (M < 0) return -1;
    const int L = M > 0 ? M : N;
    int W = 64;
    while (W > 1 && mixed_lds(prec, L, W) > 64 * 1024) W /= 2;
    if (mixed_lds(prec, L, W) > (size_t)kMixedMaxLds) return -1;
    cfg->W = W;
    cfg->threads = kMixedThreads;
    cfg->id = -1;
    cfg->resident = 0;
    return 0;
}

hipError_t mixed_launch(int prec, int kind, int sign, const KernelConfig &cfg, const StageArgs &a, hipStream_t s)
{
    const size_t lds = mixed_lds(prec, a.M > 0 ? a.M : a.N, cfg.W);
    if (lds > 64 * 1024 && mixed_prepare() != 0) return hipErrorInvalidValue;
    dim3 grid((unsigned)a.ntiles), block(kMixedThreads);
#define PFFT_MIXED(T, K) PFFT_LAUNCH((k_mixed<T, K>), grid, block, lds, s, a, a.tiles, sign, cfg.W)
    if (prec == 0) {
        if (kind == KIND_C2C) PFFT_MIXED(float, KIND_C2C);
        else if (kind == KIND_R2C) PFFT_MIXED(float, KIND_R2C);
        else PFFT_MIXED(float, KIND_C2R);
    } else {
        if (kind == KIND_C2C) PFFT_MIXED(double, KIND_C2C);
        else if (kind == KIND_R2C) PFFT_MIXED(double, KIND_R2C);
        else PFFT_MIXED(double, KIND_C2R);
    }
#undef PFFT_MIXED
    return hipGetLastError();
}

}  // namespace pfft
