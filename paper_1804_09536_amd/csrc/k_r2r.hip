// k_r2r.hip -- real-to-real partial transforms: the cosine and sine
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
// Each line goes through one N-point complex FFT (Makhoul's reordering):
//   type II:  v_n = x_{p(n)} with p(n) = 2n for n < ceil(N/2), 2(N-1-n)+1
//             after; V = FFT(v); Y_k = 2 Re(e^{-i pi k/2N} V_k).
//   type III: V_k = e^{+i pi k/2N} (X_k - i X_{N-k}) / 2 (X_N = 0);
//             v = unnormalised inverse FFT of V; y_{p(n)} = 2 Re v_n.
//   sine:     type II of x_j (-1)^j, output reversed; type III of the
//             reversed input, output times (-1)^k.
// The lines of a tile are staged as real values in LDS twice (reordering in,
// reordering out), so global accesses stay in natural order.
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

template <typename T, int N, bool CONTIG, class S>
__global__ __launch_bounds__(S::NT) void k_r2r(StageArgs a, const Tile *__restrict__ tiles)
{
    using T2 = typename V2<T>::type;
    constexpr int P = S::P, TPL = S::TPL, NL = S::NL, W = S::W, SLOTS = S::SLOTS;
    constexpr int H = S::H, WL = S::WL;
    using LT = LdsTile<T2, N, WL, CONTIG>;
    constexpr int RLINE = N + 1, RROW = W + 1;  // real staging (aliases the exchange LDS)
    static_assert((CONTIG ? W * RLINE : N * RROW) <= 2 * LT::SIZE, "real staging must fit");
    constexpr bool TQL = N * sizeof(T2) <= 8192;  // quarter-wave twiddles staged in LDS when small
    __shared__ T2 lds[LT::SIZE];
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
static hipError_t r2r_launch_v(const StageArgs &a, hipStream_t s)
{
    using S = R2RCfg<T, N, CONTIG, V>;
    hipLaunchKernelGGL((k_r2r<T, N, CONTIG, S>), dim3((unsigned)a.ntiles), dim3(S::NT), 0, s, a, a.tiles);
    return hipGetLastError();
}

// variants: 0 the default tile, 1 half as many lines (as the complex
// stages'); others use the default
template <typename T>
static int r2r_config_t(int N, int contig, int variant, KernelConfig *cfg)
{
    const int v = variant == 1 ? 1 : 0;
    switch (N) {
#define PFFT_CASE(n)                                                                         \
    case n:                                                                                  \
        if (contig)                                                                          \
            (v == 1 ? r2r_shape<T, n, true, 1> : r2r_shape<T, n, true, 0>)(cfg);            \
        else                                                                                 \
            (v == 1 ? r2r_shape<T, n, false, 1> : r2r_shape<T, n, false, 0>)(cfg);          \
        return 0;
        PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
    default:
        return -1;
    }
}

template <typename T>
static hipError_t r2r_launch_t(int N, int contig, int variant, const StageArgs &a, hipStream_t s)
{
    switch (N) {
#define PFFT_CASE(n)                                                                                   \
    case n:                                                                                            \
        if (contig)                                                                                    \
            return variant == 1 ? r2r_launch_v<T, n, true, 1>(a, s) : r2r_launch_v<T, n, true, 0>(a, s); \
        return variant == 1 ? r2r_launch_v<T, n, false, 1>(a, s) : r2r_launch_v<T, n, false, 0>(a, s);
        PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
    default:
        return hipErrorInvalidValue;
    }
}

int r2r_config(int prec, int N, int contig, int variant, KernelConfig *cfg)
{
    return prec == 0 ? r2r_config_t<float>(N, contig, variant, cfg) : r2r_config_t<double>(N, contig, variant, cfg);
}

hipError_t r2r_launch(int prec, int N, int contig, const KernelConfig &cfg, const StageArgs &a, hipStream_t s)
{
    return prec == 0 ? r2r_launch_t<float>(N, contig, cfg.id, a, s) : r2r_launch_t<double>(N, contig, cfg.id, a, s);
}

}  // namespace pfft
