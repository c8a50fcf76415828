// k_dft.hip -- partial transforms of any length by the direct sum of the
// DFT's definition (Sec. 2, Eqs. 1-2), for lengths without a Stockham radix
// plan (primes, factors 5 and 7, ...).  O(N^2) work per line, so meant for
// the occasional odd axis; the gather/scatter addressing is the same as the
// Stockham stage kernels', so every layout and redistribution is supported.
//
// One workgroup per tile: the tile's W lines and the N-point twiddle table
// go to LDS, then each output bin is one sum over its line.
#include "fft_device.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

constexpr int kDftThreads = 256;
constexpr int kDftMaxLds = 160 * 1024;

// Element (line w, position j) of a tile on side s.
__device__ __forceinline__ long dft_addr(const Side &sd, const Tile &t, int s, int w, int j, bool contig)
{
    const int2 pc = sd.pos[j];
    const long na = sd.na[pc.x];
    const long base = sd.rank_off[t.rank[s] + pc.x * sd.R];
    const long O = t.O[s] + (contig ? w : 0), I = t.I[s] + (contig ? 0 : w);
    return base + (O * na + pc.y) * t.E[s] + I;
}

// KIND_C2C: N complex points -> N bins.  KIND_R2C: N real points -> N/2+1
// bins.  KIND_C2R: N/2+1 bins (Hermitian extension, imaginary parts of bins
// 0 and N/2 ignored) -> N real points.
template <typename T, int KIND>
__global__ __launch_bounds__(kDftThreads) void k_dft(StageArgs a, const Tile *__restrict__ tiles, int sign, int contig,
                                                     int W)
{
    using T2 = typename V2<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = a.N;
    const int H = N / 2 + 1;
    const int nin = KIND == KIND_C2R ? H : N;    // positions read per line
    const int nout = KIND == KIND_R2C ? H : N;   // positions written per line
    T2 *tw = (T2 *)smem;                         // N twiddles e^{sign 2 pi i m / N}
    T2 *line = tw + N;                           // W lines of nin complex values
    const Tile &t = tiles[blockIdx.x];
    const int count = t.count;
    const T2 *tab = (const T2 *)(KIND == KIND_C2C ? a.twiddle : a.twiddle2);  // N-point table
    for (int i = threadIdx.x; i < N; i += kDftThreads) {
        T2 w = tab[i];
        if (sign > 0) w.y = -w.y;
        tw[i] = w;
    }
    const bool halve = (a.flags & SF_HALVE_INTERIOR) != 0;
    for (int e = threadIdx.x; e < count * nin; e += kDftThreads) {
        const int w = e / nin, j = e - w * nin;
        const long ad = dft_addr(a.side[0], t, 0, w, j, contig != 0);
        T2 x;
        if constexpr (KIND == KIND_R2C) {
            x.x = ((const T *)a.src)[ad];
            x.y = (T)0;
        } else {
            x = ((const T2 *)a.src)[ad];
        }
        if constexpr (KIND == KIND_C2R) {
            if (j == 0 || 2 * j == N) x.y = (T)0;
            if (halve && j > 0 && 2 * j < N) x = c_scale(x, (T)0.5);
        }
        line[w * nin + j] = x;
    }
    __syncthreads();
    const T scale = (T)a.scale;
    const bool dbl = (a.flags & SF_DOUBLE_INTERIOR) != 0;
    for (int e = threadIdx.x; e < count * nout; e += kDftThreads) {
        const int w = e / nout, k = e - w * nout;
        const T2 *x = line + w * nin;
        T2 acc = c_zero<T2>();
        if constexpr (KIND == KIND_C2R) {
            // x_k = Re(X_0) + sum_{0<j<N/2} 2 Re(X_j w^{jk}) + Re(X_{N/2} (-1)^k)
            int idx = 0;
            for (int j = 0; j < nin; j++) {
                const T2 p = c_mul(x[j], tw[idx]);
                const T f = (j == 0 || 2 * j == N) ? (T)1 : (T)2;
                acc.x += f * p.x;
                idx += k;
                if (idx >= N) idx -= N;
            }
            ((T *)a.dst)[dft_addr(a.side[1], t, 1, w, k, contig != 0)] = acc.x * scale;
        } else {
            int idx = 0;
            for (int j = 0; j < nin; j++) {
                const T2 p = c_mul(x[j], tw[idx]);
                acc.x += p.x;
                acc.y += p.y;
                idx += k;
                if (idx >= N) idx -= N;
            }
            T f = scale;
            if (KIND == KIND_R2C && dbl && k > 0 && 2 * k < N) f *= (T)2;
            ((T2 *)a.dst)[dft_addr(a.side[1], t, 1, w, k, contig != 0)] = c_scale(acc, f);
        }
    }
}

// Dynamic LDS above 64 KB has to be allowed per kernel once.
int dft_prepare()
{
    static const int rc = [] {
        const void *fns[6] = {(const void *)&k_dft<float, KIND_C2C>,  (const void *)&k_dft<float, KIND_R2C>,
                              (const void *)&k_dft<float, KIND_C2R>,  (const void *)&k_dft<double, KIND_C2C>,
                              (const void *)&k_dft<double, KIND_R2C>, (const void *)&k_dft<double, KIND_C2R>};
        for (const void *f : fns)
            if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kDftMaxLds) != hipSuccess)
                return -1;
        return 0;
    }();
    return rc;
}

static size_t dft_lds(int prec, int N, int W, int kind)
{
    const size_t esz = prec == 0 ? 8 : 16;
    const int nin = kind == KIND_C2R ? N / 2 + 1 : N;
    return esz * ((size_t)N + (size_t)W * nin);
}

int dft_config(int prec, int N, int kind, KernelConfig *cfg)
{
    if (N < 1) return -1;
    int W = 64;
    while (W > 1 && dft_lds(prec, N, W, kind) > 64 * 1024) W /= 2;
    if (dft_lds(prec, N, W, kind) > (size_t)kDftMaxLds) return -1;
    cfg->W = W;
    cfg->threads = kDftThreads;
    cfg->id = -1;
    cfg->resident = 0;
    return 0;
}

hipError_t dft_launch(int prec, int N, int kind, int contig, int sign, const KernelConfig &cfg, const StageArgs &a,
                      hipStream_t s)
{
    const size_t lds = dft_lds(prec, N, cfg.W, kind);
    if (lds > 64 * 1024 && dft_prepare() != 0) return hipErrorInvalidValue;
    dim3 grid((unsigned)a.ntiles), block(kDftThreads);
#define PFFT_DFT(T, K) hipLaunchKernelGGL((k_dft<T, K>), grid, block, lds, s, a, a.tiles, sign, contig, cfg.W)
    if (prec == 0) {
        if (kind == KIND_C2C) PFFT_DFT(float, KIND_C2C);
        else if (kind == KIND_R2C) PFFT_DFT(float, KIND_R2C);
        else PFFT_DFT(float, KIND_C2R);
    } else {
        if (kind == KIND_C2C) PFFT_DFT(double, KIND_C2C);
        else if (kind == KIND_R2C) PFFT_DFT(double, KIND_R2C);
        else PFFT_DFT(double, KIND_C2R);
    }
#undef PFFT_DFT
    return hipGetLastError();
}

}  // namespace pfft
