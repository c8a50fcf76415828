// k_energy.hip -- weighted spectral energy L = sum_i w_i |u_i|^2 of a buffer
// and its gradient 2 g w_i u_i: the quadratic loss of the differentiation
// workload (a weight such as |k|^2 on the transform's output), so that the
// forward transform, the loss and the adjoint transform all run in this
// library's kernels.  Two passes for the energy (per-workgroup partial sums
// in FP64, then one workgroup adds them in a fixed order): the result does
// not depend on scheduling.  HBM-bound: one read of u and w per pass.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fft_device.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

// Scratch of the allocation-free entry point: room for the FP64 partial sums
// of one energy call (kEnergyPartials doubles, 8 KiB).  Each device holds its
// own copy for the life of the process; every call on a device shares it.
static __device__ __align__(256) double scratch[kEnergyPartials];

constexpr int kEnergyThreads = 256;

// FP64 sum of one value per thread over the workgroup (64-wide wavefronts).
__device__ __forceinline__ double block_sum(double acc)
{
    __shared__ double red[kEnergyThreads / 64];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kEnergyThreads / 64; k++) s += red[k];
    return s;
}

template <typename T>
__global__ __launch_bounds__(kEnergyThreads) void k_energy_partial(long n, const typename V2<T>::type *__restrict__ u,
                                                                   const T *__restrict__ w,
                                                                   double *__restrict__ partials)
{
    double acc = 0.0;
    const long stride = (long)gridDim.x * kEnergyThreads;
    for (long i = (long)blockIdx.x * kEnergyThreads + threadIdx.x; i < n; i += stride) {
        const auto z = u[i];
        const double a = (double)z.x, b = (double)z.y;
        acc = fma((double)w[i], fma(a, a, b * b), acc);
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kEnergyThreads) void k_energy_total(int m, const double *__restrict__ partials,
                                                                 T *__restrict__ loss)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < m; i += kEnergyThreads) acc += partials[i];
    const double s = block_sum(acc);
    if (threadIdx.x == 0) loss[0] = (T)s;
}

template <typename T>
__global__ __launch_bounds__(kEnergyThreads) void k_energy_grad(long n, const typename V2<T>::type *__restrict__ u,
                                                                const T *__restrict__ w, const T *__restrict__ g,
                                                                typename V2<T>::type *__restrict__ grad)
{
    const T f = (T)2 * g[0];
    const long stride = (long)gridDim.x * kEnergyThreads;
    for (long i = (long)blockIdx.x * kEnergyThreads + threadIdx.x; i < n; i += stride) {
        const T c = f * w[i];
        auto z = u[i];
        z.x *= c;
        z.y *= c;
        grad[i] = z;
    }
}

static int energy_blocks(long n)
{
    const long b = (n + kEnergyThreads - 1) / kEnergyThreads;
    return (int)(b < 1 ? 1 : (b > kEnergyPartials ? kEnergyPartials : b));
}

hipError_t energy_launch(int prec, long n, const void *u, const void *w, double *partials, void *loss, hipStream_t s)
{
    const int g = energy_blocks(n);
    if (prec == 0) {
        hipLaunchKernelGGL(k_energy_partial<float>, dim3(g), dim3(kEnergyThreads), 0, s, n, (const float2 *)u,
                           (const float *)w, partials);
        hipLaunchKernelGGL(k_energy_total<float>, dim3(1), dim3(kEnergyThreads), 0, s, g, (const double *)partials,
                           (float *)loss);
    } else {
        hipLaunchKernelGGL(k_energy_partial<double>, dim3(g), dim3(kEnergyThreads), 0, s, n, (const double2 *)u,
                           (const double *)w, partials);
        hipLaunchKernelGGL(k_energy_total<double>, dim3(1), dim3(kEnergyThreads), 0, s, g, (const double *)partials,
                           (double *)loss);
    }
    return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept: in host code the array's name
// is only a host-side stand-in, never a device address.
static hipError_t scratch_address(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (double *)p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t energy_launch_noalloc(int prec, long n, const void *u, const void *w, void *loss, hipStream_t s)
{
    // every partial the total reads is written by this call's first kernel
    // (earlier calls' contents are never read), so nothing is cleared
    if (energy_blocks(n) > kEnergyPartials) return hipErrorInvalidValue;
    double *partials = nullptr;
    hipError_t e = scratch_address(&partials);
    if (e != hipSuccess) return e;
    return energy_launch(prec, n, u, w, partials, loss, s);
}

hipError_t energy_grad_launch(int prec, long n, const void *u, const void *w, const void *g, void *grad, hipStream_t s)
{
    const long b = (n + kEnergyThreads - 1) / kEnergyThreads;
    const int nb = (int)(b < 1 ? 1 : (b > 16384 ? 16384 : b));
    if (prec == 0)
        hipLaunchKernelGGL(k_energy_grad<float>, dim3(nb), dim3(kEnergyThreads), 0, s, n, (const float2 *)u,
                           (const float *)w, (const float *)g, (float2 *)grad);
    else
        hipLaunchKernelGGL(k_energy_grad<double>, dim3(nb), dim3(kEnergyThreads), 0, s, n, (const double2 *)u,
                           (const double *)w, (const double *)g, (double2 *)grad);
    return hipGetLastError();
}

}  // namespace pfft
