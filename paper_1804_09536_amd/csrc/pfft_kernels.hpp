// pfft_kernels.hpp -- host-side interface between the plan engine and the
// HIP kernels of libpfft.  Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "pfft_internal.hpp"

namespace pfft {

// Timing events of the next stage launch on this thread (both null: none).
// With them the launch goes through hipExtLaunchKernelGGL, which stamps the
// kernel's own start and end into the events: per-launch timing without
// event packets between the kernels.
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
LaunchEvents &launch_events();

#define PFFT_LAUNCH(kernel, grid, block, shmem, stream, ...)                                              \
    do {                                                                                                  \
        const ::pfft::LaunchEvents &ev_ = ::pfft::launch_events();                                      \
        if (ev_.start)                                                                                    \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, stream, ev_.start, ev_.stop, 0, __VA_ARGS__); \
        else                                                                                              \
            hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                          \
    } while (0)

// Launch shape of a stage kernel: at most W lines per tile, `threads` per
// workgroup; `id` selects a variant in the dispatch tables.
struct KernelConfig {
    int W = 0;
    int threads = 0;
    int id = 0;        // tile-shape variant (0 default, 1 half, 2 double, 3 double in two LDS portions);
                       // -1: LDS mixed-radix kernel (lengths without a register radix plan)
    int resident = 0;  // 1: grid = resident workgroups looping over tiles; 0: one tile per workgroup
    int xside = 0;     // complex stage whose destination lines step the other way (variant 6)
    int wide = 0;      // 64-bit element offsets (buffers of 2^31 elements or more; variant 7)
    int alt = 0;       // the alternative radix plan (variant 8)
};

// Fills cfg for a stage kernel (kind: StageKind; prec: 0 = f32, 1 = f64;
// N: line length; contig: transform axis is the last axis).  Returns 0, or
// -1 if there is no kernel for this combination.
int kernel_config(int kind, int prec, int N, int contig, int variant, KernelConfig *cfg);

// Enqueue one stage on `stream`.  esize: element bytes for KIND_COPY.
// Returns a hipError_t value (0 on success).
int launch_stage(int kind, int prec, int N, int contig, int sign, const KernelConfig &cfg, size_t esize,
                 const StageArgs &args, hipStream_t stream);

// Per-precision tables (defined in the c2c kernel files).
int c2c_config_f32(int N, int contig, int variant, KernelConfig *cfg);
int c2c_config_f64(int N, int contig, int variant, KernelConfig *cfg);
hipError_t c2c_launch_f32(int N, int contig, int sign, const KernelConfig &cfg, const StageArgs &a, hipStream_t s);
hipError_t c2c_launch_f64(int N, int contig, int sign, const KernelConfig &cfg, const StageArgs &a, hipStream_t s);
hipError_t c2c_launch_multi_f32(int N, int contig, int sign, const KernelConfig &c, const StageArgs *args,
                                const Tile *tiles, long nt, hipStream_t s);
hipError_t c2c_launch_multi_f64(int N, int contig, int sign, const KernelConfig &c, const StageArgs *args,
                                const Tile *tiles, long nt, hipStream_t s);
int copy_config(int N, KernelConfig *cfg);
hipError_t copy_launch(size_t esize, const KernelConfig &cfg, const StageArgs &a, hipStream_t s);
int real_config(int prec, int N, int kind, int variant, KernelConfig *cfg);
// Mixed-radix stages (k_mixed.hip): lines of any length that fits one
// workgroup's LDS; lines whose largest prime factor exceeds kBluesteinPrime
// run Bluestein's convolution of length mixed_bluestein_length(N) (7-smooth,
// >= 2N-1; 0 for the direct plan, -1 if too long).
constexpr int kBluesteinPrime = 32;
int mixed_bluestein_length(int N);
int mixed_config(int prec, int N, int kind, KernelConfig *cfg);
hipError_t mixed_launch(int prec, int kind, int sign, const KernelConfig &cfg, const StageArgs &a, hipStream_t s);
hipError_t real_launch(int prec, int N, int kind, const KernelConfig &cfg, const StageArgs &a, hipStream_t s);
// the same over the tiles of several transforms (member index in bits 8..31 of the tile flags)
hipError_t real_launch_multi(int prec, int N, int kind, const KernelConfig &cfg, const StageArgs *args,
                             const Tile *tiles, long nt, hipStream_t s);
int r2r_config_f32(int N, int contig, int variant, KernelConfig *cfg);
int r2r_config_f64(int N, int contig, int variant, KernelConfig *cfg);
hipError_t r2r_launch_f32(int N, int contig, const KernelConfig &cfg, const StageArgs &a, hipStream_t s);
hipError_t r2r_launch_f64(int N, int contig, const KernelConfig &cfg, const StageArgs &a, hipStream_t s);
// Real-to-real stages of even length N >= 4 run one N/2-point transform
// (twiddles: the N/2-point table and the post table), the others one
// N-point transform (the N-point and 4N-point tables).
bool r2r_half_length(int N);

// Weighted energy sum_i w_i |u_i|^2 of n complex elements into loss[0] (the
// precision's real type), through kEnergyPartials FP64 partial sums; and its
// gradient grad_i = 2 g[0] w_i u_i.
constexpr int kEnergyPartials = 1024;
hipError_t energy_launch(int prec, long n, const void *u, const void *w, double *partials, void *loss, hipStream_t s);
hipError_t energy_grad_launch(int prec, long n, const void *u, const void *w, const void *g, void *grad,
                              hipStream_t s);
// The energy with its partial sums in the library's static per-device scratch
// (no caller scratch, no allocation).
hipError_t energy_launch_noalloc(int prec, long n, const void *u, const void *w, void *loss, hipStream_t s);

}  // namespace pfft
