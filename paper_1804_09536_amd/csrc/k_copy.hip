// k_copy.hip -- standalone redistribution kernel: a pure permutation that
// moves every element to its place in another layout (Eq. gt), line by line
// along the last axis, with both sides addressed through the same tables as
// the transform kernels.  Used by pfft_redistribute and by the unfused and
// pack+realign execution paths.
#include "fft_device.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

constexpr int kCopyThreads = 256;
constexpr int kCopyUnroll = 8;

// One workgroup per tile of lines; TPL threads per line slot (a power of two
// <= 64), positions j = jt + u*TPL in chunks of kCopyUnroll per thread.
template <typename E, typename Off>
__global__ __launch_bounds__(kCopyThreads) void k_copy(StageArgs a, int TPL)
{
    const Tile &t = a.tiles[blockIdx.x];
    const int count = t.count;
    const int N = a.N;
    const int jt = threadIdx.x % TPL;
    const int slot = threadIdx.x / TPL;
    const int SLOTS = kCopyThreads / TPL;
    const E *__restrict__ in = (const E *)a.src;
    E *__restrict__ out = (E *)a.dst;
    for (int j0 = 0; j0 < N; j0 += TPL * kCopyUnroll) {
        SideAddr<kCopyUnroll, Off> s, d;
        // lines step in O (contiguous lines) unless the tile says I on that side
        s.init(a.side[0], t, 0, j0 + jt, TPL, N, !(t.flags & 4));
        d.init(a.side[1], t, 1, j0 + jt, TPL, N, !(t.flags & 8));
        bool ok[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; u++) ok[u] = j0 + jt + u * TPL < N;
        for (int w0 = slot; w0 < count; w0 += 2 * SLOTS) {
            const int w1 = w0 + SLOTS;
            E v0[kCopyUnroll], v1[kCopyUnroll];
#pragma unroll
            for (int u = 0; u < kCopyUnroll; u++) {
                if (ok[u]) v0[u] = in[s.off[u] + w0 * s.stride[u]];
                if (ok[u] && w1 < count) v1[u] = in[s.off[u] + w1 * s.stride[u]];
            }
#pragma unroll
            for (int u = 0; u < kCopyUnroll; u++) {
                if (ok[u]) out[d.off[u] + w0 * d.stride[u]] = v0[u];
                if (ok[u] && w1 < count) out[d.off[u] + w1 * d.stride[u]] = v1[u];
            }
        }
    }
}

static int copy_tpl(int N)
{
    int tpl = 1;
    while (tpl < 64 && tpl * kCopyUnroll < N) tpl *= 2;
    return tpl;
}

int copy_config(int N, KernelConfig *cfg)
{
    if (N < 1) return -1;
    const int tpl = copy_tpl(N);
    const int slots = kCopyThreads / tpl;
    // enough lines per tile for ~4096 elements of work per workgroup
    int w = slots;
    while (w * N < 4096 && w < 4096) w *= 2;
    cfg->W = w;
    cfg->threads = kCopyThreads;
    cfg->id = tpl;
    return 0;
}

hipError_t copy_launch(size_t esize, const KernelConfig &cfg, const StageArgs &a, hipStream_t s)
{
    dim3 grid((unsigned)a.ntiles), block(kCopyThreads);
    // 64-bit offsets in plans with buffers of 2^31 elements or more
    const long key = (long)esize * (cfg.wide ? -1 : 1);
    switch (key) {
    case 4: PFFT_LAUNCH((k_copy<float, int>), grid, block, 0, s, a, cfg.id); break;
    case 8: PFFT_LAUNCH((k_copy<float2, int>), grid, block, 0, s, a, cfg.id); break;
    case 16: PFFT_LAUNCH((k_copy<double2, int>), grid, block, 0, s, a, cfg.id); break;
    case -4: PFFT_LAUNCH((k_copy<float, long>), grid, block, 0, s, a, cfg.id); break;
    case -8: PFFT_LAUNCH((k_copy<float2, long>), grid, block, 0, s, a, cfg.id); break;
    case -16: PFFT_LAUNCH((k_copy<double2, long>), grid, block, 0, s, a, cfg.id); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pfft
