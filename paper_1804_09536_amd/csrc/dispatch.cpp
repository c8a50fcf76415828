// dispatch.cpp -- routes a stage to its kernel family.
#include <mutex>
#include <unordered_map>

#include "pfft_kernels.hpp"

namespace pfft {

LaunchEvents &launch_events()
{
    static thread_local LaunchEvents ev;
    return ev;
}

int resident_workgroups(const void *kernel, int nt)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess || per_cu < 1) per_cu = 1;
    return cus * per_cu;
}

int kernel_config(int kind, int prec, int N, int contig, int variant, KernelConfig *cfg)
{
    switch (kind) {
    case KIND_C2C: {
        int rc = prec == 0 ? c2c_config_f32(N, contig, variant, cfg) : c2c_config_f64(N, contig, variant, cfg);
        return rc == 0 ? 0 : mixed_config(prec, N, kind, cfg);
    }
    case KIND_COPY: return copy_config(N, cfg);
    case KIND_R2R:
        return prec == 0 ? r2r_config_f32(N, contig, variant, cfg) : r2r_config_f64(N, contig, variant, cfg);
    case KIND_R2C:
    case KIND_C2R: {
        if (!contig) return -1;
        int rc = (N % 2 == 0) ? real_config(prec, N, kind, variant, cfg) : -1;
        return rc == 0 ? 0 : mixed_config(prec, N, kind, cfg);
    }
    default: return -1;
    }
}

int launch_stage(int kind, int prec, int N, int contig, int sign, const KernelConfig &cfg, size_t esize,
                 const StageArgs &a, hipStream_t s)
{
    if (cfg.id < 0 && kind != KIND_COPY && kind != KIND_R2R)
        return (int)mixed_launch(prec, kind, sign, cfg, a, s);
    switch (kind) {
    case KIND_C2C:
        return (int)(prec == 0 ? c2c_launch_f32(N, contig, sign, cfg, a, s) : c2c_launch_f64(N, contig, sign, cfg, a, s));
    case KIND_COPY: return (int)copy_launch(esize, cfg, a, s);
    case KIND_R2C:
    case KIND_C2R: return (int)real_launch(prec, N, kind, cfg, a, s);
    case KIND_R2R:
        return (int)(prec == 0 ? r2r_launch_f32(N, contig, cfg, a, s) : r2r_launch_f64(N, contig, cfg, a, s));
    default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace pfft
