// k_r2r_f64.hip -- double instantiations of the real-to-real stage kernels.
#include "k_r2r.hpp"

namespace pfft {

int r2r_config_f64(int N, int contig, int variant, KernelConfig *cfg) { return r2r_config_t<double>(N, contig, variant, cfg); }

hipError_t r2r_launch_f64(int N, int contig, const KernelConfig &cfg, const StageArgs &a, hipStream_t s)
{
    return r2r_launch_t<double>(N, contig, cfg.id, a, s);
}

}  // namespace pfft
