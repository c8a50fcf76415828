// k_r2r_f32.hip -- float instantiations of the real-to-real stage kernels.
#include "k_r2r.hpp"

namespace pfft {

int r2r_config_f32(int N, int contig, int variant, KernelConfig *cfg) { return r2r_config_t<float>(N, contig, variant, cfg); }

hipError_t r2r_launch_f32(int N, int contig, const KernelConfig &cfg, const StageArgs &a, hipStream_t s)
{
    return r2r_launch_t<float>(N, contig, cfg.id, a, s);
}

bool r2r_half_length(int N) { return r2r_half_length_impl(N); }

}  // namespace pfft
