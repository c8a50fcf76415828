// k_c2c_f32.hip -- complex64 partial-transform stage kernels.
#include "k_c2c_impl.hpp"

namespace pfft {

int c2c_config_f32(int N, int contig, KernelConfig *cfg) { return c2c_config_t<float>(N, contig, cfg); }

hipError_t c2c_launch_f32(int N, int contig, int sign, const KernelConfig &, const StageArgs &a, hipStream_t s)
{
    return c2c_launch_t<float>(N, contig, sign, a, s);
}

}  // namespace pfft
