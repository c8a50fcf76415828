// k_c2c_f64.hip -- complex128 partial-transform stage kernels.
#include "k_c2c_impl.hpp"

namespace pfft {

int c2c_config_f64(int N, int contig, KernelConfig *cfg) { return c2c_config_t<double>(N, contig, cfg); }

hipError_t c2c_launch_f64(int N, int contig, int sign, const KernelConfig &, const StageArgs &a, hipStream_t s)
{
    return c2c_launch_t<double>(N, contig, sign, a, s);
}

}  // namespace pfft
