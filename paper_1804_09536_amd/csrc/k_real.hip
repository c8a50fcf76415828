// k_real.hip -- real-to-complex / complex-to-real stage kernels (placeholder
// until the half-length packing kernels land).
#include "pfft_kernels.hpp"

namespace pfft {

int real_config(int, int, int, KernelConfig *) { return -1; }

hipError_t real_launch(int, int, int, const KernelConfig &, const StageArgs &, hipStream_t)
{
    return hipErrorInvalidValue;
}

}  // namespace pfft
