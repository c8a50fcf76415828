// k_c2c_f32_c_fwd.hip -- complex64 stage kernels, contiguous tiles, sign -1.
#include "k_c2c_impl.hpp"

namespace pfft {

hipError_t c2c_f32_c_fwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    return c2c_launch_ms<float, true, -1>(N, c, a, s);
}

}  // namespace pfft
