// k_c2c_f64_s_fwd.hip -- complex128 stage kernels, strided tiles, sign -1.
#include "k_c2c_impl.hpp"

namespace pfft {

hipError_t c2c_f64_s_fwd(int N, const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    return c2c_launch_ms<double, false, -1>(N, c, a, s);
}

hipError_t c2c_multi_f64_s_fwd(int N, const KernelConfig &c, const StageArgs *args, const Tile *tiles, long nt,
                              hipStream_t s)
{
    return c2c_launch_multi_ms<double, false, -1>(N, c, args, tiles, nt, s);
}

}  // namespace pfft
