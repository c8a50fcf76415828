// k_c2c_f64.cpp -- complex128 stage kernel configuration and routing.
#include "k_c2c_impl.hpp"

namespace pfft {

int c2c_config_f64(int N, int contig, int variant, KernelConfig *cfg) { return c2c_config_t<double>(N, contig, variant, cfg); }

hipError_t c2c_launch_f64(int N, int contig, int sign, const KernelConfig &c, const StageArgs &a, hipStream_t s)
{
    if (contig) return sign < 0 ? c2c_f64_c_fwd(N, c, a, s) : c2c_f64_c_bwd(N, c, a, s);
    return sign < 0 ? c2c_f64_s_fwd(N, c, a, s) : c2c_f64_s_bwd(N, c, a, s);
}

hipError_t c2c_launch_multi_f64(int N, int contig, int sign, const KernelConfig &c, const StageArgs *args,
                                const Tile *tiles, long nt, hipStream_t s)
{
    if (contig) return sign < 0 ? c2c_multi_f64_c_fwd(N, c, args, tiles, nt, s) : c2c_multi_f64_c_bwd(N, c, args, tiles, nt, s);
    return sign < 0 ? c2c_multi_f64_s_fwd(N, c, args, tiles, nt, s) : c2c_multi_f64_s_bwd(N, c, args, tiles, nt, s);
}

}  // namespace pfft
