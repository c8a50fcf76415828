// k_c2c_impl.hpp -- host dispatch over the instantiated lengths of k_c2c.
#pragma once

#include "k_c2c.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

template <typename T, int N, bool CONTIG>
static hipError_t c2c_launch_n(int sign, const StageArgs &a, hipStream_t s)
{
    using S = C2CShape<T, N, CONTIG>;
    dim3 grid((unsigned)a.ntiles), block(S::NT);
    if (sign < 0)
        hipLaunchKernelGGL((k_c2c<T, N, CONTIG, -1>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_c2c<T, N, CONTIG, 1>), grid, block, 0, s, a);
    return hipGetLastError();
}

template <typename T, int N>
static void c2c_cfg_n(int contig, KernelConfig *c)
{
    if (contig) {
        c->W = C2CShape<T, N, true>::W;
        c->threads = C2CShape<T, N, true>::NT;
    } else {
        c->W = C2CShape<T, N, false>::W;
        c->threads = C2CShape<T, N, false>::NT;
    }
    c->id = 0;
}

#define PFFT_FOR_EACH_N(X)                                                                          \
    X(2) X(4) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096) X(3) X(6) X(12) X(24) \
        X(48) X(96) X(192) X(384) X(768) X(1536) X(3072)

template <typename T>
static int c2c_config_t(int N, int contig, KernelConfig *cfg)
{
    switch (N) {
#define PFFT_CASE(n)              \
    case n:                       \
        c2c_cfg_n<T, n>(contig, cfg); \
        return 0;
        PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
    default:
        return -1;
    }
}

template <typename T>
static hipError_t c2c_launch_t(int N, int contig, int sign, const StageArgs &a, hipStream_t s)
{
    switch (N) {
#define PFFT_CASE(n)                                                                   \
    case n:                                                                            \
        return contig ? c2c_launch_n<T, n, true>(sign, a, s) : c2c_launch_n<T, n, false>(sign, a, s);
        PFFT_FOR_EACH_N(PFFT_CASE)
#undef PFFT_CASE
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace pfft
