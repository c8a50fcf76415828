// k_c2c.hpp -- the complex partial-transform stage kernel (one template,
// instantiated per precision in k_c2c_f32.hip / k_c2c_f64.hip).
//
// One workgroup transforms one tile of up to W lines of N points along the
// transform axis.  Each line is read from the source layout's rank blocks
// (a line along an axis split over a grid direction is read from every rank
// of that direction's subgroup: the subarray gather of the exchange) and
// written to the destination layout's blocks, so a redistribution followed by
// a partial transform costs one read and one write of the data.
//
// Strided tiles (transform axis is not the last axis): the tile's lines are
// adjacent in memory, so lanes run across lines and every point of the tile
// is a coalesced row of W elements; fp32 lanes move two lines per 16-byte
// access.  Contiguous tiles (last axis): lanes run along the line.
#pragma once

#include "fft_device.hpp"

namespace pfft {

template <typename T, int N, bool CONTIG>
struct C2CShape {
    static constexpr int P = fft_points(N);
    static constexpr int TPL = N / P;
    static constexpr int VEC = (!CONTIG && sizeof(T) == 4) ? 2 : 1;  // lines per access
    static constexpr int ESZ = 2 * (int)sizeof(T);
    static constexpr int W0 = (fft_npasses(N) > 1) ? (64 * 1024) / (N * ESZ) : 128;
    static constexpr int floor_pow2(int x) { return x < 2 ? 1 : 2 * floor_pow2(x / 2); }
    static constexpr int W1 = floor_pow2(W0 > 64 && fft_npasses(N) > 1 ? 64 : W0);
    static constexpr int W = W1 < VEC ? VEC : W1;  // lines per tile
    static constexpr int nl_for(int nl) { return (TPL * W / nl > 512 && nl < W) ? nl_for(nl * 2) : nl; }
    static constexpr int NL = nl_for(VEC);  // lines per thread
    static constexpr int SLOTS = W / NL;    // line slots per pass
    static constexpr int NT = TPL * SLOTS;  // threads per workgroup
    static_assert(W % NL == 0 && NL % VEC == 0, "tile shape");
};

template <typename T, int N, bool CONTIG, int SIGN>
__global__ __launch_bounds__((C2CShape<T, N, CONTIG>::NT)) void k_c2c(StageArgs a)
{
    using T2 = typename V2<T>::type;
    using T4 = typename V2<T>::quad;
    using S = C2CShape<T, N, CONTIG>;
    constexpr int P = S::P, TPL = S::TPL, VEC = S::VEC, NL = S::NL, SLOTS = S::SLOTS, W = S::W;
    using LT = LdsTile<T2, N, W, CONTIG>;
    __shared__ T2 lds[(fft_npasses(N) > 1) ? LT::SIZE : 1];

    const Tile &t = a.tiles[blockIdx.x];
    const int count = t.count;
    const int tid = threadIdx.x;
    int jt, slot;
    if constexpr (CONTIG) {
        jt = tid % TPL;
        slot = tid / TPL;
    } else {
        slot = tid % SLOTS;
        jt = tid / SLOTS;
    }
    int wl[NL];
#pragma unroll
    for (int l = 0; l < NL; l++) {
        if constexpr (CONTIG)
            wl[l] = slot + l * SLOTS;
        else
            wl[l] = (slot + (l / VEC) * SLOTS) * VEC + (l % VEC);
    }

    SideAddr<P> src, dst;
    src.init(a.side[0], t, 0, jt, TPL, N, CONTIG);
    dst.init(a.side[1], t, 1, jt, TPL, N, CONTIG);
    const T2 *__restrict__ in = (const T2 *)a.src;
    T2 *__restrict__ out = (T2 *)a.dst;
    const T2 *__restrict__ tw = (const T2 *)a.twiddle;

    T2 v[NL][P];
    bool valid[NL];
#pragma unroll
    for (int l = 0; l < NL; l++) valid[l] = wl[l] < count;
    if constexpr (VEC == 2) {
#pragma unroll
        for (int l = 0; l < NL; l += 2) {
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int addr = src.off[m] + wl[l];
                if (valid[l] && valid[l + 1] && (addr & 1) == 0) {
                    T4 q = *(const T4 *)(in + addr);
                    v[l][m].x = q.x;
                    v[l][m].y = q.y;
                    v[l + 1][m].x = q.z;
                    v[l + 1][m].y = q.w;
                } else {
                    v[l][m] = valid[l] ? in[addr] : c_zero<T2>();
                    v[l + 1][m] = valid[l + 1] ? in[addr + 1] : c_zero<T2>();
                }
            }
        }
    } else {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++)
                v[l][m] = valid[l] ? in[src.off[m] + wl[l] * src.stride[m]] : c_zero<T2>();
    }

    fft_passes<T2, N, W, CONTIG, SIGN, NL, 0>(v, wl, jt, lds, tw);

    const T scale = (T)a.scale;
    if (scale != (T)1) {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++) v[l][m] = c_scale(v[l][m], scale);
    }
    if constexpr (VEC == 2) {
#pragma unroll
        for (int l = 0; l < NL; l += 2) {
#pragma unroll
            for (int m = 0; m < P; m++) {
                const int addr = dst.off[m] + wl[l];
                if (valid[l] && valid[l + 1] && (addr & 1) == 0) {
                    T4 q;
                    q.x = v[l][m].x;
                    q.y = v[l][m].y;
                    q.z = v[l + 1][m].x;
                    q.w = v[l + 1][m].y;
                    *(T4 *)(out + addr) = q;
                } else {
                    if (valid[l]) out[addr] = v[l][m];
                    if (valid[l + 1]) out[addr + 1] = v[l + 1][m];
                }
            }
        }
    } else {
#pragma unroll
        for (int l = 0; l < NL; l++)
#pragma unroll
            for (int m = 0; m < P; m++)
                if (valid[l]) out[dst.off[m] + wl[l] * dst.stride[m]] = v[l][m];
    }
}

}  // namespace pfft
