// pfft_internal.hpp -- structures shared by the host plan engine and the HIP
// kernels of libpfft.  Not part of the public ABI.
#pragma once

#include <stdint.h>

namespace pfft {

constexpr int kMaxDims = 8;

// One line tile of a stage: up to W lines that share, on both the source
// side (0) and the destination side (1), the virtual rank coordinates of every
// grid direction except the one splitting the transform axis and the inner
// extent E (product of local extents after the transform axis).  O is the
// local "outer" index (C-order index over the axes before the transform axis)
// and I the inner index of a line.
//
// The element at position j of a line (O, I) on side s lives at
//   rank_off[rank + c(j)*R] + (O * na[c(j)] + loc(j)) * E + I
// where (c(j), loc(j)) = pos[j] names the block along the transform axis and
// the local index there, na[c] is that block's local extent of the axis and R
// the rank stride of the grid direction splitting it (0 if whole).
//
// Lines w = 0..count-1 of a tile:
//   run == 0, contiguous mode (transform axis last): (O + w, I);
//   run == 0, strided mode: (O, I + w);
//   run > 0 (strided mode only, a tile that continues over consecutive runs
//   of `run` lines, e.g. where the inner extent is shorter than W): with
//   q = b0 + w, line w is (O + q / run, I + q % run), i.e. element offset
//   (q % run) + (q / run) * ostr[s] from line (O, I) of the tile's first run.
struct Tile {
    int32_t rank[2];
    int32_t count;
    int32_t flags;  // bit 0: every line pair (2i, 2i+1) is two adjacent elements starting at an even one, on both sides
    int32_t O[2];
    int32_t E[2];
    int32_t I[2];
    int32_t b0;
    int32_t run;
    int32_t ostr[2];
    int32_t reserved[2];
};
static_assert(sizeof(Tile) == 64, "Tile must be 64 bytes");

struct Side {
    const int64_t *rank_off;  // element offset of each rank's block
    const int2 *pos;          // per position along the axis: (block, local index)
    const int32_t *na;        // per block along the axis: local extent
    int32_t R;                // rank stride of the direction splitting the axis
    int32_t un;               // uniform layouts: local extent of the axis in every block
    int64_t ublock;           // uniform layouts (all blocks equal): block size, else 0
};

// Kind of a stage kernel.
enum StageKind : int32_t {
    KIND_C2C = 0,   // complex line transform
    KIND_COPY = 1,  // pure permutation of lines (redistribution)
    KIND_R2C = 2,   // real line of N -> N/2+1 bins
    KIND_C2R = 3,   // N/2+1 bins -> real line of N
    KIND_R2R = 4,   // real line -> real line (cosine / sine transform of type II, or its inverse of type III)
};

// Flags of a stage launch.
enum StageFlags : int32_t {
    SF_HALVE_INTERIOR = 1,   // C2R: halve bins 0<k<N-k first (adjoint of R2C)
    SF_DOUBLE_INTERIOR = 2,  // R2C: double bins 0<k<N-k after (adjoint of C2R)
    SF_R2R_INVERSE = 4,      // R2R: type III (the inverse) instead of type II
    SF_R2R_SINE = 8,         // R2R: sine instead of cosine transform
    SF_R2R_ADJOINT = 16,     // R2R: the transpose of the transform (type III: special input
                             // element doubled; type II: special output element halved)
    SF_XCD_ORDER = 32,       // complex strided stage, one tile per workgroup: each of the 8 XCDs
                             // (workgroup b runs on XCD b % 8) takes one contiguous range of tiles
    SF_LOAD_NT = 64,         // complex strided stage: full aligned tiles read with streaming loads
    SF_STORE_NT = 128,       // complex strided stage: full aligned tiles written with streaming stores
    SF_LATE_TWIDDLES = 256,  // the workgroup stages its twiddle table in LDS while its first loads are
                             // in flight (complex strided and FP64 stages, real stages of the kinds
                             // that gain; set on stages beyond the last-level cache)
};

struct StageArgs {
    const void *src;
    void *dst;
    Side side[2];
    const Tile *tiles;
    const void *twiddle;  // N entries e^{-2 pi i m / N} (R2C/C2R: N/2-point table + N-point post table;
                          // R2R: N-point table + e^{-i pi k / 2N}, k < N, in twiddle2; mixed-radix
                          // stages: L = N or M entries here, the chirp e^{-pi i m^2 / N} in twiddle2)
    const void *twiddle2;
    const void *twiddle3;  // mixed-radix stage with Bluestein: DFT_M of the conjugate chirp (M entries)
    int64_t ntiles;
    double scale;
    int32_t N;      // positions per line on the complex side (C2C/COPY); real length for R2C/C2R
    int32_t flags;
    int32_t M;      // mixed-radix stage: Bluestein convolution length (0: direct plan)
    int32_t reserved;
};

}  // namespace pfft
