/*
 * pfft.h -- C ABI of libpfft: the transpose-based parallel multidimensional
 * FFT of Dalcin, Mortensen & Keyes ("Fast parallel multidimensional FFT using
 * advanced MPI", arXiv:1804.09536) for one AMD Instinct MI355X (gfx950).
 *
 * Model.  A d-dimensional array (C row-major, Sec. 3) is decomposed over a
 * Cartesian grid of P "virtual ranks" (Sec. 3.3; ranks are numbered row-major
 * over their grid coordinates).  Each axis is either whole on every rank or
 * split over one grid direction with the balanced block-contiguous rule of
 * Eq. decompose (Sec. 3.1).  One *layout* (alignment) of the array is the
 * concatenation, in rank order, of every rank's local block, each block a
 * C-order array.  All ranks' blocks of one layout live in ONE device buffer.
 *
 * A plan walks a chain of layouts.  With the paper's rule (Secs. 3.2.1, 3.4,
 * 3.5) grid direction i starts on axis i and redistribution t = 1..g moves
 * direction g-t from axis g-t to axis g-t+1 (slab: 1 -> 0; pencil: 2 -> 1 then
 * 1 -> 0; 4-D on a 3-D grid: 3 -> 2 -> 1 -> 0).  The forward transform applies
 * the partial transforms last axis first (Eq. fftn_forward), each on the first
 * layout of the chain where its axis is whole; the backward runs the mirror
 * chain (Eq. fftn_backward).  Every redistribution is a pure permutation
 * (Eq. gt) and is fused into the load of the next partial transform's kernel,
 * so the chain costs one HBM read and one HBM write per partial transform.
 *
 * Layout indices in this API count along the chain: 0 is the input layout
 * (aligned in the last axis for the paper's rule), pfft_num_layouts()-1 the
 * forward output layout.
 *
 * Conventions.  Forward sign -1, backward +1 (Eqs. 1-2).  Normalisation
 * PFFT_NORM_FORWARD is the paper's (1/N_m on each forward partial transform,
 * Eq. multifft), PFFT_NORM_BACKWARD puts it on the backward, PFFT_NORM_NONE
 * nowhere.  Complex data is interleaved (re, im): complex64 for PFFT_F32,
 * complex128 for PFFT_F64.  A PFFT_R2C plan takes a real array (float or
 * double) and produces the half spectrum N_{d-1}/2+1 along the last axis
 * (footnote of Sec. 2); its backward is the matching complex-to-real
 * transform, which ignores the imaginary parts of bins 0 and N/2.  A PFFT_R2R
 * plan (pfft_plan_create_r2r) applies per axis a real-to-real cosine or sine
 * transform of type II forward and its inverse of type III backward, on real
 * data in every layout (the "similar" transforms the method carries, Sec. 1);
 * its per-axis factor is 1/(2 N_m), with which type III undoes type II.
 *
 * Memory.  The library never allocates device memory.  The caller allocates
 * the device state (pfft_device_state_bytes), binds it once
 * (pfft_bind_device_state), and passes input, output and workspace buffers
 * to every call.  All transform calls are asynchronous on the given stream,
 * out-of-place, never write their input, and make no host synchronisation;
 * they may be captured into a HIP graph.  Pointers are device pointers unless
 * stated otherwise; the input, output and workspace buffers of the transform
 * calls and batches must be 16-byte aligned (PFFT_EINVAL otherwise: kernels
 * move 16-byte pieces at offsets the plan checked from the buffers' starts;
 * hipMalloc and torch allocations are), and must not overlap each other
 * (PFFT_EINVAL otherwise).  A plan is immutable after binding;
 * calls on different streams may share a plan if each call has its own output
 * and workspace.
 *
 * Errors.  Every function returns an int status: PFFT_OK (0) or a negative
 * code below.  No function aborts or throws.  pfft_strerror() names a code.
 */
#ifndef PFFT_H
#define PFFT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pfft_plan_s *pfft_plan;

enum { PFFT_C2C = 0, PFFT_R2C = 1, PFFT_R2R = 2 };
/* Real-to-real transform of one axis (forward type; the backward applies its
   inverse):  PFFT_DCT2: Y_k = 2 sum_j x_j cos(pi (2j+1) k / 2N), inverse
   Y_k = x_0 + 2 sum_{j>0} x_j cos(pi j (2k+1) / 2N);  PFFT_DST2:
   Y_k = 2 sum_j x_j sin(pi (2j+1) (k+1) / 2N), inverse
   Y_k = (-1)^k x_{N-1} + 2 sum_{j<N-1} x_j sin(pi (j+1) (2k+1) / 2N). */
enum { PFFT_DCT2 = 0, PFFT_DST2 = 1 };
enum { PFFT_F32 = 0, PFFT_F64 = 1 };
enum { PFFT_NORM_FORWARD = 0, PFFT_NORM_BACKWARD = 1, PFFT_NORM_NONE = 2 };

/* plan flags */
#define PFFT_PATH_FUSED 0u        /* redistribution fused into the next transform's load (default) */
#define PFFT_PATH_UNFUSED 1u      /* standalone redistribution kernel, then transform in place of the new layout */
#define PFFT_PATH_PACK_REALIGN 2u /* traditional method: local transpose, contiguous exchange, realign (Sec. 3.2.1) */
#define PFFT_PATH_MASK 3u
/* Placement of intermediate results on the fused path, chosen separately for the forward
   (bits 3-4) and the backward (bits 5-6) chain; same results, different access patterns.
   GATHER (0): each partial transform leaves its result in the layout where it was computed and
   the next one gathers (redistribution fused into the load).  SCATTER: into the next partial
   transform's layout (fused into the store).  DIRECT: the first result in its own layout, every
   later one straight into the chain's final layout (the middle alignments are never stored and
   consecutive exchanges fuse into one stage).  FINAL: every result into the final layout. */
#define PFFT_PLACE_SCATTER (1u << 3)
#define PFFT_PLACE_DIRECT (2u << 3)
#define PFFT_PLACE_FINAL (3u << 3)
#define PFFT_PLACE_MASK (3u << 3)
#define PFFT_PLACE_BWD_SCATTER (1u << 5)
#define PFFT_PLACE_BWD_DIRECT (2u << 5)
#define PFFT_PLACE_BWD_FINAL (3u << 5)
#define PFFT_PLACE_BWD_MASK (3u << 5)
#define PFFT_LAYOUTS_ONLY 4u      /* plan layouts and redistributions only: no transform kernels are
                                     set up (any lengths), pfft_forward & co. return PFFT_EUNSUPPORTED */
/* The transforms may overwrite a complex input buffer and use it for intermediate results (the
   two-largest-buffers scheme of Sec. 3.5): a c2c plan then needs no workspace at all when its
   chain has an odd number of partial transforms or its first partial transform stays in its own
   layout (it then runs in place), an R2C plan one spectrum-sized buffer instead of two.  `in` and
   `out` must not overlap.  A real input is never written. */
#define PFFT_DESTROY_INPUT (1u << 8)
/* Transposed output (Sec. 3.2.1, Eq. fftw_transposed_out): every rank's block of the last layout of
   the chain (the forward output, the backward input) is stored with its split axes first, in
   grid-direction order, then its whole axes in increasing order; the slab (N0/P, N1, N2) ->
   (N1/P, N0, N2) of the paper, a pencil (N0, N1/P0, N2/P1) -> (N1/P0, N2/P1, N0).  The global index of
   every element and the blocks' extents and starts are unchanged (pfft_local_block reports them per
   axis); pfft_layout_axis_order gives each layout's storage order.  Not for PFFT_R2R plans.  On
   grids of two or more directions the forward placement GATHER with the backward placement
   BWD_SCATTER keeps every stage on the register kernels (others leave a stage whose lines are
   adjacent along different indices on its two sides, which runs one line per tile). */
#define PFFT_TRANSPOSED_OUT (1u << 9)

/* status codes */
#define PFFT_OK 0
#define PFFT_EINVAL (-1)       /* null pointer, bad enum or index */
#define PFFT_ESHAPE (-2)       /* bad global shape */
#define PFFT_EGRID (-3)        /* bad virtual process grid or chain */
#define PFFT_EDTYPE (-4)       /* bad precision / kind */
#define PFFT_EUNSUPPORTED (-5) /* a transform length with no kernel */
#define PFFT_EWORKSPACE (-6)   /* device state not bound, or buffer too small */
#define PFFT_EHIP (-7)         /* a HIP runtime call failed (also forced for every stage launch,
                                  without launching, when the environment variable
                                  PFFT_FAULT_INJECT is "launch": a test of callers' error paths) */
#define PFFT_EINTERNAL (-8)

#define PFFT_MAX_DIMS 8

/*
 * Create a plan (host memory only): the setup phase of Sec. 3.2.2 (index
 * tables built once and reused, the role of the subarray datatypes of
 * Alg. SubArray), the decomposition of Sec. 3.1 (Eq. decompose) over the
 * Cartesian grid of Sec. 3.3, and the chain of alignments of Eqs.
 * pencil0-pencil2 / 4d_fft0-4d_fft3.
 *   ndim, global_shape: the global array, 1 <= ndim <= 8, every extent >= 1.
 *     For PFFT_R2C, global_shape is the real array's shape.
 *   grid_ndim, grid_dims: the virtual process grid, 1 <= grid_ndim < ndim,
 *     every extent >= 1; P = product of grid_dims virtual ranks.  A direction
 *     may be larger than the axis it splits (those ranks get empty blocks).
 *   precision: PFFT_F32 or PFFT_F64.  kind: PFFT_C2C or PFFT_R2C (PFFT_R2R
 *     plans come from pfft_plan_create_r2r).
 *   norm: PFFT_NORM_*.
 *   chain: NULL for the paper's rule, else 2*nsteps ints {dir, new_axis}: step
 *     s moves grid direction dir onto axis new_axis (which must be whole
 *     before the step).  Initially direction i splits axis i.
 *   nsteps: number of chain steps (ignored when chain is NULL).
 *   flags: PFFT_PATH_* (selects how redistributions are executed), optionally
 *     or-ed with one forward and one backward placement (PFFT_PLACE_*,
 *     PFFT_PLACE_BWD_*), PFFT_DESTROY_INPUT, PFFT_TRANSPOSED_OUT and
 *     PFFT_LAYOUTS_ONLY.
 * The chain must leave every axis transformed (each axis whole in some
 * layout).  For PFFT_R2C the last axis must be whole in layout 0.
 * Returns PFFT_OK and *out, or an error (then *out is NULL).
 */
int pfft_plan_create(pfft_plan *out, int ndim, const int64_t *global_shape, int grid_ndim,
                     const int *grid_dims, int precision, int kind, int norm, const int *chain,
                     int nsteps, unsigned flags);

/*
 * Create a real-to-real plan (kind PFFT_R2R): as pfft_plan_create, with
 * kinds[m] (PFFT_DCT2 or PFFT_DST2) the forward transform of axis m.  Every
 * layout holds real values (float for PFFT_F32, double for PFFT_F64).  Axis
 * lengths need a radix plan (2^a <= 4096 or 3*2^a <= 3072), else
 * PFFT_EUNSUPPORTED.  The adjoints are the transposed transforms (type III
 * with its first input element doubled for the cosine, its last for the
 * sine; type II with that output element halved).
 */
int pfft_plan_create_r2r(pfft_plan *out, int ndim, const int64_t *global_shape, int grid_ndim,
                         const int *grid_dims, int precision, const int *kinds, int norm,
                         const int *chain, int nsteps, unsigned flags);

/*
 * Performance knobs of a plan (results never change).  tile_*: 0 default
 * lines per tile, 1 half as many (more workgroups per CU), 2 twice as many
 * (wider coalesced rows, more LDS), 3 twice as many exchanged through the
 * default LDS in two portions (wider rows at the default LDS size), 4 four
 * times as many with 1024-thread workgroups exchanged in two portions
 * (widest rows, one workgroup per CU), 5 chosen by stage (1 for contiguous
 * and real-to-real stages; 3 for strided lines below 1024 points, 4 at 1024,
 * 6 at 1536, 7 from 2048 on; 6 for float real-to-real strided stages: the
 * measured best, and the default of tile_strided); tile_strided 6 / 7: for
 * complex lines of 1024 points and more, 512 / 1024 threads with one line
 * pair (complex64) or line (complex128) per thread and slot, the LDS
 * exchanging slot groups in turn; for strided real-to-real stages of even
 * length, the row-addressed kernel (the reordering folded into the row
 * addresses; 8 / 4 groups of lines per tile, a 16-byte piece of each row per
 * group); lengths without a shape use the
 * default; resident_*: 1 launches only as many
 * workgroups as the device holds at once, each looping over tiles, 0 one
 * workgroup per tile.  *_contig applies to partial transforms along the last
 * axis (tile_contig also to the real-to-complex and complex-to-real stages,
 * which have shapes 0, 1 and 2 = a quarter of the default lines, one line per
 * slot; by rule real-to-complex stages take 2, complex-to-real 1), *_strided
 * to the others.  Strided tiles
 * continue over consecutive short runs of lines (inner extents below the
 * tile width) where the blocks allow it.  xcd_order: see the field.  pfft_plan_set_tuning rebuilds the plan's
 * tables: query pfft_device_state_bytes again and bind again before use.
 * Not a field: stages on buffers beyond the 256 MiB last-level cache stage
 * their twiddle tables while their first loads are in flight, others first;
 * PFFT_LATE_TWIDDLES=1 in the environment at plan creation (or set_tuning)
 * takes the late order on every stage.  Results are bitwise the same.
 */
typedef struct {
    int tile_contig;
    int tile_strided;
    int resident_contig;
    int resident_strided;
    int xcd_order;  /* complex strided stages launched one tile per workgroup: 0 by the plan's rule
                       (unwrapped tiles of stages that store straight into a layout splitting their
                       axis, lines up to 512 points, destinations beyond 256 MiB; and unwrapped tiles
                       whose rows are narrower than 128 bytes, the long lines), 1 always, 2 never.
                       With it, each of the 8 XCDs (workgroup b runs on XCD b mod 8) takes one
                       contiguous range of tiles. */
    int stream_strided; /* complex strided stages, full tiles: 0 ordinary loads and stores, 1 streaming
                           (non-temporal) loads, 2 streaming stores, 3 both, 4 by the plan's rule
                           (the default): where source and destination together exceed 256 MiB
                           (the last-level cache), streaming loads, and streaming stores except on
                           stages with the XCD tile order, whose half-row writes are completed in
                           L2 by the neighbouring tile; otherwise 0 */
    int wide_offsets;   /* 0: 64-bit element offsets only in plans with a buffer of 2^31 elements or
                           more (those kernels use the default tile shapes); 1: in every stage */
    int radix_alt;      /* complex stages of 32-32768 points (powers of two from 32, 3*2^a from 48):
                           bit 0 contiguous stages, bit 1 strided stages take the alternative radix
                           plan (16 points per thread instead of 8, or 8 instead of 16 from 1024
                           points on; 8 instead of 4 times 3, or 4 instead of 8, for 3*2^a), with the
                           mode's default tile width; 0 (the default) none.  Results change only by
                           rounding.  Stages with 64-bit offsets or differently stepping sides, and
                           other lengths, keep their kernels; such stages leave the multi-transform
                           kernel of batches. */
    int stream_contig;  /* complex contiguous stages: 0 ordinary loads and stores, 1 streaming loads,
                           2 streaming stores (of whole destination lines), 3 both, 4 by the plan's
                           rule (the default): both where source and destination together exceed
                           256 MiB (the last-level cache), else streaming loads only */
} pfft_tuning;

int pfft_plan_set_tuning(pfft_plan plan, const pfft_tuning *tuning);
int pfft_plan_get_tuning(pfft_plan plan, pfft_tuning *tuning);

/* Destroy a plan (host memory).  The caller frees the device state. */
int pfft_plan_destroy(pfft_plan plan);

/* Number of layouts in the chain: g+1 for the paper's rule on a g-dimensional
   grid (Secs. 3.2.1, 3.4, 3.5: one alignment per redistribution plus the
   input alignment). */
int pfft_num_layouts(pfft_plan plan, int *n);

/*
 * Rank `rank`'s block in chain layout `layout` (the role of the appendix
 * programs' local-size helper).  shape/start receive ndim extents / global
 * starts; *offset the block's first element in the layout's buffer.  For
 * PFFT_R2C plans layout 0 is described in the real shape when `real` is
 * nonzero, else every layout in the half-spectrum shape.
 */
int pfft_local_block(pfft_plan plan, int layout, int real, int rank, int64_t *shape, int64_t *start,
                     int64_t *offset);

/* Storage order of every block of chain layout `layout`: order[k] (ndim ints) is the axis at
   position k of the block's C-order index (the identity except for the last layout of a
   PFFT_TRANSPOSED_OUT plan). */
int pfft_layout_axis_order(pfft_plan plan, int layout, int *order);

/* Bytes of a layout's buffer (real = as above): the sum over the ranks of
   the local block sizes of Eq. decompose (Sec. 3.1), times the element size. */
int pfft_buffer_bytes(pfft_plan plan, int layout, int real, size_t *bytes);

/* Bytes of device state (tile and index tables, twiddles) the plan needs. */
int pfft_device_state_bytes(pfft_plan plan, size_t *bytes);

/*
 * Upload the plan's tables into caller-allocated device memory `dev`
 * (>= pfft_device_state_bytes, 256-byte aligned) on `stream`, then wait for
 * the copy.  Must precede every call below.  The memory must outlive the
 * plan's use; binding again (e.g. to another buffer) is allowed.
 */
int pfft_bind_device_state(pfft_plan plan, void *dev, hipStream_t stream);

/* Workspace bytes needed by pfft_forward/backward/adjoint_* (256-aligned;
   0 when the transforms need none: `work` may then be NULL). */
int pfft_workspace_bytes(pfft_plan plan, size_t *bytes);

/*
 * Global redistribution (Eq. gt) between chain layouts layout_from and
 * layout_to = layout_from +/- 1 (they differ by exactly one exchange): for
 * every global index g, out[to(g)] = in[from(g)], bit-exact.  Elements are
 * the plan's complex type (for R2C plans: the half-spectrum layouts).
 */
int pfft_redistribute(pfft_plan plan, int layout_from, int layout_to, const void *in, void *out,
                      hipStream_t stream);

/*
 * Forward transform (Eq. fftn_forward through the chain's redistributions,
 * e.g. Eqs. pencil0-pencil2; Eq. multifft with the norm's factors): `in` in
 * layout 0 (real for R2C), `out` in the last layout (half spectrum for R2C).
 * `work`: pfft_workspace_bytes bytes.  `in` is left unchanged unless the
 * plan has PFFT_DESTROY_INPUT.  Errors: PFFT_EINVAL (null, misaligned or
 * overlapping buffers), PFFT_EWORKSPACE (device state not bound),
 * PFFT_EUNSUPPORTED (layouts-only plan), PFFT_EHIP (a launch failed).
 */
int pfft_forward(pfft_plan plan, const void *in, void *out, void *work, hipStream_t stream);

/* Backward transform (Eq. fftn_backward, the mirror chain, sign +1):
   `in` in the last layout, `out` in layout 0.  Errors as pfft_forward. */
int pfft_backward(pfft_plan plan, const void *in, void *out, void *work, hipStream_t stream);

/*
 * Adjoint of pfft_forward under the real inner product Re<a,b> (the gradient
 * map for automatic differentiation): reversed chain, inverse
 * redistributions, sign +1 and the forward's per-axis factors; for R2C the
 * result is Re(F^H S^T z), i.e. a complex-to-real with interior bins halved.
 * `in` in the last layout, `out` in layout 0.
 */
int pfft_adjoint_forward(pfft_plan plan, const void *in, void *out, void *work, hipStream_t stream);

/* Adjoint of pfft_backward: forward chain, sign -1, the backward's factors;
 * for R2C an r2c with interior bins doubled. */
int pfft_adjoint_backward(pfft_plan plan, const void *in, void *out, void *work, hipStream_t stream);

/*
 * Batches: many plans (any shapes and grids, one precision) executed
 * together.  Launch k of every member that runs the same stage kernel shape
 * becomes one launch over all their tiles (complex stages of the default
 * radix plan with 32-bit offsets, and the real-to-complex / complex-to-real
 * stages; other stages -- real-to-real, copies, XS, 64-bit offsets, the
 * alternative radix plan, the long-line shapes -- are launched per member
 * inside the batch), so a batch of n transforms costs
 * about as many kernel launches as one transform of each distinct shape;
 * execution is asynchronous, allocates nothing and can be captured into a
 * HIP graph.  The batch copies what it needs from its plans at creation
 * (member plans may be changed or destroyed afterwards).
 *
 * Buffers are bound once (pfft_batch_bind), not passed to every execution:
 * the grouped launches read every member's kernel arguments from device
 * memory, so binding writes them once and an execution (or a captured graph
 * of it) only launches.  One input, one output and one workspace buffer for
 * the whole batch, each holding every member's region at the offsets
 * pfft_batch_member_offsets returns (256-byte aligned); a member's input
 * region is its layout 0, its output region its last layout.  Direction 0
 * runs every member's forward transform (input -> output), direction 1 every
 * backward transform (output -> input, overwriting the input region).
 */
typedef struct pfft_batch_s *pfft_batch;

int pfft_batch_create(pfft_batch *out, int nplans, const pfft_plan *plans);
int pfft_batch_destroy(pfft_batch batch);
int pfft_batch_buffer_bytes(pfft_batch batch, size_t *in_bytes, size_t *out_bytes, size_t *work_bytes);
int pfft_batch_member_offsets(pfft_batch batch, int member, size_t *in_offset, size_t *out_offset);
int pfft_batch_device_state_bytes(pfft_batch batch, size_t *bytes);
/* Upload tables and kernel arguments for these buffers (device pointers, the
 * state 256-byte aligned); waits for the upload.  Bind again to use other
 * buffers. */
int pfft_batch_bind(pfft_batch batch, void *state, void *in, void *out, void *work, hipStream_t stream);
int pfft_batch_execute(pfft_batch batch, int direction, hipStream_t stream);

/*
 * Host-side self-check of a plan (no device needed): emulates the address
 * arithmetic of every kernel launch the plan can make and verifies that each
 * access stays inside its rank block and buffer and that every destination
 * element is written exactly once.  Returns PFFT_OK or PFFT_EINTERNAL (see
 * pfft_last_error).  Cost is proportional to the array size.
 */
int pfft_validate_plan(pfft_plan plan);

/*
 * Per-launch timing.  While enabled, every stage kernel of later calls on
 * this plan is launched with hipExtLaunchKernelGGL, which stamps the kernel's
 * start and end into two HIP events of the plan (no event packets between
 * kernels, no host synchronisation).  pfft_profile_read waits for the logged launches,
 * fills up to max_entries records (oldest first), sets *n to the number
 * logged, and clears the log.  kind: 0 complex transform, 1 redistribution
 * copy, 2 real-to-complex, 3 complex-to-real, 4 real-to-real; direction: 0 forward, 1 backward,
 * 2 adjoint of forward, 3 adjoint of backward, 4 pfft_redistribute; bytes: the
 * launch's algorithmic traffic (source read once + destination written once).
 * Not for use while a call on the plan is being captured into a graph, nor from
 * several host threads at once (the log is the plan's own).
 */
typedef struct {
    int kind;
    int axis;
    int contig;
    int length;
    int direction;
    float ms;
    double bytes;
} pfft_profile_entry;

int pfft_set_profiling(pfft_plan plan, int enable);
int pfft_profile_read(pfft_plan plan, int max_entries, pfft_profile_entry *entries, int *n);

/*
 * Weighted spectral energy, the quadratic loss of the differentiation
 * workload (not part of the paper's method: it exercises the adjoint
 * transforms, with w = |k|^2 on the forward output):
 *   loss[0] = sum_i w_i |u_i|^2  over n complex elements u (complex64 for
 *   PFFT_F32, complex128 for PFFT_F64) with real weights w of the same
 *   precision; loss is one real of that precision on the device.
 * Per-workgroup FP64 partial sums go to `partials` (caller scratch of
 * PFFT_ENERGY_PARTIALS doubles), then are added in a fixed order, so the
 * result does not depend on scheduling.  Asynchronous on `stream`; buffers
 * naturally aligned for their element types.  n = 0 gives 0.
 */
#define PFFT_ENERGY_PARTIALS 1024
int pfft_weighted_energy(int precision, int64_t n, const void *u, const void *w, double *partials, void *loss,
                         hipStream_t stream);

/*
 * pfft_weighted_energy for callers that cannot allocate device memory or
 * provide scratch (code under HIP graph capture, tight training or serving
 * loops): the same kernels and result, with the partial sums in the library's
 * own static device scratch of PFFT_ENERGY_PARTIALS doubles (8 KiB per
 * device, held until the process ends; every n fits it: the kernels use at
 * most that many partial sums).  Allocates nothing and calls no allocating
 * routine; the scratch's device address is looked up once per device on its
 * first call (with the current device set to the device of `stream` and the
 * buffers).  All calls on one device share the scratch: calls that overlap
 * in time on one device (e.g. on two streams) race and give wrong losses;
 * calls ordered on one stream are safe.  Arguments and errors as
 * pfft_weighted_energy (PFFT_EHIP if the scratch cannot be looked up).
 */
int pfft_weighted_energy_noalloc(int precision, int64_t n, const void *u, const void *w, void *loss,
                                 hipStream_t stream);

/*
 * Its gradient under torch's convention for complex inputs:
 *   grad_i = 2 g w_i u_i,  g = *g_dev (one real of the precision, on the
 * device: the incoming gradient of the loss).  grad may not overlap u.
 */
int pfft_weighted_energy_grad(int precision, int64_t n, const void *u, const void *w, const void *g_dev,
                              void *grad, hipStream_t stream);

/* Human-readable name of a status code (static string). */
const char *pfft_strerror(int status);

/* Last error detail for this thread (static buffer), e.g. the HIP message. */
const char *pfft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PFFT_H */
