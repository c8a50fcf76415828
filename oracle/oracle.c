/*
 * oracle.c -- plain, slow CPU reference (FP64) for the transpose-based
 * parallel multidimensional FFT of Dalcin, Mortensen & Keyes,
 * "Fast parallel multidimensional FFT using advanced MPI" (arXiv:1804.09536).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only tests, the smoke check and the bench's CPU-baseline leg
 * do.  It shares no code, header, table or helper with the HIP library.
 *
 * Conventions (all from the paper):
 *   - arrays are C row-major (Sec. 3, notation paragraph);
 *   - a block-contiguous decomposition of N over M parts gives part p the
 *     length n_p = q + [r > p] and start s_p = q*p + min(r, p), q = N div M,
 *     r = N mod M (Sec. 3.1, Eq. decompose);
 *   - virtual ranks of a Cartesian grid are numbered row-major over their grid
 *     coordinates (Sec. 3.3, the 3x4 example where (2,3) is rank 11);
 *   - the forward DFT carries e^{-2 pi i jk/N}, the backward e^{+...}
 *     (Sec. 2, Eqs. 1-2 and Eq. multifft).
 *
 * Memory model (not in the paper, which gives each process its own array):
 * the local blocks of all virtual ranks of one alignment are C-order arrays
 * concatenated in rank order in one buffer.  A "layout" is
 *   ndim, global shape[ndim], ngrid, grid[ngrid], axis_dir[ndim]
 * where axis_dir[m] is the grid direction that distributes axis m, or -1 if
 * axis m is whole (aligned) on every rank.
 *
 * Complex numbers are interleaved (re, im) doubles, i.e. numpy complex128.
 *
 * Every routine is written for clarity, not speed: lines are copied out,
 * transformed and copied back; owners are found by search.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OMAXD 8

/* ---------------------------------------------------------------- layout -- */

/* Eq. decompose (Sec. 3.1): length and start of part p of N split in M. */
void oracle_decompose(int64_t N, int64_t M, int64_t p, int64_t *n, int64_t *s)
{
    int64_t q = N / M;
    int64_t r = N % M;
    *n = q + (r > p ? 1 : 0);
    *s = q * p + (r < p ? r : p);
}

/* Number of virtual ranks of a grid. */
static int64_t grid_size(int ngrid, const int64_t *grid)
{
    int64_t P = 1;
    for (int i = 0; i < ngrid; i++) P *= grid[i];
    return P;
}

/* Row-major grid coordinates of rank r (Sec. 3.3). */
static void rank_coords(int64_t r, int ngrid, const int64_t *grid, int64_t *c)
{
    for (int i = ngrid - 1; i >= 0; i--) {
        c[i] = r % grid[i];
        r /= grid[i];
    }
}

/* Local shape and global start of rank r's block; returns its element count. */
int64_t oracle_block(int ndim, const int64_t *shape, int ngrid, const int64_t *grid,
                     const int *axis_dir, int64_t rank, int64_t *lshape, int64_t *lstart)
{
    int64_t c[OMAXD];
    rank_coords(rank, ngrid, grid, c);
    int64_t count = 1;
    for (int m = 0; m < ndim; m++) {
        int dir = axis_dir[m];
        if (dir < 0) {
            lshape[m] = shape[m];
            lstart[m] = 0;
        } else {
            oracle_decompose(shape[m], grid[dir], c[dir], &lshape[m], &lstart[m]);
        }
        count *= lshape[m];
    }
    return count;
}

/* Element offset of every rank's block: prefix sums of block sizes in rank
 * order.  offsets must hold P+1 entries; offsets[P] is the total size. */
void oracle_rank_offsets(int ndim, const int64_t *shape, int ngrid, const int64_t *grid,
                         const int *axis_dir, int64_t *offsets)
{
    int64_t P = grid_size(ngrid, grid);
    int64_t lshape[OMAXD], lstart[OMAXD];
    offsets[0] = 0;
    for (int64_t r = 0; r < P; r++)
        offsets[r + 1] = offsets[r] + oracle_block(ndim, shape, ngrid, grid, axis_dir, r, lshape, lstart);
}

/* Per-axis owner table: for every global index g of axis m, the grid
 * coordinate (along the direction distributing m) that holds it and the local
 * index there.  Found by searching the parts, not by inverting the formula. */
static void owner_table(int64_t N, int64_t M, int64_t *own, int64_t *loc)
{
    for (int64_t g = 0; g < N; g++) {
        own[g] = -1;
        for (int64_t p = 0; p < M; p++) {
            int64_t n, s;
            oracle_decompose(N, M, p, &n, &s);
            if (g >= s && g < s + n) {
                own[g] = p;
                loc[g] = g - s;
                break;
            }
        }
    }
}

typedef struct {
    int ndim, ngrid;
    int64_t shape[OMAXD], grid[OMAXD];
    int axis_dir[OMAXD];
    int64_t *own[OMAXD], *loc[OMAXD];
    int64_t *offsets; /* P+1 */
    int64_t *lshape;  /* P*ndim */
} olayout;

static void olayout_init(olayout *L, int ndim, const int64_t *shape, int ngrid, const int64_t *grid,
                         const int *axis_dir)
{
    L->ndim = ndim;
    L->ngrid = ngrid;
    for (int m = 0; m < ndim; m++) {
        L->shape[m] = shape[m];
        L->axis_dir[m] = axis_dir[m];
    }
    for (int i = 0; i < ngrid; i++) L->grid[i] = grid[i];
    int64_t P = grid_size(ngrid, grid);
    L->offsets = (int64_t *)malloc((size_t)(P + 1) * sizeof(int64_t));
    L->lshape = (int64_t *)malloc((size_t)(P * ndim + 1) * sizeof(int64_t));
    oracle_rank_offsets(ndim, shape, ngrid, grid, axis_dir, L->offsets);
    int64_t lstart[OMAXD];
    for (int64_t r = 0; r < P; r++)
        oracle_block(ndim, shape, ngrid, grid, axis_dir, r, L->lshape + r * ndim, lstart);
    for (int m = 0; m < ndim; m++) {
        L->own[m] = (int64_t *)malloc((size_t)(shape[m] + 1) * sizeof(int64_t));
        L->loc[m] = (int64_t *)malloc((size_t)(shape[m] + 1) * sizeof(int64_t));
        if (axis_dir[m] < 0) {
            for (int64_t g = 0; g < shape[m]; g++) {
                L->own[m][g] = 0;
                L->loc[m][g] = g;
            }
        } else {
            owner_table(shape[m], grid[axis_dir[m]], L->own[m], L->loc[m]);
        }
    }
}

static void olayout_free(olayout *L)
{
    free(L->offsets);
    free(L->lshape);
    for (int m = 0; m < L->ndim; m++) {
        free(L->own[m]);
        free(L->loc[m]);
    }
}

/* Position in the layout's buffer of the element with global index g[]. */
static int64_t olayout_offset(const olayout *L, const int64_t *g)
{
    int64_t c[OMAXD];
    for (int i = 0; i < L->ngrid; i++) c[i] = 0;
    for (int m = 0; m < L->ndim; m++)
        if (L->axis_dir[m] >= 0) c[L->axis_dir[m]] = L->own[m][g[m]];
    int64_t r = 0;
    for (int i = 0; i < L->ngrid; i++) r = r * L->grid[i] + c[i];
    const int64_t *ls = L->lshape + r * L->ndim;
    int64_t off = 0;
    for (int m = 0; m < L->ndim; m++) off = off * ls[m] + L->loc[m][g[m]];
    return L->offsets[r] + off;
}

/* ------------------------------------------------------ redistribution -- */

/*
 * Global-view redistribution (Eq. general_gt / Eq. gt): every element keeps its
 * global index; out[layout_B(g)] = in[layout_A(g)] for all g.  esize is the
 * element size in bytes.  Both layouts must describe the same global shape.
 */
void oracle_redistribute_global(int ndim, const int64_t *shape, int ngrid, const int64_t *grid,
                                const int *dirA, const int *dirB, const void *in, void *out,
                                int64_t esize)
{
    olayout A, B;
    olayout_init(&A, ndim, shape, ngrid, grid, dirA);
    olayout_init(&B, ndim, shape, ngrid, grid, dirB);
    int64_t total = 1;
    for (int m = 0; m < ndim; m++) total *= shape[m];
    const char *src = (const char *)in;
    char *dst = (char *)out;
#pragma omp parallel for schedule(static)
    for (int64_t flat = 0; flat < total; flat++) {
        int64_t g[OMAXD], t = flat;
        for (int m = ndim - 1; m >= 0; m--) {
            g[m] = t % shape[m];
            t /= shape[m];
        }
        int64_t oa = olayout_offset(&A, g), ob = olayout_offset(&B, g);
        memcpy(dst + ob * esize, src + oa * esize, (size_t)esize);
    }
    olayout_free(&A);
    olayout_free(&B);
}

/*
 * Exchange emulated pair by pair (Alg. SubArray + Alg. Exchange, Sec. 3.2.2).
 * Within every one-dimensional subgroup along grid direction `dir` of size M,
 * rank p's array A (aligned in axis v, axis w split by dir) is cut along v into
 * M subarrays S_A[q]; rank q's array B (aligned in w, axis v split by dir) is
 * cut along w into S_B[p].  The generalized all-to-all sends S_A[q] of A_p to
 * S_B[p] of B_q; the k-th element (C order) of one goes to the k-th of the other.
 * Layout A: axis v whole, axis w distributed by dir.  Layout B: the reverse.
 * Returns 0, or -1 if the two layouts are not related by this exchange.
 */
int oracle_redistribute_pairs(int ndim, const int64_t *shape, int ngrid, const int64_t *grid,
                              const int *dirA, const int *dirB, int dir, int v, int w,
                              const void *in, void *out, int64_t esize)
{
    if (dirA[v] != -1 || dirA[w] != dir || dirB[w] != -1 || dirB[v] != dir) return -1;
    for (int m = 0; m < ndim; m++)
        if (m != v && m != w && dirA[m] != dirB[m]) return -1;
    int64_t offA[4097], offB[4097];
    int64_t P = grid_size(ngrid, grid);
    if (P > 4096) return -1;
    oracle_rank_offsets(ndim, shape, ngrid, grid, dirA, offA);
    oracle_rank_offsets(ndim, shape, ngrid, grid, dirB, offB);
    int64_t M = grid[dir];
    int64_t stride = 1; /* rank-number distance between neighbours along dir */
    for (int i = dir + 1; i < ngrid; i++) stride *= grid[i];
    const char *src = (const char *)in;
    char *dst = (char *)out;
    for (int64_t ra = 0; ra < P; ra++) {
        int64_t c[OMAXD];
        rank_coords(ra, ngrid, grid, c);
        int64_t p = c[dir];
        int64_t sizesA[OMAXD], startA[OMAXD];
        oracle_block(ndim, shape, ngrid, grid, dirA, ra, sizesA, startA);
        for (int64_t q = 0; q < M; q++) {
            int64_t rb = ra + (q - p) * stride; /* rank q of the same subgroup */
            int64_t sizesB[OMAXD], startB[OMAXD];
            oracle_block(ndim, shape, ngrid, grid, dirB, rb, sizesB, startB);
            /* S_A[q]: sizesA with axis v cut to q's part.  S_B[p]: sizesB with
             * axis w cut to p's part. */
            int64_t subA[OMAXD], stA[OMAXD], subB[OMAXD], stB[OMAXD];
            for (int m = 0; m < ndim; m++) {
                subA[m] = sizesA[m];
                stA[m] = 0;
                subB[m] = sizesB[m];
                stB[m] = 0;
            }
            oracle_decompose(sizesA[v], M, q, &subA[v], &stA[v]);
            oracle_decompose(sizesB[w], M, p, &subB[w], &stB[w]);
            int64_t count = 1;
            for (int m = 0; m < ndim; m++) {
                if (subA[m] != subB[m]) return -1; /* type signatures must match */
                count *= subA[m];
            }
            for (int64_t k = 0; k < count; k++) {
                int64_t idx[OMAXD], t = k;
                for (int m = ndim - 1; m >= 0; m--) {
                    idx[m] = t % subA[m];
                    t /= subA[m];
                }
                int64_t a = 0, b = 0;
                for (int m = 0; m < ndim; m++) {
                    a = a * sizesA[m] + (stA[m] + idx[m]);
                    b = b * sizesB[m] + (stB[m] + idx[m]);
                }
                memcpy(dst + (offB[rb] + b) * esize, src + (offA[ra] + a) * esize, (size_t)esize);
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------- 1-D DFT -- */

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* e^{sign * 2 pi i m / n} with the index reduced exactly in integers. */
static void twiddle(int64_t m, int64_t n, int sign, double *re, double *im)
{
    m %= n;
    double a = 2.0 * M_PI * (double)m / (double)n;
    *re = cos(a);
    *im = (double)sign * sin(a);
}

/* Smallest prime factor of n >= 2 (n itself when n is prime). */
static int64_t smallest_factor(int64_t n)
{
    for (int64_t f = 2; f * f <= n; f++)
        if (n % f == 0) return f;
    return n;
}

/*
 * Mixed-radix decimation in time (the Cooley-Tukey factorisation of Eq. 1):
 * with n = p * m, p the smallest prime factor of n, the p subsequences
 * x_{r + p j} (j < m) are transformed with length m into Y_r, and then
 *   y_k = sum_{r<p} e^{sign 2 pi i r k / n} Y_r[k mod m],  k < n.
 * Prime lengths are the direct sum of Eq. 1.  x is read with a stride of
 * `xs` complex elements; y receives n contiguous results.  tw holds
 * e^{sign 2 pi i t / ntw} for t < ntw (n divides ntw), so the factor of
 * exponent r k / n is tw[(r k mod n) * (ntw / n)]; work holds n complex.
 */
static void dft_mixed(const double *x, int64_t xs, double *y, int64_t n, const double *tw, int64_t ntw,
                      double *work)
{
    const int64_t step = ntw / n;
    const int64_t p = n > 1 ? smallest_factor(n) : 1;
    if (p == n) {
        for (int64_t k = 0; k < n; k++) {
            double sr = 0.0, si = 0.0;
            for (int64_t j = 0; j < n; j++) {
                const double *w = tw + 2 * (((j * k) % n) * step);
                const double *u = x + 2 * j * xs;
                sr += u[0] * w[0] - u[1] * w[1];
                si += u[0] * w[1] + u[1] * w[0];
            }
            y[2 * k] = sr;
            y[2 * k + 1] = si;
        }
        return;
    }
    const int64_t m = n / p;
    /* Y_r into y[r m .. (r+1) m) (each sub-transform uses work only before
       this level's combination below) */
    for (int64_t r = 0; r < p; r++) dft_mixed(x + 2 * r * xs, xs * p, y + 2 * r * m, m, tw, ntw, work);
    for (int64_t k = 0; k < n; k++) {
        double sr = 0.0, si = 0.0;
        for (int64_t r = 0; r < p; r++) {
            const double *w = tw + 2 * (((r * k) % n) * step);
            const double *u = y + 2 * (r * m + k % m);
            sr += u[0] * w[0] - u[1] * w[1];
            si += u[0] * w[1] + u[1] * w[0];
        }
        work[2 * k] = sr;
        work[2 * k + 1] = si;
    }
    memcpy(y, work, (size_t)(2 * n) * sizeof(double));
}

/*
 * Unnormalised 1-D DFT of x (n complex, interleaved), result into y:
 *   y_k = sum_j x_j e^{sign 2 pi i jk/n}.
 * Powers of two use an iterative radix-2 decimation-in-time FFT (bit-reversal
 * permutation, then log2 n butterfly passes); other composite lengths the
 * mixed-radix recursion above; primes the direct sum.
 */
static void dft1(const double *x, double *y, int64_t n, int sign)
{
    if (is_pow2(n)) {
        int bits = 0;
        while (((int64_t)1 << bits) < n) bits++;
        for (int64_t j = 0; j < n; j++) {
            int64_t r = 0;
            for (int b = 0; b < bits; b++)
                if (j & ((int64_t)1 << b)) r |= (int64_t)1 << (bits - 1 - b);
            y[2 * r] = x[2 * j];
            y[2 * r + 1] = x[2 * j + 1];
        }
        for (int64_t len = 2; len <= n; len <<= 1) {
            int64_t half = len / 2;
            for (int64_t start = 0; start < n; start += len) {
                for (int64_t k = 0; k < half; k++) {
                    double wr, wi;
                    twiddle(k, len, sign, &wr, &wi);
                    double *a = y + 2 * (start + k);
                    double *b = y + 2 * (start + k + half);
                    double tr = wr * b[0] - wi * b[1];
                    double ti = wr * b[1] + wi * b[0];
                    b[0] = a[0] - tr;
                    b[1] = a[1] - ti;
                    a[0] = a[0] + tr;
                    a[1] = a[1] + ti;
                }
            }
        }
    } else {
        double *tw = (double *)malloc((size_t)(2 * n) * sizeof(double));
        double *work = (double *)malloc((size_t)(2 * n) * sizeof(double));
        for (int64_t t = 0; t < n; t++) twiddle(t, n, sign, &tw[2 * t], &tw[2 * t + 1]);
        dft_mixed(x, 1, y, n, tw, n, work);
        free(tw);
        free(work);
    }
}

/* Exposed for tests: one line, unnormalised. */
void oracle_dft1(const double *x, double *y, int64_t n, int sign) { dft1(x, y, n, sign); }

/*
 * Partial transform F_a (Sec. 2, the equation defining the partial transform):
 * a 1-D DFT of every line along axis a of every rank block, in place, with the
 * result multiplied by `scale`.  Axis a must be whole in this layout.
 * Returns 0, or -1 if axis a is distributed.
 */
int oracle_fft_axis(int ndim, const int64_t *shape, int ngrid, const int64_t *grid,
                    const int *axis_dir, double *data, int a, int sign, double scale)
{
    if (axis_dir[a] >= 0) return -1;
    int64_t P = grid_size(ngrid, grid);
    int64_t *offs = (int64_t *)malloc((size_t)(P + 1) * sizeof(int64_t));
    oracle_rank_offsets(ndim, shape, ngrid, grid, axis_dir, offs);
    int64_t n = shape[a];
    for (int64_t r = 0; r < P; r++) {
        int64_t ls[OMAXD], st[OMAXD];
        int64_t count = oracle_block(ndim, shape, ngrid, grid, axis_dir, r, ls, st);
        if (count == 0) continue;
        int64_t inner = 1;
        for (int m = a + 1; m < ndim; m++) inner *= ls[m];
        int64_t outer = count / (inner * n);
        double *blk = data + 2 * offs[r];
#pragma omp parallel
        {
            double *x = (double *)malloc((size_t)(2 * n) * sizeof(double));
            double *y = (double *)malloc((size_t)(2 * n) * sizeof(double));
#pragma omp for schedule(static)
            for (int64_t line = 0; line < outer * inner; line++) {
                int64_t o = line / inner, i = line % inner;
                double *base = blk + 2 * (o * n * inner + i);
                for (int64_t j = 0; j < n; j++) {
                    x[2 * j] = base[2 * j * inner];
                    x[2 * j + 1] = base[2 * j * inner + 1];
                }
                dft1(x, y, n, sign);
                for (int64_t k = 0; k < n; k++) {
                    base[2 * k * inner] = y[2 * k] * scale;
                    base[2 * k * inner + 1] = y[2 * k + 1] * scale;
                }
            }
            free(x);
            free(y);
        }
    }
    free(offs);
    return 0;
}

/*
 * Real-to-complex transform along the last axis (footnote of Sec. 2: the
 * half index set k = 0..N/2 suffices for real input).  Input: real layout with
 * last axis N; output: complex layout with last axis N/2+1, same grid and
 * axis_dir (the last axis must be whole).  Each output line is the first
 * N/2+1 bins of the full complex DFT of the real line, times `scale`.
 */
int oracle_r2c_last(int ndim, const int64_t *shape_real, int ngrid, const int64_t *grid,
                    const int *axis_dir, const double *in, double *out, double scale)
{
    int a = ndim - 1;
    if (axis_dir[a] >= 0) return -1;
    int64_t n = shape_real[a], h = n / 2 + 1;
    int64_t shape_c[OMAXD];
    for (int m = 0; m < ndim; m++) shape_c[m] = shape_real[m];
    shape_c[a] = h;
    (void)shape_c;
    (void)ngrid;
    (void)grid;
    /* The last axis is whole in both layouts and every other axis is split the
     * same way, so both buffers hold the same sequence of lines (rank order,
     * then C order inside each block): line l of one is line l of the other. */
    int64_t total = 1;
    for (int m = 0; m < ndim; m++) total *= shape_real[m];
    int64_t lines = total / n;
#pragma omp parallel
    {
        double *x = (double *)malloc((size_t)(2 * n) * sizeof(double));
        double *y = (double *)malloc((size_t)(2 * n) * sizeof(double));
#pragma omp for schedule(static)
        for (int64_t l = 0; l < lines; l++) {
            for (int64_t j = 0; j < n; j++) {
                x[2 * j] = in[l * n + j];
                x[2 * j + 1] = 0.0;
            }
            dft1(x, y, n, -1);
            for (int64_t k = 0; k < h; k++) {
                out[2 * (l * h + k)] = y[2 * k] * scale;
                out[2 * (l * h + k) + 1] = y[2 * k + 1] * scale;
            }
        }
        free(x);
        free(y);
    }
    return 0;
}

/*
 * Complex-to-real along the last axis: the inverse of the above.  The N/2+1
 * stored bins are extended to N by Hermitian symmetry (bin N-k = conj of bin
 * k for 0 < k < N-k), transformed with sign +, and the real part kept (which
 * ignores the imaginary parts of bin 0 and, for even N, bin N/2).  If
 * `halve_interior` is set, bins 0 < k < N-k are first halved: that turns the
 * operation into Re(sum_{k<=N/2} z_k e^{+2 pi i jk/N}), the adjoint of the
 * truncated real transform.  Result times `scale`.
 */
int oracle_c2r_last(int ndim, const int64_t *shape_real, int ngrid, const int64_t *grid,
                    const int *axis_dir, const double *in, double *out, double scale,
                    int halve_interior)
{
    int a = ndim - 1;
    (void)ngrid;
    (void)grid;
    if (axis_dir[a] >= 0) return -1;
    int64_t n = shape_real[a], h = n / 2 + 1;
    int64_t total = 1;
    for (int m = 0; m < ndim; m++) total *= shape_real[m];
    int64_t lines = total / n;
#pragma omp parallel
    {
        double *x = (double *)malloc((size_t)(2 * n) * sizeof(double));
        double *y = (double *)malloc((size_t)(2 * n) * sizeof(double));
#pragma omp for schedule(static)
        for (int64_t l = 0; l < lines; l++) {
            for (int64_t k = 0; k < n; k++) {
                x[2 * k] = 0.0;
                x[2 * k + 1] = 0.0;
            }
            for (int64_t k = 0; k < h && k < n; k++) {
                double f = (halve_interior && k > 0 && k < n - k) ? 0.5 : 1.0;
                x[2 * k] = in[2 * (l * h + k)] * f;
                x[2 * k + 1] = in[2 * (l * h + k) + 1] * f;
            }
            for (int64_t k = 1; k < n - k; k++) {
                x[2 * (n - k)] = x[2 * k];
                x[2 * (n - k) + 1] = -x[2 * k + 1];
            }
            dft1(x, y, n, +1);
            for (int64_t j = 0; j < n; j++) out[l * n + j] = y[2 * j] * scale;
        }
        free(x);
        free(y);
    }
    return 0;
}

/* ---------------------------------------------------- brute force (tiny) -- */

/*
 * Full d-dimensional DFT straight from Eq. multifft on the global array
 * (C order), no FFT, no separation into partial transforms: every output
 * element is the full sum over every input element with twiddle exponent
 * sum_m k_m j_m / N_m (each term reduced exactly), times `scale`.
 * O(total^2): tiny arrays only.
 */
void oracle_bruteforce_dft(int ndim, const int64_t *shape, const double *in, double *out, int sign,
                           double scale)
{
    int64_t total = 1;
    for (int m = 0; m < ndim; m++) total *= shape[m];
#pragma omp parallel for schedule(static)
    for (int64_t kf = 0; kf < total; kf++) {
        int64_t k[OMAXD], t = kf;
        for (int m = ndim - 1; m >= 0; m--) {
            k[m] = t % shape[m];
            t /= shape[m];
        }
        double sr = 0.0, si = 0.0;
        for (int64_t jf = 0; jf < total; jf++) {
            int64_t j[OMAXD], u = jf;
            for (int m = ndim - 1; m >= 0; m--) {
                j[m] = u % shape[m];
                u /= shape[m];
            }
            /* phase = sum_m (k_m j_m mod N_m)/N_m, as a fraction of a turn */
            double phase = 0.0;
            for (int m = 0; m < ndim; m++) phase += (double)((k[m] * j[m]) % shape[m]) / (double)shape[m];
            double ang = (double)sign * 2.0 * M_PI * phase;
            double wr = cos(ang), wi = sin(ang);
            sr += in[2 * jf] * wr - in[2 * jf + 1] * wi;
            si += in[2 * jf] * wi + in[2 * jf + 1] * wr;
        }
        out[2 * kf] = sr * scale;
        out[2 * kf + 1] = si * scale;
    }
}

/*
 * Selected bins of the d-dimensional DFT, each evaluated as the full sum of
 * Eq. multifft over every input element (no FFT): for bin k,
 *   out_k = scale * sum_j in_j * prod_m e^{sign 2 pi i (k_m j_m mod N_m) / N_m}.
 * ks holds nk multi-indices (ndim each).  The per-axis factors are tabulated
 * once per bin; the sum runs in parallel over the leading axis.  O(total) per
 * bin, so it can check single outputs of arrays far too large to brute-force.
 */
void oracle_dft_bins(int ndim, const int64_t *shape, const double *in, int64_t nk, const int64_t *ks,
                     double *out, int sign, double scale)
{
    int64_t total = 1;
    for (int m = 0; m < ndim; m++) total *= shape[m];
    int64_t inner = total / shape[0];
    double *tab[OMAXD];
    for (int m = 0; m < ndim; m++) tab[m] = (double *)malloc((size_t)(2 * shape[m]) * sizeof(double));
    for (int64_t b = 0; b < nk; b++) {
        const int64_t *k = ks + b * ndim;
        for (int m = 0; m < ndim; m++)
            for (int64_t j = 0; j < shape[m]; j++) twiddle((k[m] * j) % shape[m], shape[m], sign, &tab[m][2 * j], &tab[m][2 * j + 1]);
        double sr = 0.0, si = 0.0;
#pragma omp parallel for reduction(+ : sr, si) schedule(static)
        for (int64_t j0 = 0; j0 < shape[0]; j0++) {
            double ar = 0.0, ai = 0.0;
            for (int64_t r = 0; r < inner; r++) {
                /* product of the factors of axes 1..d-1 */
                int64_t t = r;
                double wr = 1.0, wi = 0.0;
                for (int m = ndim - 1; m >= 1; m--) {
                    int64_t jm = t % shape[m];
                    t /= shape[m];
                    double xr = tab[m][2 * jm], xi = tab[m][2 * jm + 1];
                    double nr = wr * xr - wi * xi;
                    wi = wr * xi + wi * xr;
                    wr = nr;
                }
                const double *u = in + 2 * (j0 * inner + r);
                ar += u[0] * wr - u[1] * wi;
                ai += u[0] * wi + u[1] * wr;
            }
            double xr = tab[0][2 * j0], xi = tab[0][2 * j0 + 1];
            sr += ar * xr - ai * xi;
            si += ar * xi + ai * xr;
        }
        out[2 * b] = sr * scale;
        out[2 * b + 1] = si * scale;
    }
    for (int m = 0; m < ndim; m++) free(tab[m]);
}
