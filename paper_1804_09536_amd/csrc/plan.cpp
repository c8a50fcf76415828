// plan.cpp -- host plan engine and C ABI of libpfft.
//
// Implements the decomposition (Sec. 3.1, Eq. decompose), the virtual
// Cartesian grid with row-major rank numbering (Sec. 3.3), the chain of
// alignments of the slab / pencil / higher-dimensional methods (Secs. 3.2.1,
// 3.4, 3.5), the order of partial transforms (Eq. fftn_forward and
// Eq. fftn_backward) and the setup-phase construction of the index tables
// that the kernels use to move subarrays (the role the subarray datatypes of
// Alg. SubArray play for Alg. Exchange, built once and reused, Sec. 3.2.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "pfft.h"
#include "pfft_internal.hpp"
#include "pfft_kernels.hpp"

namespace pfft {

static thread_local std::string g_last_error;

static int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

// Eq. decompose: part p of N elements split in M parts gets n = q + [r > p]
// elements starting at s = q*p + min(r, p), with q = N div M, r = N mod M.
static void decompose(int64_t N, int64_t M, int64_t p, int64_t *n, int64_t *s)
{
    int64_t q = N / M, r = N % M;
    *n = q + (r > p ? 1 : 0);
    *s = q * p + std::min(r, p);
}

// One alignment of the array over a (possibly extended) virtual grid.
struct Layout {
    int ndim = 0, ngrid = 0;
    int64_t shape[kMaxDims] = {};
    int64_t grid[kMaxDims] = {};
    int axis_dir[kMaxDims] = {};
    int64_t P = 1;
    int64_t rstride[kMaxDims] = {};  // rank distance between neighbours along a direction
    std::vector<int64_t> rank_off;   // P+1 prefix sums of block sizes
    std::vector<int32_t> own[kMaxDims], loc[kMaxDims];
    std::vector<int64_t> dir_n[kMaxDims];  // per direction d and coordinate c: local extent of the axis d splits
    // Storage order of every rank's block: order[k] is the axis at position k
    // of the block's C-order index (identity for the paper's layouts; the
    // transposed output layout stores its split axes first), pos_of its inverse.
    int order[kMaxDims] = {};
    int pos_of[kMaxDims] = {};

    void init(int nd, const int64_t *shp, int ng, const int64_t *grd, const int *dirs, const int *ord = nullptr)
    {
        ndim = nd;
        ngrid = ng;
        for (int m = 0; m < nd; m++) {
            shape[m] = shp[m];
            axis_dir[m] = dirs[m];
            order[m] = ord ? ord[m] : m;
        }
        for (int k = 0; k < nd; k++) pos_of[order[k]] = k;
        P = 1;
        for (int i = 0; i < ng; i++) {
            grid[i] = grd[i];
            P *= grd[i];
        }
        for (int i = ng - 1, st = 1; i >= 0; i--) {
            rstride[i] = st;
            st *= (int)grd[i];
        }
        for (int m = 0; m < nd; m++) {
            own[m].assign(shape[m], 0);
            loc[m].assign(shape[m], 0);
            int d = axis_dir[m];
            if (d < 0) {
                for (int64_t g = 0; g < shape[m]; g++) loc[m][g] = (int32_t)g;
            } else {
                dir_n[d].assign(grid[d], 0);
                for (int64_t c = 0; c < grid[d]; c++) {
                    int64_t n, s;
                    decompose(shape[m], grid[d], c, &n, &s);
                    dir_n[d][c] = n;
                    for (int64_t g = s; g < s + n; g++) {
                        own[m][g] = (int32_t)c;
                        loc[m][g] = (int32_t)(g - s);
                    }
                }
            }
        }
        rank_off.assign(P + 1, 0);
        for (int64_t r = 0; r < P; r++) {
            int64_t ls[kMaxDims], st[kMaxDims];
            rank_off[r + 1] = rank_off[r] + block(r, ls, st);
        }
        uniform = true;
        for (int m = 0; m < nd; m++)
            if (axis_dir[m] >= 0 && shape[m] % grid[axis_dir[m]] != 0) uniform = false;
    }
    bool uniform = false;  // every axis split evenly: all blocks have one shape

    void coords(int64_t r, int64_t *c) const
    {
        for (int i = ngrid - 1; i >= 0; i--) {
            c[i] = r % grid[i];
            r /= grid[i];
        }
    }

    int64_t block(int64_t r, int64_t *ls, int64_t *st) const
    {
        int64_t c[kMaxDims];
        coords(r, c);
        int64_t cnt = 1;
        for (int m = 0; m < ndim; m++) {
            int d = axis_dir[m];
            if (d < 0) {
                ls[m] = shape[m];
                st[m] = 0;
            } else {
                decompose(shape[m], grid[d], c[d], &ls[m], &st[m]);
            }
            cnt *= ls[m];
        }
        return cnt;
    }

    int64_t total() const { return rank_off[P]; }

    // Local extent of axis m in a block whose coordinate along m's direction is c.
    int64_t local_extent(int m, int64_t c) const
    {
        int d = axis_dir[m];
        return d < 0 ? shape[m] : dir_n[d][c];
    }
};

// One kernel launch of a direction's list.
struct Launch {
    int kind = KIND_C2C;
    int axis = 0;
    int N = 0;        // transform / line length
    int contig = 1;   // transform axis is the last axis
    int src = 0, dst = 0;  // layout ids
    int sign = -1;
    int scale_axis = -1;   // axis whose 1/N_m factor may apply (-1: none)
    int sine = 0;          // R2R: sine (1) or cosine (0) transform
    int xcd = 0;           // complex strided stage whose tiles go to the XCDs in contiguous ranges
    int stream = 0;        // complex strided stage: bit 0 streaming loads, bit 1 streaming stores
    int late_tw = 0;       // stage the twiddle table while the first loads are in flight
    int mixed_sides = 0;   // transform axis stored last on one side only (into / out of a transposed layout)
    // device blob offsets
    size_t off_tiles = 0;
    int64_t ntiles = 0;
    size_t off_pos[2] = {0, 0}, off_na[2] = {0, 0}, off_rank[2] = {0, 0};
    int32_t R[2] = {0, 0};
    size_t off_tw = 0, off_tw2 = 0, off_tw3 = 0;
    int M = 0;             // mixed-radix stage: Bluestein convolution length (0: direct plan)
    KernelConfig cfg{};
};

}  // namespace pfft

using namespace pfft;

struct pfft_plan_s {
    int ndim = 0;
    int64_t shape[kMaxDims] = {};
    int ngrid = 0;
    int64_t grid[kMaxDims] = {};
    int precision = PFFT_F32, kind = PFFT_C2C, norm = PFFT_NORM_FORWARD;
    unsigned flags = 0;
    int nlayouts = 0;                             // chain length
    std::vector<std::array<int, kMaxDims>> dirs;  // per chain layout
    std::vector<Layout> layouts;                  // 0..nlayouts-1: spectral; then extras
    int real0 = -1;                               // id of the real input layout (R2C)
    int r2r[kMaxDims] = {};                       // R2R: per axis PFFT_DCT2 or PFFT_DST2
    std::vector<std::pair<int, int>> sched;       // (chain layout, axis), forward order
    std::vector<Launch> fwd, bwd;
    std::vector<Launch> up, down;  // redistribution between chain neighbours
    std::vector<uint8_t> blob;
    std::map<std::pair<int, int>, std::array<size_t, 3>> side_cache;
    std::map<int, std::pair<size_t, size_t>> tw_cache;
    std::map<std::pair<int, int>, size_t> aux_cache;  // (table kind, length) -> blob offset
    pfft_tuning tuning{};  // performance knobs (kernel tile variants, grid policy)
    std::vector<int> chain_in;  // creation arguments kept for rebuilding
    bool has_chain = false;
    void *dev = nullptr;
    size_t spec_bytes = 0;
    size_t elem = 8;  // element bytes of the spectral layouts (complex; real for R2R)
    // optional per-launch timing
    bool profiling = false;
    struct Prof {
        int kind, axis, contig, N, direction;
        double bytes;
        hipEvent_t a, b;
    };
    std::vector<Prof> prof;
    std::vector<hipEvent_t> pool;
};

namespace pfft {

static size_t blob_put(pfft_plan_s *p, const void *data, size_t bytes)
{
    size_t off = (p->blob.size() + 255) & ~(size_t)255;
    p->blob.resize(off + std::max<size_t>(bytes, 1), 0);
    if (bytes) memcpy(p->blob.data() + off, data, bytes);
    return off;
}

// Side tables of layout `lid` for lines along `axis`: per position the block
// index along the axis and the local index there; per block its local extent;
// the per-rank offsets.
static void side_tables(pfft_plan_s *p, int lid, int axis, size_t *off_pos, size_t *off_na, size_t *off_rank,
                        int32_t *R)
{
    const Layout &L = p->layouts[lid];
    auto key = std::make_pair(lid, axis);
    auto it = p->side_cache.find(key);
    int d = L.axis_dir[axis];
    *R = d < 0 ? 0 : (int32_t)L.rstride[d];
    if (it != p->side_cache.end()) {
        *off_pos = it->second[0];
        *off_na = it->second[1];
        *off_rank = it->second[2];
        return;
    }
    int64_t N = L.shape[axis];
    std::vector<int32_t> pos(2 * N);
    for (int64_t j = 0; j < N; j++) {
        pos[2 * j] = L.own[axis][j];
        pos[2 * j + 1] = L.loc[axis][j];
    }
    std::vector<int32_t> na;
    if (d < 0)
        na.push_back((int32_t)N);
    else
        for (int64_t c = 0; c < L.grid[d]; c++) na.push_back((int32_t)L.dir_n[d][c]);
    *off_pos = blob_put(p, pos.data(), pos.size() * 4);
    *off_na = blob_put(p, na.data(), na.size() * 4);
    *off_rank = blob_put(p, L.rank_off.data(), L.rank_off.size() * 8);
    p->side_cache[key] = {*off_pos, *off_na, *off_rank};
}

// Twiddle table e^{-2 pi i m / n}, m = 0..n-1, from FP64 libm cos/sin with the
// angle reduced exactly in integers, rounded once to the plan precision.
static size_t twiddle_table(pfft_plan_s *p, int n)
{
    auto it = p->tw_cache.find(n);
    if (it != p->tw_cache.end()) return it->second.first;
    size_t off;
    if (p->precision == PFFT_F32) {
        std::vector<float> t(2 * (size_t)n);
        for (int m = 0; m < n; m++) {
            double a = 2.0 * M_PI * (double)m / (double)n;
            t[2 * m] = (float)cos(a);
            t[2 * m + 1] = (float)(-sin(a));
        }
        off = blob_put(p, t.data(), t.size() * 4);
    } else {
        std::vector<double> t(2 * (size_t)n);
        for (int m = 0; m < n; m++) {
            double a = 2.0 * M_PI * (double)m / (double)n;
            t[2 * m] = cos(a);
            t[2 * m + 1] = -sin(a);
        }
        off = blob_put(p, t.data(), t.size() * 8);
    }
    p->tw_cache[n] = {off, 0};
    return off;
}

// Post/pre-processing table of the half-length real-to-real stage of length
// N = 2M: e^{-2 pi i k / N} for k = 0..M, then e^{-i pi k / 2N} for k = 0..M.
static size_t r2r_post_table(pfft_plan_s *p, int N)
{
    auto it = p->tw_cache.find(-N);
    if (it != p->tw_cache.end()) return it->second.first;
    const int M = N / 2;
    std::vector<double> t(4 * (size_t)(M + 1));
    for (int k = 0; k <= M; k++) {
        const double a = 2.0 * M_PI * (double)k / (double)N;
        const double b = 2.0 * M_PI * (double)k / (4.0 * (double)N);
        t[2 * k] = cos(a);
        t[2 * k + 1] = -sin(a);
        t[2 * (M + 1 + k)] = cos(b);
        t[2 * (M + 1 + k) + 1] = -sin(b);
    }
    size_t off;
    if (p->precision == PFFT_F32) {
        std::vector<float> f(t.begin(), t.end());
        off = blob_put(p, f.data(), f.size() * 4);
    } else {
        off = blob_put(p, t.data(), t.size() * 8);
    }
    p->tw_cache[-N] = {off, 0};
    return off;
}

// The chirp e^{-pi i m^2 / N}, m < N, of Bluestein's identity, with the
// angle reduced exactly (m^2 mod 2N) before the FP64 cos/sin.
static size_t chirp_table(pfft_plan_s *p, int N)
{
    auto key = std::make_pair(1, N);
    auto it = p->aux_cache.find(key);
    if (it != p->aux_cache.end()) return it->second;
    std::vector<double> t(2 * (size_t)N);
    for (int64_t m = 0; m < N; m++) {
        const double a = M_PI * (double)((m * m) % (2 * (int64_t)N)) / (double)N;
        t[2 * m] = cos(a);
        t[2 * m + 1] = -sin(a);
    }
    size_t off;
    if (p->precision == PFFT_F32) {
        std::vector<float> f(t.begin(), t.end());
        off = blob_put(p, f.data(), f.size() * 4);
    } else {
        off = blob_put(p, t.data(), t.size() * 8);
    }
    p->aux_cache[key] = off;
    return off;
}

// Host DFT in FP64 (Cooley-Tukey over the smallest prime factor, used only
// for plan-time tables): x <- sum_j x_j e^{-2 pi i jk / n}.
static void host_dft(std::vector<std::complex<double>> &x)
{
    const int64_t n = (int64_t)x.size();
    if (n < 2) return;
    int64_t f = n;
    for (int64_t d = 2; d * d <= n; d++)
        if (n % d == 0) {
            f = d;
            break;
        }
    const int64_t m = n / f;
    std::vector<std::vector<std::complex<double>>> sub((size_t)f, std::vector<std::complex<double>>((size_t)m));
    for (int64_t r = 0; r < f; r++) {
        for (int64_t j = 0; j < m; j++) sub[r][j] = x[(size_t)(r + f * j)];
        if (m > 1) host_dft(sub[r]);
    }
    for (int64_t k = 0; k < n; k++) {
        std::complex<double> acc = 0.0;
        for (int64_t r = 0; r < f; r++) {
            const double a = 2.0 * M_PI * (double)((r * k) % n) / (double)n;
            acc += std::complex<double>(cos(a), -sin(a)) * sub[r][(size_t)(k % m)];
        }
        x[(size_t)k] = acc;
    }
}

// Bluestein's kernel for length N and convolution length M: the M-point DFT
// of v, v_m = e^{+pi i m^2 / N} for |m| < N placed at m mod M, zero elsewhere.
static size_t bluestein_table(pfft_plan_s *p, int N, int M)
{
    auto key = std::make_pair(2, N);
    auto it = p->aux_cache.find(key);
    if (it != p->aux_cache.end()) return it->second;
    std::vector<std::complex<double>> v((size_t)M, 0.0);
    for (int64_t m = 0; m < N; m++) {
        const double a = M_PI * (double)((m * m) % (2 * (int64_t)N)) / (double)N;
        const std::complex<double> c(cos(a), sin(a));
        v[(size_t)m] = c;
        if (m > 0) v[(size_t)(M - m)] = c;
    }
    host_dft(v);
    std::vector<double> t(2 * (size_t)M);
    for (int64_t k = 0; k < M; k++) {
        t[2 * k] = v[(size_t)k].real();
        t[2 * k + 1] = v[(size_t)k].imag();
    }
    size_t off;
    if (p->precision == PFFT_F32) {
        std::vector<float> f(t.begin(), t.end());
        off = blob_put(p, f.data(), f.size() * 4);
    } else {
        off = blob_put(p, t.data(), t.size() * 8);
    }
    p->aux_cache[key] = off;
    return off;
}

struct LineRec {
    int32_t rank[2];
    int64_t O[2], E[2], I[2];
};

// Enumerate every line of a stage along `axis` (source layout A, destination
// layout B) and group them into tiles of at most W lines that are adjacent in
// both layouts.
static bool build_tiles(pfft_plan_s *p, Launch &ln, int W, bool wrap)
{
    const Layout &A = p->layouts[ln.src];
    const Layout &B = p->layouts[ln.dst];
    const Layout *S[2] = {&A, &B};
    const int nd = A.ndim, a = ln.axis;
    // global extents of the non-transform axes; the two sides may differ in
    // the transform axis only (real vs half-spectrum length)
    int64_t ext[kMaxDims];
    int64_t nlines = 1;
    for (int m = 0; m < nd; m++) {
        ext[m] = (m == a) ? 1 : A.shape[m];
        nlines *= ext[m];
    }
    std::vector<LineRec> lines;
    lines.reserve(nlines);
    int64_t g[kMaxDims];
    for (int64_t f = 0; f < nlines; f++) {
        int64_t t = f;
        for (int m = nd - 1; m >= 0; m--) {
            g[m] = t % ext[m];
            t /= ext[m];
        }
        LineRec rec;
        for (int s = 0; s < 2; s++) {
            const Layout &L = *S[s];
            int64_t c[kMaxDims] = {};
            for (int m = 0; m < nd; m++)
                if (m != a && L.axis_dir[m] >= 0) c[L.axis_dir[m]] = L.own[m][g[m]];
            int64_t rank = 0;
            for (int i = 0; i < L.ngrid; i++) rank += c[i] * L.rstride[i];
            // outer index over the axes stored before the transform axis,
            // inner index and extent over those stored after it
            int64_t O = 0, E = 1, I = 0;
            const int pa = L.pos_of[a];
            for (int k = 0; k < pa; k++) {
                const int m = L.order[k];
                int64_t n = L.local_extent(m, L.axis_dir[m] >= 0 ? c[L.axis_dir[m]] : 0);
                O = O * n + L.loc[m][g[m]];
            }
            for (int k = pa + 1; k < nd; k++) {
                const int m = L.order[k];
                int64_t n = L.local_extent(m, L.axis_dir[m] >= 0 ? c[L.axis_dir[m]] : 0);
                I = I * n + L.loc[m][g[m]];
                E *= n;
            }
            rec.rank[s] = (int32_t)rank;
            rec.O[s] = O;
            rec.E[s] = E;
            rec.I[s] = I;
            if (O > INT32_MAX || E > INT32_MAX) return false;  // tile records hold 32-bit indices
        }
        lines.push_back(rec);
    }
    const bool contig = ln.contig != 0;
    // lines of a tile step in I on a side where the transform axis is not
    // stored last (the lines are adjacent there), in O where it is (each line
    // is contiguous); the two sides differ only on a stage into or out of a
    // layout with another storage order, which runs the LDS kernel
    bool istep[2];
    for (int s = 0; s < 2; s++) istep[s] = S[s]->pos_of[a] != nd - 1;
    const bool mixed_sides = istep[0] != istep[1];
    auto less = [contig, mixed_sides](const LineRec &x, const LineRec &y) {
        if (x.rank[1] != y.rank[1]) return x.rank[1] < y.rank[1];
        if (x.rank[0] != y.rank[0]) return x.rank[0] < y.rank[0];
        if (x.E[1] != y.E[1]) return x.E[1] < y.E[1];
        if (x.E[0] != y.E[0]) return x.E[0] < y.E[0];
        if (mixed_sides) {
            if (x.O[1] != y.O[1]) return x.O[1] < y.O[1];
            return x.I[1] < y.I[1];
        }
        if (contig) return x.O[1] < y.O[1];
        if (x.O[1] != y.O[1]) return x.O[1] < y.O[1];
        if (x.O[0] != y.O[0]) return x.O[0] < y.O[0];
        return x.I[1] < y.I[1];
    };
    std::sort(lines.begin(), lines.end(), less);

    // Runs: maximal sequences of lines that are adjacent on both sides (same
    // ranks and inner extents; consecutive O with the same I where lines step
    // in O, consecutive I with the same O where they step in I).
    std::vector<size_t> run_first;
    for (size_t i = 0; i < lines.size(); i++) {
        bool cont = i > 0;
        const LineRec &x = lines[i], &h = lines[i > 0 ? i - 1 : 0];
        for (int s = 0; s < 2 && cont; s++) {
            if (x.rank[s] != h.rank[s] || x.E[s] != h.E[s]) cont = false;
            else if (!istep[s]) cont = (x.O[s] == h.O[s] + 1) && (x.I[s] == h.I[s]);
            else cont = (x.O[s] == h.O[s]) && (x.I[s] == h.I[s] + 1);
        }
        if (!cont) run_first.push_back(i);
    }
    run_first.push_back(lines.size());
    const size_t nruns = run_first.size() - 1;
    auto run_len = [&](size_t r) { return (int64_t)(run_first[r + 1] - run_first[r]); };

    // A strided tile may continue from the end of one run into the next
    // (line (O + 1, same run start I) on both sides) when every block has the
    // same local extent of the transform axis on both sides, so that the step
    // between runs is one number per side.
    int64_t ostr_na[2] = {0, 0};
    if (wrap && !contig) {
        for (int s = 0; s < 2; s++) {
            const Layout &L = *S[s];
            const int d = L.axis_dir[a];
            const int64_t n0 = L.local_extent(a, 0);
            bool uni = true;
            if (d >= 0)
                for (int64_t c = 1; c < L.grid[d]; c++) uni = uni && L.local_extent(a, c) == n0;
            ostr_na[s] = uni ? n0 : 0;
        }
        if (ostr_na[0] == 0 || ostr_na[1] == 0) wrap = false;
    } else {
        wrap = false;
    }
    auto chains = [&](size_t r) {  // run r + 1 continues run r
        if (r + 1 >= nruns || run_len(r + 1) != run_len(r)) return false;
        const LineRec &x = lines[run_first[r]], &y = lines[run_first[r + 1]];
        for (int s = 0; s < 2; s++)
            if (x.rank[s] != y.rank[s] || x.E[s] != y.E[s] || y.O[s] != x.O[s] + 1 || y.I[s] != x.I[s]) return false;
        return true;
    };

    std::vector<Tile> tiles;
    size_t r = 0;
    int64_t off = 0;  // next line: offset `off` in run r
    while (r < nruns) {
        const int64_t len = run_len(r);
        Tile t;
        memset(&t, 0, sizeof t);
        const LineRec &h = lines[run_first[r] + off];
        for (int s = 0; s < 2; s++) {
            t.rank[s] = h.rank[s];
            t.O[s] = (int32_t)h.O[s];
            t.E[s] = (int32_t)h.E[s];
            t.I[s] = (int32_t)h.I[s];
        }
        int64_t cnt = std::min<int64_t>(W, len - off);
        size_t nr = r;
        int64_t noff = off + cnt;
        if (wrap && cnt < W && chains(r)) {
            // continue over the following runs of the same length
            const LineRec &r0 = lines[run_first[r]];
            t.b0 = (int32_t)off;
            t.run = (int32_t)len;
            for (int s = 0; s < 2; s++) {
                t.I[s] = (int32_t)r0.I[s];
                t.ostr[s] = (int32_t)(ostr_na[s] * r0.E[s]);
            }
            while (cnt < W && chains(nr)) {
                nr++;
                const int64_t take = std::min<int64_t>(W - cnt, len);
                cnt += take;
                noff = take;
            }
        }
        t.count = (int32_t)cnt;
        if (noff == run_len(nr)) {
            nr++;
            noff = 0;
        }
        r = nr;
        off = noff;
        // flag bit 0: in strided mode, every line pair (2i, 2i+1) sits at two
        // adjacent elements starting at an even one, at every position on
        // both sides (so fp32 line pairs move as 16-byte units); bit 1: the
        // same for groups of four lines (four 4-byte reals per 16 bytes)
        // In contiguous mode (real-to-real stages only, the one kernel that
        // reads them there) the bits say the same of the positions of a line:
        // each aligned pair (quad) of positions is adjacent in one block and
        // starts at an even (multiple-of-four) element for every line.
        bool even = !contig, quad = !contig;
        if (contig && ln.kind == KIND_R2R) {
            even = quad = true;
            for (int s = 0; s < 2 && (even || quad); s++) {
                const Layout &L = *S[s];
                const int64_t npos = L.shape[a];
                const int d = L.axis_dir[a];
                const int64_t R = d < 0 ? 0 : L.rstride[d];
                if (npos % 2) even = false;
                if (npos % 4) quad = false;
                for (int64_t j = 0; j < npos && (even || quad); j++) {
                    const int64_t c = L.own[a][j], loc = L.loc[a][j];
                    const int64_t na = L.local_extent(a, c);
                    const int64_t addr = L.rank_off[t.rank[s] + c * R] + ((int64_t)t.O[s] * na + loc) * t.E[s] + t.I[s];
                    const int64_t lstride = na * t.E[s];
                    if (j % 2 == 0 && ((addr & 1) || (lstride & 1) || j + 1 >= npos || L.own[a][j + 1] != c))
                        even = false;
                    if (j % 4 == 0 && ((addr & 3) || (lstride & 3) || j + 3 >= npos || L.own[a][j + 3] != c))
                        quad = false;
                }
            }
        }
        if (t.run > 0) {
            even = even && (t.run % 2 == 0) && (t.b0 % 2 == 0) && (t.ostr[0] % 2 == 0) && (t.ostr[1] % 2 == 0);
            quad = quad && (t.run % 4 == 0) && (t.b0 % 4 == 0) && (t.ostr[0] % 4 == 0) && (t.ostr[1] % 4 == 0);
        }
        for (int s = 0; s < 2 && !contig && (even || quad); s++) {
            if (!istep[s]) continue;  // (a stage with mixed sides pairs lines on its adjacent side only)
            const Layout &L = *S[s];
            const int64_t npos = L.shape[a];
            const int d = L.axis_dir[a];
            const int64_t R = d < 0 ? 0 : L.rstride[d];
            const int64_t first = t.run > 0 ? t.b0 : 0;  // element offset of line 0 from (O, I)
            for (int64_t j = 0; j < npos && (even || quad); j++) {
                const int64_t c = L.own[a][j], loc = L.loc[a][j];
                const int64_t na = L.local_extent(a, c);
                const int64_t addr =
                    L.rank_off[t.rank[s] + c * R] + ((int64_t)t.O[s] * na + loc) * t.E[s] + t.I[s] + first;
                if (addr & 1) even = false;
                if (addr & 3) quad = false;
            }
        }
        // bits 2 / 3: the lines of side 0 / 1 step in I (else in O)
        t.flags = (even ? 1 : 0) | (quad ? 2 : 0) | (istep[0] ? 4 : 0) | (istep[1] ? 8 : 0);
        tiles.push_back(t);
    }
    ln.ntiles = (int64_t)tiles.size();
    ln.off_tiles = blob_put(p, tiles.data(), tiles.size() * sizeof(Tile));
    // A complex strided stage that stores straight into a layout splitting its
    // axis (rows of a tile scattered over the blocks of that direction) with
    // unwrapped tiles: neighbouring tiles complete each other's row segments,
    // so they are kept in one XCD's L2 (measured -6 % on such a 512^3 stage).
    // Gathering stages, wrapped tiles, the one-workgroup-per-CU tiles of 1024
    // and 1536 points, and buffers that fit the 256 MB last-level cache (whose
    // writes stay there: 256^3 measured 2 % slower) keep the round-robin order.
    // Tiles whose rows are narrower than a 128-byte cache line (the long lines
    // of 2048 points and more, whose LDS holds only 2-8 lines) share every
    // line with their neighbours, so they take the XCD order in every stage
    // (2048^3 stages 2.1-2.3x faster, 2048-4096-point stages of smaller arrays
    // 2-2.5x).
    bool wrapped = false;
    for (const Tile &t : tiles) wrapped = wrapped || t.run > 0;
    const double esz = p->precision == PFFT_F32 ? 8.0 : 16.0;
    const double dst_bytes = (double)B.total() * esz;
    const bool narrow = (double)W * esz < 128.0;
    ln.xcd = (ln.kind == KIND_C2C && !contig && !wrapped &&
              ((B.axis_dir[a] >= 0 && ln.N <= 512 && dst_bytes > 256.0 * 1048576.0) || narrow))
                 ? 1
                 : 0;
    return true;
}

static int add_layout(pfft_plan_s *p, const int64_t *shape, int ngrid, const int64_t *grid, const int *dirs,
                      const int *order = nullptr)
{
    Layout L;
    L.init(p->ndim, shape, ngrid, grid, dirs, order);
    p->layouts.push_back(std::move(L));
    return (int)p->layouts.size() - 1;
}

static int finish_launch(pfft_plan_s *p, Launch &ln)
{
    const int prec = p->precision;
    if (ln.kind == KIND_COPY) {
        const bool last_s = p->layouts[ln.src].pos_of[ln.axis] == p->ndim - 1;
        const bool last_d = p->layouts[ln.dst].pos_of[ln.axis] == p->ndim - 1;
        ln.mixed_sides = last_s != last_d;
    }
    const pfft_tuning &tu = p->tuning;
    // 64-bit element offsets where a buffer has 2^31 elements or more (or
    // where the tuning asks for them): the kernels' own variants with the
    // default tile shapes
    const bool wide = p->layouts[ln.src].total() >= ((int64_t)1 << 31) ||
                      p->layouts[ln.dst].total() >= ((int64_t)1 << 31) || tu.wide_offsets == 1;
    if (wide && ln.kind == KIND_R2R)
        return fail(PFFT_EUNSUPPORTED, "real-to-real plans with buffers of 2^31 or more elements are not supported");
    int variant = (ln.kind == KIND_C2C || ln.kind == KIND_R2C || ln.kind == KIND_C2R || ln.kind == KIND_R2R)
                      ? (ln.contig ? tu.tile_contig : tu.tile_strided)
                      : 0;
    // 5: the measured choice per length (wider tiles for long strided lines,
    // the long-line shapes from 1536 points: 512 threads at 1536, 1024
    // beyond; real-to-real stages are fastest with more, smaller workgroups,
    // real-to-complex stages with a quarter of the default lines per tile:
    // 512^3 0.264 -> 0.247 ms, while complex-to-real stages lose 12 % there;
    // strided real-to-real stages in complex64 with the row-addressed kernel:
    // 512^3 type II cosine transform 1.61 -> 1.51 ms, while complex128 loses)
    if (variant == 5)
        variant = ln.kind == KIND_R2C                                      ? 2
                  : (ln.kind == KIND_R2R && !ln.contig && prec == PFFT_F32) ? 6
                  : (ln.contig || ln.kind == KIND_R2R)               ? 1
                  : ln.N < 1024                      ? 3
                  : ln.N == 1024                     ? 4
                  : ln.N == 1536                     ? 6
                                                     : 7;
    // 6 / 7: the slot-group shapes of complex strided stages (kernel variants 9 / 10),
    // the row-addressed kernel of strided real-to-real stages (11 / 12)
    if (variant == 6 || variant == 7)
        variant = (ln.kind == KIND_C2C && !ln.contig)   ? variant + 3
                  : (ln.kind == KIND_R2R && !ln.contig) ? variant + 5
                                                        : 0;
    int rc;
    if (ln.mixed_sides && ln.kind != KIND_COPY) {
        // lines contiguous on one side and adjacent on the other: the stage
        // kernel in the source's mode with the destination stepped the other
        // way (or, for lengths without a register plan and in plans with
        // 64-bit offsets, the LDS kernel, which loads and stores each side in
        // its own order)
        ln.contig = p->layouts[ln.src].pos_of[ln.axis] == p->ndim - 1 ? 1 : 0;
        if (ln.kind != KIND_C2C) rc = -1;
        else if (wide) rc = mixed_config(prec, ln.N, ln.kind, &ln.cfg);
        else rc = kernel_config(ln.kind, prec, ln.N, ln.contig, 6, &ln.cfg);
    } else {
        // the alternative radix plan where the tuning asks for it (complex
        // stages of lengths that have one; others keep their variant)
        if (ln.kind == KIND_C2C && !wide && (tu.radix_alt & (ln.contig ? 1 : 2)) != 0) variant = 8;
        rc = kernel_config(ln.kind, prec, ln.N, ln.contig, wide && ln.kind != KIND_COPY ? 7 : variant, &ln.cfg);
        if (ln.kind == KIND_COPY) ln.cfg.wide = wide ? 1 : 0;
    }
    if (ln.kind == KIND_C2C && !ln.cfg.wide && !ln.cfg.xside && !ln.cfg.alt && ln.cfg.id <= 4)
        ln.cfg.resident = ln.contig ? tu.resident_contig : tu.resident_strided;
    if (rc != 0) {
        if (ln.kind == KIND_R2R)
            return fail(PFFT_EUNSUPPORTED, "no real-to-real kernel for length " + std::to_string(ln.N) +
                                               " (needs 2^a <= 4096 or 3*2^a <= 3072)");
        const int M = mixed_bluestein_length(ln.N);
        return fail(PFFT_EUNSUPPORTED, "length " + std::to_string(ln.N) + ": the line" +
                                           (M > 0 ? " (through Bluestein's convolution of length " + std::to_string(M) + ")"
                                                  : std::string()) +
                                           " does not fit one workgroup's LDS");
    }
    const int sides[2] = {ln.src, ln.dst};
    for (int s = 0; s < 2; s++) side_tables(p, sides[s], ln.axis, &ln.off_pos[s], &ln.off_na[s], &ln.off_rank[s], &ln.R[s]);
    if (ln.cfg.id < 0 && ln.kind != KIND_COPY && ln.kind != KIND_R2R) {
        // mixed-radix stage: the L-point table, and Bluestein's chirp and kernel
        const int M = mixed_bluestein_length(ln.N);
        ln.M = M > 0 ? M : 0;
        ln.off_tw = twiddle_table(p, M > 0 ? M : ln.N);
        if (M > 0) {
            ln.off_tw2 = chirp_table(p, ln.N);
            ln.off_tw3 = bluestein_table(p, ln.N, M);
        }
    } else if (ln.kind == KIND_C2C) {
        ln.off_tw = twiddle_table(p, ln.N);
    } else if (ln.kind == KIND_R2C || ln.kind == KIND_C2R) {
        ln.off_tw = twiddle_table(p, ln.N / 2 > 0 ? ln.N / 2 : 1);
        ln.off_tw2 = twiddle_table(p, ln.N);
    } else if (ln.kind == KIND_R2R && r2r_half_length(ln.N)) {
        ln.off_tw = twiddle_table(p, ln.N / 2);
        ln.off_tw2 = r2r_post_table(p, ln.N);
    } else if (ln.kind == KIND_R2R) {
        ln.off_tw = twiddle_table(p, ln.N);
        ln.off_tw2 = twiddle_table(p, 4 * ln.N);  // its first N entries are e^{-i pi k / 2N}
    }
    // runs shorter than a tile are chained only for the Stockham stage kernels
    if (!build_tiles(p, ln, ln.cfg.W, ln.kind == KIND_C2C && ln.cfg.id >= 0 && !ln.contig && !ln.mixed_sides && !wide))
        return fail(PFFT_EUNSUPPORTED, "a block's outer or inner index range exceeds 2^31 elements");
    if (ln.kind == KIND_C2C && !ln.contig && tu.xcd_order != 0) ln.xcd = tu.xcd_order == 1 ? 1 : 0;
    // Streaming accesses on strided rows where source and destination
    // together exceed the 256 MB last-level cache (512^3 pencil stages -4..-7 %
    // with both, 384^3 -7 %; the XCD-ordered scatter stage +4 % with streaming
    // stores but -5 % with streaming loads alone).  Buffers the cache holds
    // are read from it by the next stage, which streaming stores would
    // bypass (64^4 +9 %, 192^3 +3 % with streaming).
    if (ln.kind == KIND_C2C && !ln.contig) {
        const double esz = p->precision == PFFT_F32 ? 8.0 : 16.0;
        const double bytes = ((double)p->layouts[ln.src].total() + (double)p->layouts[ln.dst].total()) * esz;
        const int rule = bytes > 256.0 * 1048576.0 ? (ln.xcd ? 1 : 3) : 0;
        ln.stream = tu.stream_strided == 4 ? rule : tu.stream_strided;
    }
    // Contiguous stages: streaming loads always; streaming stores of whole
    // destination lines only where source and destination exceed the
    // last-level cache (the next stage reads a smaller output from there:
    // 64^4 0.475 -> 0.464 ms, 256^3 0.369 -> 0.363, 128x256x512 0.377 -> 0.373).
    if (ln.kind == KIND_C2C && ln.contig) {
        const double esz = p->precision == PFFT_F32 ? 8.0 : 16.0;
        const double bytes = ((double)p->layouts[ln.src].total() + (double)p->layouts[ln.dst].total()) * esz;
        const int rule = bytes > 256.0 * 1048576.0 ? 3 : 1;
        ln.stream = tu.stream_contig == 4 ? rule : tu.stream_contig;
    }
    // Twiddle tables staged while the first tile's loads are in flight, where
    // those loads come from HBM (source and destination beyond the last-level
    // cache: 512^3 strided stages -1..-3 %, real stages -3..-6 %); stages on
    // cached buffers measured 0.5-2 % slower that way (the 168-transform
    // batch), so they stage the table first.  PFFT_LATE_TWIDDLES=1 in the
    // environment at plan creation takes the late order on every stage (for
    // tests: both orders give bitwise equal results).
    {
        const double esz = p->precision == PFFT_F32 ? 8.0 : 16.0;
        const double bytes = ((double)p->layouts[ln.src].total() + (double)p->layouts[ln.dst].total()) * esz;
        const char *force = getenv("PFFT_LATE_TWIDDLES");
        ln.late_tw = (bytes > 256.0 * 1048576.0 || (force && strcmp(force, "1") == 0)) ? 1 : 0;
    }
    return PFFT_OK;
}

static Launch make_copy(int src, int dst, int last_axis, int64_t n)
{
    Launch c;
    c.kind = KIND_COPY;
    c.axis = last_axis;
    c.N = (int)n;
    c.contig = 1;
    c.src = src;
    c.dst = dst;
    return c;
}

// The redistribution from layout a to layout b as kernel launches, per the
// plan's path flag.  Fused: none (the caller's transform gathers).  Unfused:
// one copy.  Pack+realign: local transpose into per-destination contiguous
// chunks, contiguous chunk exchange, realign on the receiving side
// (Sec. 3.2.1, Eq. transpose).
static int redistribution_launches(pfft_plan_s *p, int a, int b, std::vector<Launch> &out)
{
    // copies: add_layout below may reallocate p->layouts
    const Layout A = p->layouts[a];
    const Layout B = p->layouts[b];
    const int nd = p->ndim;
    unsigned path = p->flags & PFFT_PATH_MASK;
    if (path == PFFT_PATH_PACK_REALIGN) {
        // v: whole in A, split in B; w: split in A, whole in B; both by dir.
        int v = -1, w = -1, n_diff = 0;
        for (int m = 0; m < nd; m++) {
            if (A.axis_dir[m] != B.axis_dir[m]) {
                n_diff++;
                if (A.axis_dir[m] < 0) v = m;
                if (B.axis_dir[m] < 0) w = m;
            }
        }
        if (n_diff == 2 && v >= 0 && w >= 0 && A.axis_dir[w] == B.axis_dir[v]) {
            int dir = A.axis_dir[w];
            int64_t grid2[kMaxDims];
            for (int i = 0; i < A.ngrid; i++) grid2[i] = A.grid[i];
            grid2[A.ngrid] = A.grid[dir];
            int send_dirs[kMaxDims], recv_dirs[kMaxDims];
            for (int m = 0; m < nd; m++) send_dirs[m] = recv_dirs[m] = A.axis_dir[m];
            send_dirs[v] = A.ngrid;  // chunk index q innermost: contiguous per destination
            recv_dirs[w] = A.ngrid;  // chunk index p innermost: contiguous per source
            recv_dirs[v] = dir;
            int ls = add_layout(p, A.shape, A.ngrid + 1, grid2, send_dirs);
            int lr = add_layout(p, A.shape, A.ngrid + 1, grid2, recv_dirs);
            int64_t n = A.shape[nd - 1];
            out.push_back(make_copy(a, ls, nd - 1, n));
            out.push_back(make_copy(ls, lr, nd - 1, n));
            out.push_back(make_copy(lr, b, nd - 1, n));
            return PFFT_OK;
        }
    }
    out.push_back(make_copy(a, b, nd - 1, A.shape[nd - 1]));
    return PFFT_OK;
}

// Build the launch list of one direction.  Each step is (src, li, dst, axis,
// kind): the data sit in layout src, the partial transform along `axis` is
// the one the chain performs on layout li (where the axis is whole), and its
// result must end in layout dst.  R2C reads the real layout src directly into
// li; C2R writes the real layout dst directly from li.
static int build_direction(pfft_plan_s *p, const std::vector<std::array<int, 5>> &steps, int sign,
                           std::vector<Launch> &out)
{
    const bool fused = (p->flags & PFFT_PATH_MASK) == PFFT_PATH_FUSED;
    for (const auto &st : steps) {
        int src = st[0], li = st[1], dst = st[2], axis = st[3], kind = st[4];
        int tsrc = src, tdst = dst;
        if (!fused) {
            if (kind != KIND_R2C && src != li) {
                int rc = redistribution_launches(p, src, li, out);
                if (rc) return rc;
                tsrc = li;
            }
            if (kind != KIND_C2R) tdst = li;
        }
        Launch ln;
        ln.kind = kind;
        ln.axis = axis;
        {
            // contiguous mode where the transform axis is stored last on both sides
            const bool last_s = p->layouts[tsrc].pos_of[axis] == p->ndim - 1;
            const bool last_d = p->layouts[tdst].pos_of[axis] == p->ndim - 1;
            ln.contig = last_s && last_d;
            ln.mixed_sides = last_s != last_d;
        }
        ln.src = tsrc;
        ln.dst = tdst;
        ln.sign = sign;
        ln.scale_axis = axis;
        ln.sine = (kind == KIND_R2R && p->r2r[axis] == PFFT_DST2) ? 1 : 0;
        if (kind == KIND_R2C) ln.N = (int)p->layouts[tsrc].shape[axis];
        else if (kind == KIND_C2R) ln.N = (int)p->layouts[tdst].shape[axis];
        else ln.N = (int)p->layouts[tdst].shape[axis];
        out.push_back(ln);
        if (!fused && kind != KIND_C2R && tdst != dst) {
            int rc = redistribution_launches(p, tdst, dst, out);
            if (rc) return rc;
        }
    }
    for (auto &ln : out) {
        int rc = finish_launch(p, ln);
        if (rc) return rc;
    }
    return PFFT_OK;
}

static int build_plan(pfft_plan_s *p, const int *chain, int nsteps)
{
    const int nd = p->ndim, ng = p->ngrid;
    std::array<int, kMaxDims> dirs;
    dirs.fill(-1);
    for (int i = 0; i < ng; i++) dirs[i] = i;
    p->dirs.push_back(dirs);
    if (chain == nullptr) {
        // paper's rule: step t = 1..g moves direction g-t from axis g-t to g-t+1
        for (int t = 1; t <= ng; t++) {
            int i = ng - t;
            dirs[i] = -1;
            dirs[i + 1] = i;
            p->dirs.push_back(dirs);
        }
    } else {
        for (int s = 0; s < nsteps; s++) {
            int d = chain[2 * s], na = chain[2 * s + 1];
            if (d < 0 || d >= ng || na < 0 || na >= nd) return fail(PFFT_EGRID, "chain step out of range");
            if (dirs[na] != -1) return fail(PFFT_EGRID, "chain step onto a distributed axis");
            int old = -1;
            for (int m = 0; m < nd; m++)
                if (dirs[m] == d) old = m;
            if (old < 0) return fail(PFFT_EINTERNAL, "lost grid direction");
            dirs[old] = -1;
            dirs[na] = d;
            p->dirs.push_back(dirs);
        }
    }
    p->nlayouts = (int)p->dirs.size();
    // forward schedule: on each layout, every newly whole axis, highest first
    bool done[kMaxDims] = {};
    for (int li = 0; li < p->nlayouts; li++)
        for (int m = nd - 1; m >= 0; m--)
            if (p->dirs[li][m] < 0 && !done[m]) {
                p->sched.push_back({li, m});
                done[m] = true;
            }
    for (int m = 0; m < nd; m++)
        if (!done[m]) return fail(PFFT_EGRID, "chain leaves axis " + std::to_string(m) + " distributed everywhere");
    if (p->kind == PFFT_R2C && (p->sched[0].first != 0 || p->sched[0].second != nd - 1))
        return fail(PFFT_EGRID, "r2c needs the last axis whole in the input layout");

    int64_t spec[kMaxDims];
    for (int m = 0; m < nd; m++) spec[m] = p->shape[m];
    if (p->kind == PFFT_R2C) spec[nd - 1] = p->shape[nd - 1] / 2 + 1;
    for (int li = 0; li < p->nlayouts; li++) {
        int order[kMaxDims];
        if ((p->flags & PFFT_TRANSPOSED_OUT) && li == p->nlayouts - 1) {
            // transposed output: the split axes first, in grid-direction
            // order, then the whole axes (slab: (N1/P, N0, N2), Eq. fftw_transposed_out)
            int k = 0;
            for (int d = 0; d < ng; d++)
                for (int m = 0; m < nd; m++)
                    if (p->dirs[li][m] == d) order[k++] = m;
            for (int m = 0; m < nd; m++)
                if (p->dirs[li][m] < 0) order[k++] = m;
            add_layout(p, spec, ng, p->grid, p->dirs[li].data(), order);
        } else {
            add_layout(p, spec, ng, p->grid, p->dirs[li].data());
        }
    }
    if (p->kind == PFFT_R2C) p->real0 = add_layout(p, p->shape, ng, p->grid, p->dirs[0].data());
    p->elem = (p->precision == PFFT_F32 ? 8 : 16) / (p->kind == PFFT_R2R ? 2 : 1);
    p->spec_bytes = (size_t)p->layouts[0].total() * p->elem;

    const int last = p->nlayouts - 1;
    const int K = (int)p->sched.size();
    // forward: stage k reads where stage k-1 wrote; the last writes the last layout
    std::vector<std::array<int, 5>> fsteps, bsteps;
    // placement of intermediates: in the layout of the stage that made them
    // (the next stage gathers) or in the layout of the stage that uses them
    // (this stage scatters)
    const unsigned fwd_place = (p->flags & PFFT_PLACE_MASK) >> 3, bwd_place = (p->flags & PFFT_PLACE_BWD_MASK) >> 5;
    // where stage k of a direction with final layout `fin` leaves its result
    // (placement 0 gather, 1 scatter, 2 direct, 3 final)
    auto place = [&](unsigned mode, int k, int li, int next_li, int fin) {
        if (k == K - 1 || mode == 3) return fin;
        if (mode == 2) return k == 0 ? li : fin;
        return mode == 1 ? next_li : li;
    };
    int where = (p->kind == PFFT_R2C) ? p->real0 : 0;
    for (int k = 0; k < K; k++) {
        int li = p->sched[k].first, axis = p->sched[k].second;
        int dst = place(fwd_place, k, li, k + 1 < K ? p->sched[k + 1].first : last, last);
        int kind = (k == 0 && p->kind == PFFT_R2C) ? KIND_R2C : p->kind == PFFT_R2R ? KIND_R2R : KIND_C2C;
        // the real-to-complex stage writes a layout stored in C order
        if (kind == KIND_R2C && dst != li && p->layouts[dst].pos_of[nd - 1] != nd - 1) dst = li;
        fsteps.push_back({where, li, dst, axis, kind});
        where = dst;
    }
    where = last;
    for (int k = 0; k < K; k++) {
        int li = p->sched[K - 1 - k].first, axis = p->sched[K - 1 - k].second;
        int dst = place(bwd_place, k, li, k + 1 < K ? p->sched[K - 2 - k].first : 0, 0);
        int kind = p->kind == PFFT_R2R ? KIND_R2R : KIND_C2C;
        if (k == K - 1 && p->kind == PFFT_R2C) {
            kind = KIND_C2R;
            dst = p->real0;
        } else if (k == K - 2 && p->kind == PFFT_R2C && p->layouts[dst].pos_of[nd - 1] != nd - 1) {
            // the complex-to-real stage reads a layout stored in C order
            dst = p->sched[0].first;
        }
        bsteps.push_back({where, li, dst, axis, kind});
        where = dst;
    }
    int rc;
    if (!(p->flags & PFFT_LAYOUTS_ONLY)) {
        rc = build_direction(p, fsteps, -1, p->fwd);
        if (rc) return rc;
        rc = build_direction(p, bsteps, +1, p->bwd);
        if (rc) return rc;
    }
    // standalone redistributions between chain neighbours
    for (int li = 0; li + 1 < p->nlayouts; li++) {
        Launch u = make_copy(li, li + 1, nd - 1, spec[nd - 1]);
        Launch d = make_copy(li + 1, li, nd - 1, spec[nd - 1]);
        rc = finish_launch(p, u);
        if (rc) return rc;
        rc = finish_launch(p, d);
        if (rc) return rc;
        p->up.push_back(u);
        p->down.push_back(d);
    }
    return PFFT_OK;
}

// Defaults from a sweep of the 512^3 complex64 pencil workload on MI355X:
// contiguous stages with half-size tiles (four workgroups per CU), strided
// stages with double-width tiles exchanged in two LDS portions (256-byte rows,
// two workgroups per CU), one tile per workgroup for both.
static pfft_tuning default_tuning()
{
    pfft_tuning t;
    t.tile_contig = 1;
    t.tile_strided = 5;  // by length: 3 below 1024 points, 4 from 1024 on
    t.resident_contig = 0;
    t.resident_strided = 0;
    t.xcd_order = 0;
    t.stream_strided = 4;
    t.wide_offsets = 0;
    t.radix_alt = 0;
    t.stream_contig = 4;
    return t;
}

static double axis_scale(const pfft_plan_s *p, int axis, bool forward_factors)
{
    if (axis < 0) return 1.0;
    // real-to-real: the type III transform undoes type II up to 2N
    double n = (double)p->shape[axis] * (p->kind == PFFT_R2R ? 2.0 : 1.0);
    if (p->norm == PFFT_NORM_FORWARD) return forward_factors ? 1.0 / n : 1.0;
    if (p->norm == PFFT_NORM_BACKWARD) return forward_factors ? 1.0 : 1.0 / n;
    return 1.0;
}

static hipEvent_t pool_event(pfft_plan_s *p)
{
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Algorithmic bytes of a launch: its source read once plus its destination
// written once.
static double launch_bytes(const pfft_plan_s *p, const Launch &ln)
{
    auto esz = [p](int lid) { return (double)(lid == p->real0 ? p->elem / 2 : p->elem); };
    return (double)p->layouts[ln.src].total() * esz(ln.src) + (double)p->layouts[ln.dst].total() * esz(ln.dst);
}

// Kernel arguments of one launch, with the plan's tables at device address dev.
static StageArgs stage_args(const pfft_plan_s *p, const Launch &ln, const uint8_t *dev, const void *src, void *dst,
                            double scale, int flags)
{
    StageArgs a;
    memset(&a, 0, sizeof a);
    a.src = src;
    a.dst = dst;
    for (int s = 0; s < 2; s++) {
        a.side[s].rank_off = (const int64_t *)(dev + ln.off_rank[s]);
        a.side[s].pos = (const int2 *)(dev + ln.off_pos[s]);
        a.side[s].na = (const int32_t *)(dev + ln.off_na[s]);
        a.side[s].R = ln.R[s];
        const Layout &L = p->layouts[s == 0 ? ln.src : ln.dst];
        if (L.uniform) {
            a.side[s].ublock = L.total() / L.P;
            int d = L.axis_dir[ln.axis];
            a.side[s].un = (int32_t)(d < 0 ? L.shape[ln.axis] : L.shape[ln.axis] / L.grid[d]);
        }
    }
    a.tiles = (const Tile *)(dev + ln.off_tiles);
    a.twiddle = dev + ln.off_tw;
    a.twiddle2 = dev + ln.off_tw2;
    a.twiddle3 = dev + ln.off_tw3;
    a.M = ln.M;
    a.ntiles = ln.ntiles;
    a.scale = scale;
    a.N = ln.N;
    a.flags = flags;
    return a;
}

static size_t launch_esize(const pfft_plan_s *p, const Launch &ln)
{
    if (ln.kind == KIND_COPY && (ln.src == p->real0 || ln.dst == p->real0)) return p->elem / 2;
    return p->elem;
}

// Kernel flags of a launch in a chain of direction `sign`.  chain_flags:
// SF_HALVE_INTERIOR / SF_DOUBLE_INTERIOR on the adjoint chains; real-to-real
// stages turn them into SF_R2R_ADJOINT, complex stages ignore them.
static int stage_flags(const Launch &ln, int sign, int chain_flags)
{
    if (ln.kind == KIND_R2R)
        return (sign > 0 ? SF_R2R_INVERSE : 0) | (ln.sine ? SF_R2R_SINE : 0) |
               ((chain_flags & (SF_HALVE_INTERIOR | SF_DOUBLE_INTERIOR)) ? SF_R2R_ADJOINT : 0);
    const int late = ln.late_tw ? SF_LATE_TWIDDLES : 0;
    if (ln.kind == KIND_R2C || ln.kind == KIND_C2R) return chain_flags | late;
    return (ln.xcd ? SF_XCD_ORDER : 0) | ((ln.stream & 1) ? SF_LOAD_NT : 0) | ((ln.stream & 2) ? SF_STORE_NT : 0) |
           late;
}

// Fault injection for tests of the error path: with PFFT_FAULT_INJECT=launch
// in the environment every stage launch reports a launch failure instead of
// launching (nothing reaches the device).
static bool launch_fault_injected()
{
    const char *e = getenv("PFFT_FAULT_INJECT");
    return e && strcmp(e, "launch") == 0;
}

static int run_launch(pfft_plan_s *p, const Launch &ln, const void *src, void *dst, double scale, int sign,
                      int flags, hipStream_t stream, int direction = 4)
{
    if (ln.ntiles == 0) return PFFT_OK;
    hipEvent_t ea = nullptr, eb = nullptr;
    if (p->profiling) {
        // the kernel's own start and end (every stage is one kernel launch)
        ea = pool_event(p);
        eb = pool_event(p);
        if (!ea || !eb) return fail(PFFT_EHIP, "hipEventCreate failed");
    }
    flags = stage_flags(ln, sign, flags);
    const StageArgs a = stage_args(p, ln, (const uint8_t *)p->dev, src, dst, scale, flags);
    launch_events() = LaunchEvents{ea, eb};
    int rc = launch_fault_injected()
                 ? (int)hipErrorLaunchFailure
                 : launch_stage(ln.kind, p->precision, ln.N, ln.contig, sign, ln.cfg, launch_esize(p, ln), a, stream);
    launch_events() = LaunchEvents{};
    if (rc != 0) return fail(PFFT_EHIP, std::string("kernel launch failed: ") + hipGetErrorString((hipError_t)rc));
    if (p->profiling) p->prof.push_back({ln.kind, ln.axis, ln.contig, ln.N, direction, launch_bytes(p, ln), ea, eb});
    return PFFT_OK;
}

// Buffers of a launch list: launch k reads srcs[k] and writes dsts[k]; the
// last one writes `out`.  Intermediates ping-pong between `out` and one
// workspace buffer (two when `out` is real), or, with PFFT_DESTROY_INPUT and a
// complex input, between `out` and `in` (the first launch runs in place on
// `in` when it keeps its own layout, else it writes the workspace once).
// Returns the number of workspace buffers used.
static int assign_buffers(const pfft_plan_s *p, const std::vector<Launch> &list, const void *in, void *out,
                          void *work, std::vector<const void *> &srcs, std::vector<void *> &dsts)
{
    const int n = (int)list.size();
    uint8_t *w0 = (uint8_t *)work;
    uint8_t *w1 = w0 ? w0 + ((p->spec_bytes + 255) & ~(size_t)255) : nullptr;
    const bool out_is_real = n > 0 && list.back().dst == p->real0;
    const bool in_is_real = n > 0 && list[0].src == p->real0;
    const bool destroy = (p->flags & PFFT_DESTROY_INPUT) != 0 && !in_is_real;
    void *in_w = const_cast<void *>(in);
    const void *cur = in;
    int used = 0;
    srcs.assign(n, nullptr);
    dsts.assign(n, nullptr);
    // (the workspace buffers in use are counted where they are chosen: the
    // caller's pointers may coincide with w1's address)
    for (int k = 0; k < n; k++) {
        void *dst;
        int slot = -1;  // workspace buffer taken by this launch
        if (k == n - 1) {
            dst = out;
        } else if (out_is_real) {
            if (destroy)
                slot = (k % 2 == 0) ? 0 : -1;
            else
                slot = k % 2;
            dst = slot == 0 ? (void *)w0 : slot == 1 ? (void *)w1 : in_w;
        } else if ((n - 1 - k) % 2 == 0) {
            dst = out;
        } else if (destroy) {
            // only the first launch can land on `in`; in place if it keeps its layout
            const bool in_place = list[0].src == list[0].dst && list[0].kind == KIND_C2C;
            slot = (k > 0 || in_place) ? -1 : 0;
            dst = slot == 0 ? (void *)w0 : in_w;
        } else {
            slot = 0;
            dst = w0;
        }
        used = std::max(used, slot + 1);
        srcs[k] = cur;
        dsts[k] = dst;
        cur = dst;
    }
    return used;
}

// Workspace buffers (of the spectrum's size) the plan's lists need.
static int work_buffers(const pfft_plan_s *p)
{
    static uint8_t probe[3];  // distinct stand-in addresses for in, out, work
    std::vector<const void *> srcs;
    std::vector<void *> dsts;
    int used = 0;
    for (const std::vector<Launch> *list : {&p->fwd, &p->bwd}) {
        // the backward and the adjoints run these lists too; which one is
        // `in` only decides whether the input is real
        used = std::max(used, assign_buffers(p, *list, probe, probe + 1, probe + 2, srcs, dsts));
    }
    return used;
}

// Run a launch list so that the last launch writes `out` (buffers as
// assign_buffers chooses); forward_factors selects the norm's forward or
// backward per-axis factors.
// Byte ranges [a, a + na) and [b, b + nb) share a byte.
static bool overlap(const void *a, size_t na, const void *b, size_t nb)
{
    if (!a || !b || na == 0 || nb == 0) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Bytes of the buffer of layout `lid` (real layouts hold reals).
static size_t layout_bytes(const pfft_plan_s *p, int lid)
{
    return (size_t)p->layouts[lid].total() * (lid == p->real0 ? p->elem / 2 : p->elem);
}

static int run_list(pfft_plan_s *p, const std::vector<Launch> &list, const void *in, void *out, void *work,
                    bool forward_factors, int sign, int r2c_flags, hipStream_t stream, int direction)
{
    if (p->flags & PFFT_LAYOUTS_ONLY) return fail(PFFT_EUNSUPPORTED, "plan was created with PFFT_LAYOUTS_ONLY");
    if (!in || !out) return fail(PFFT_EINVAL, "null buffer");
    // full aligned tiles move 16-byte pieces at offsets the plan checked
    // relative to the buffers' starts
    if (((uintptr_t)in | (uintptr_t)out | (uintptr_t)work) & 15u)
        return fail(PFFT_EINVAL, "in, out and work must be 16-byte aligned");
    const int n = (int)list.size();
    std::vector<const void *> srcs;
    std::vector<void *> dsts;
    const int used = assign_buffers(p, list, in, out, work, srcs, dsts);
    if (used > 0 && !work) return fail(PFFT_EINVAL, "null workspace");
    if (n > 0) {
        // a stage that read and wrote overlapping buffers would race
        const bool destroy = (p->flags & PFFT_DESTROY_INPUT) != 0 && list[0].src != p->real0;
        const size_t in_b = destroy ? std::max(layout_bytes(p, list[0].src), p->spec_bytes)
                                    : layout_bytes(p, list[0].src);
        const size_t out_b = layout_bytes(p, list.back().dst);
        const size_t work_b = (size_t)used * ((p->spec_bytes + 255) & ~(size_t)255);
        if (overlap(in, in_b, out, out_b) || overlap(in, in_b, work, work_b) || overlap(out, out_b, work, work_b))
            return fail(PFFT_EINVAL, "in, out and work must not overlap");
    }
    if (!p->dev) return fail(PFFT_EWORKSPACE, "device state not bound");
    for (int k = 0; k < n; k++) {
        const Launch &ln = list[k];
        double scale = (ln.kind == KIND_COPY) ? 1.0 : axis_scale(p, ln.scale_axis, forward_factors);
        int rc = run_launch(p, ln, srcs[k], dsts[k], scale, sign, r2c_flags, stream, direction);
        if (rc) return rc;
    }
    return PFFT_OK;
}


// Host emulation of the address arithmetic every kernel of a launch performs:
// all reads and writes must stay inside their buffers and every destination
// element must be written exactly once.  Tiles are checked in parallel (host
// threads over ranges of tiles; write counts are atomic).
static int validate_launch(const pfft_plan_s *p, const Launch &ln, const char *what)
{
    const Layout &A = p->layouts[ln.src];
    const Layout &B = p->layouts[ln.dst];
    const Layout *S[2] = {&A, &B};
    const int nd = A.ndim;
    const int64_t size[2] = {A.total(), B.total()};
    // positions per side along the axis (real side of R2C/C2R is N real values)
    const int64_t npos[2] = {A.shape[ln.axis], B.shape[ln.axis]};
    const int64_t jall = std::max(npos[0], npos[1]);
    // the element read and the element written at one position are the same
    // global element (C2C and COPY: every axis; R2C/C2R: every other axis)
    const bool same_pos = npos[0] == npos[1];
    std::vector<uint8_t> hits((size_t)size[1], 0);
    const Tile *tiles = (const Tile *)(p->blob.data() + ln.off_tiles);
    if (ln.ntiles >= ((int64_t)1 << 31)) return fail(PFFT_EINTERNAL, std::string(what) + ": grid too large");
    const int32_t *pos[2], *na[2];
    const int64_t *roff[2];
    // every rank's block shape and global start, per side
    std::vector<int64_t> bls[2], bst[2];
    for (int s = 0; s < 2; s++) {
        pos[s] = (const int32_t *)(p->blob.data() + ln.off_pos[s]);
        na[s] = (const int32_t *)(p->blob.data() + ln.off_na[s]);
        roff[s] = (const int64_t *)(p->blob.data() + ln.off_rank[s]);
        const Layout &L = *S[s];
        bls[s].resize((size_t)L.P * nd);
        bst[s].resize((size_t)L.P * nd);
        for (int64_t r = 0; r < L.P; r++) L.block(r, &bls[s][(size_t)r * nd], &bst[s][(size_t)r * nd]);
    }
    std::atomic<bool> failed{false};
    std::mutex mu;
    std::string first_error;
    auto report = [&](const std::string &msg) {
        std::lock_guard<std::mutex> g(mu);
        if (!failed.exchange(true)) first_error = msg;
    };
    auto check_tiles = [&](int64_t t_begin, int64_t t_end) {
        std::vector<int64_t> ad;  // the tile's addresses, (line, position, side)
        for (int64_t ti = t_begin; ti < t_end && !failed.load(std::memory_order_relaxed); ti++) {
            const Tile &t = tiles[ti];
            if (t.count < 1 || t.count > ln.cfg.W) return report(std::string(what) + ": tile count");
            for (int s = 0; s < 2; s++)
                if (((t.flags >> (2 + s)) & 1) != (S[s]->pos_of[ln.axis] != nd - 1 ? 1 : 0))
                    return report(std::string(what) + ": line step flag");
            ad.assign((size_t)t.count * (size_t)jall * 2, -1);
            if (t.run < 0 || (t.run > 0 && (ln.contig || t.b0 < 0 || t.b0 >= t.run)))
                return report(std::string(what) + ": tile run");
            for (int w = 0; w < t.count; w++) {
                for (int64_t j = 0; j < jall; j++) {
                    int64_t addr[2] = {-1, -1}, rank_of[2] = {0, 0};
                    for (int s = 0; s < 2; s++) {
                        if (j >= npos[s]) continue;
                        const Layout &L = *S[s];
                        int c = pos[s][2 * j], loc = pos[s][2 * j + 1];
                        int64_t rank = t.rank[s] + (int64_t)c * ln.R[s];
                        if (rank < 0 || rank >= L.P) return report(std::string(what) + ": rank");
                        int64_t O = t.O[s], I = t.I[s];
                        if (t.run > 0) {
                            const int64_t q = t.b0 + w;
                            O += q / t.run;
                            I += q % t.run;
                            // the kernels step between runs by ostr elements
                            const int64_t a0 = roff[s][rank] + ((int64_t)t.O[s] * na[s][c] + loc) * t.E[s] + t.I[s];
                            const int64_t a1 = roff[s][rank] + (O * na[s][c] + loc) * t.E[s] + I;
                            if (a1 - a0 != (q % t.run) + (q / t.run) * (int64_t)t.ostr[s])
                                return report(std::string(what) + ": run stride");
                        } else if (!((t.flags >> (2 + s)) & 1)) {
                            O += w;  // lines step in O on this side
                        } else {
                            I += w;
                        }
                        addr[s] = roff[s][rank] + (O * na[s][c] + loc) * t.E[s] + I;
                        rank_of[s] = rank;
                        ad[((size_t)w * (size_t)jall + (size_t)j) * 2 + (size_t)s] = addr[s];
                        if (I < 0 || I >= t.E[s] || addr[s] < roff[s][rank] || addr[s] >= roff[s][rank + 1] ||
                            addr[s] >= size[s])
                            return report(std::string(what) + ": address out of its block");
                        if (s == 1 && __atomic_fetch_add(&hits[(size_t)addr[s]], (uint8_t)1, __ATOMIC_RELAXED) == 255)
                            return report(std::string(what) + ": overflow");
                    }
                    if (j < npos[0] && j < npos[1]) {
                        // global index of both elements, from their rank block and offset in it
                        int64_t g[2][kMaxDims];
                        for (int s = 0; s < 2; s++) {
                            const int64_t *ls = &bls[s][(size_t)rank_of[s] * nd];
                            const int64_t *st = &bst[s][(size_t)rank_of[s] * nd];
                            int64_t e = addr[s] - roff[s][rank_of[s]];
                            for (int k = nd - 1; k >= 0; k--) {  // C order over the storage order
                                const int m = S[s]->order[k];
                                g[s][m] = st[m] + e % ls[m];
                                e /= ls[m];
                            }
                        }
                        for (int m = 0; m < nd; m++)
                            if ((m != ln.axis || same_pos) && g[0][m] != g[1][m])
                                return report(std::string(what) + ": source and destination differ");
                        if (g[0][ln.axis] != j && same_pos) return report(std::string(what) + ": position");
                    }
                }
            }
            // the alignment flags promise groups of G adjacent elements starting
            // at a multiple of G: lines 2i.. (strided) or positions 2i.. of every
            // line (contiguous), G = 2 (bit 0) or 4 (bit 1), on both sides
            for (int bit = 0; bit < 2; bit++) {
                if (!(t.flags & (1 << bit))) continue;
                const int64_t G = bit == 0 ? 2 : 4;
                for (int s = 0; s < 2; s++)
                    for (int w = 0; w < t.count; w++)
                        for (int64_t j = 0; j < npos[s]; j++) {
                            if (ln.mixed_sides && !((t.flags >> (2 + s)) & 1)) break;  // claims the adjacent side only
                            const bool first = ln.contig ? (j % G == 0) : (w % G == 0 && w + G <= t.count);
                            if (!first) continue;
                            const int64_t a0 = ad[((size_t)w * (size_t)jall + (size_t)j) * 2 + (size_t)s];
                            bool ok = a0 % G == 0 && (!ln.contig || j + G <= npos[s]);
                            for (int64_t k = 1; k < G && ok; k++) {
                                const int64_t wk = ln.contig ? w : w + k, jk = ln.contig ? j + k : j;
                                ok = ad[((size_t)wk * (size_t)jall + (size_t)jk) * 2 + (size_t)s] == a0 + k;
                            }
                            if (!ok) return report(std::string(what) + ": tile alignment flag");
                        }
            }
        }
    };
    const int64_t work = ln.ntiles * std::max<int64_t>(1, jall) * 64;  // rough cost per tile
    int nthreads = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
    if (work < ((int64_t)1 << 22)) nthreads = 1;
    if (nthreads > ln.ntiles) nthreads = (int)std::max<int64_t>(1, ln.ntiles);
    std::vector<std::thread> pool;
    for (int k = 1; k < nthreads; k++)
        pool.emplace_back(check_tiles, ln.ntiles * k / nthreads, ln.ntiles * (k + 1) / nthreads);
    check_tiles(0, ln.ntiles / nthreads);
    for (auto &th : pool) th.join();
    if (failed.load()) return fail(PFFT_EINTERNAL, first_error);
    if (ln.xcd) {
        // the kernel's XCD tile order (one tile per workgroup) must visit every tile once
        std::vector<uint8_t> seen((size_t)ln.ntiles, 0);
        const int64_t nt = ln.ntiles, q = nt / 8, r = nt % 8;
        for (int64_t b = 0; b < nt; b++) {
            const int64_t x = b % 8, k = b / 8, ti = x * q + std::min(x, r) + k;
            if (ti < 0 || ti >= nt || seen[(size_t)ti]++)
                return fail(PFFT_EINTERNAL, std::string(what) + ": XCD tile order is not a permutation");
        }
    }
    for (int64_t e = 0; e < size[1]; e++)
        if (hits[e] != 1) return fail(PFFT_EINTERNAL, std::string(what) + ": destination element written " +
                                                          std::to_string(hits[e]) + " times");
    return PFFT_OK;
}


// ------------------------------------------------------------- batches --

// Stages that the multi-transform kernel runs (the default radix plan, both
// sides stepping alike, 32-bit offsets, a register plan for the length).
static bool multi_kernel(const KernelConfig &c) { return c.id >= 0 && c.id <= 4 && !c.xside && !c.alt && !c.wide; }

// Stages of a batch that run as one launch over the tiles of all members of
// a group: complex stages with a multi-transform kernel, and real-to-complex
// / complex-to-real stages with 32-bit offsets.
static bool batch_multi(int kind, const KernelConfig &c)
{
    if (kind == KIND_C2C) return multi_kernel(c);
    return (kind == KIND_R2C || kind == KIND_C2R) && !c.wide && c.id >= 0 && c.id <= 2;
}

struct BatchGroup {
    int k = 0;              // launch index within each member's list
    int kind = KIND_C2C;
    int N = 0, contig = 0;
    KernelConfig cfg;
    std::vector<int> members;  // member plan indices (C2C groups)
    size_t off_tiles = 0;      // merged tiles in the batch state
    int64_t ntiles = 0;
    size_t off_args = 0;       // one StageArgs per member
};

}  // namespace pfft

struct pfft_batch_s {
    std::vector<pfft_plan_s *> plans;  // members (pointers into `owned`)
    std::vector<pfft_plan_s *> owned;  // private copies of the distinct plans
    ~pfft_batch_s()
    {
        for (auto *p : owned) delete p;
    }
    int precision = 0;
    std::vector<size_t> in_off, out_off, work_off, blob_off;
    size_t in_bytes = 0, out_bytes = 0, work_bytes = 0;
    std::vector<pfft::BatchGroup> groups[2];  // forward, backward; in execution order
    std::vector<uint8_t> blob;                 // host image of the batch device state
    void *dev = nullptr, *in = nullptr, *out = nullptr, *work = nullptr;
};

namespace pfft {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t blob_reserve(std::vector<uint8_t> &b, size_t bytes)
{
    size_t off = align256(b.size());
    b.resize(off + std::max<size_t>(bytes, 1), 0);
    return off;
}

// Group the members' launches: launch k of every member with the same kernel
// shape runs in one multi-transform launch (complex stages); other kinds run
// per member.  Groups are ordered by k, so every member's launches keep their
// order.
static int batch_plan(pfft_batch_s *b)
{
    const int nm = (int)b->plans.size();
    for (int m = 0; m < nm; m++) {
        pfft_plan_s *p = b->plans[m];
        b->in_off.push_back(b->in_bytes);
        b->out_off.push_back(b->out_bytes);
        b->work_off.push_back(b->work_bytes);
        size_t ib = (size_t)p->layouts[p->kind == PFFT_R2C ? p->real0 : 0].total() *
                    (p->kind == PFFT_R2C ? p->elem / 2 : p->elem);
        size_t ob = (size_t)p->layouts[p->nlayouts - 1].total() * p->elem;
        // the backward writes the input layout, so both buffers hold either
        b->in_bytes += align256(std::max(ib, ob));
        b->out_bytes += align256(std::max(ib, ob));
        b->work_bytes += align256(p->spec_bytes) * (size_t)work_buffers(p);
        // members that are the same plan share one copy of its tables
        size_t off = SIZE_MAX;
        for (int q = 0; q < m; q++)
            if (b->plans[q] == p) off = b->blob_off[q];
        if (off == SIZE_MAX) {
            off = blob_reserve(b->blob, p->blob.size());
            memcpy(b->blob.data() + off, p->blob.data(), p->blob.size());
        }
        b->blob_off.push_back(off);
    }
    for (int dir = 0; dir < 2; dir++) {
        size_t maxk = 0;
        for (auto *p : b->plans) maxk = std::max(maxk, (dir == 0 ? p->fwd : p->bwd).size());
        for (size_t k = 0; k < maxk; k++) {
            std::vector<BatchGroup> gs;
            for (int m = 0; m < nm; m++) {
                const auto &list = dir == 0 ? b->plans[m]->fwd : b->plans[m]->bwd;
                if (k >= list.size()) continue;
                const Launch &ln = list[k];
                BatchGroup *g = nullptr;
                // a multi-transform kernel exists (not for stages whose sides step differently)
                const bool multi = batch_multi(ln.kind, ln.cfg);
                if (multi)
                    for (auto &x : gs)
                        if (x.kind == ln.kind && batch_multi(x.kind, x.cfg) && x.N == ln.N && x.contig == ln.contig &&
                            x.cfg.id == ln.cfg.id && x.cfg.resident == ln.cfg.resident)
                            g = &x;
                if (!g) {
                    gs.emplace_back();
                    g = &gs.back();
                    g->k = (int)k;
                    g->kind = ln.kind;
                    g->N = ln.N;
                    g->contig = ln.contig;
                    g->cfg = ln.cfg;
                }
                g->members.push_back(m);
            }
            for (auto &g : gs) {
                if (batch_multi(g.kind, g.cfg)) {
                    int64_t nt = 0;
                    for (int m : g.members) nt += (dir == 0 ? b->plans[m]->fwd : b->plans[m]->bwd)[k].ntiles;
                    if ((int64_t)g.members.size() >= (1 << 23)) return fail(PFFT_EINVAL, "too many batch members");
                    g.ntiles = nt;
                    g.off_tiles = blob_reserve(b->blob, (size_t)nt * sizeof(Tile));
                    Tile *dst = (Tile *)(b->blob.data() + g.off_tiles);
                    for (size_t mi = 0; mi < g.members.size(); mi++) {
                        const pfft_plan_s *p = b->plans[g.members[mi]];
                        const Launch &ln = (dir == 0 ? p->fwd : p->bwd)[k];
                        const Tile *src = (const Tile *)(p->blob.data() + ln.off_tiles);
                        for (int64_t t = 0; t < ln.ntiles; t++) {
                            *dst = src[t];
                            dst->flags = (src[t].flags & 0xff) | (int32_t)(mi << 8);
                            dst++;
                        }
                    }
                    g.off_args = blob_reserve(b->blob, g.members.size() * sizeof(StageArgs));
                }
                b->groups[dir].push_back(g);
            }
        }
    }
    return PFFT_OK;
}

// With the batch's buffers known, write every member's kernel arguments.
static void batch_fill_args(pfft_batch_s *b)
{
    const uint8_t *dev = (const uint8_t *)b->dev;
    for (int dir = 0; dir < 2; dir++) {
        for (auto &g : b->groups[dir]) {
            if (!batch_multi(g.kind, g.cfg)) continue;
            StageArgs *args = (StageArgs *)(b->blob.data() + g.off_args);
            for (size_t mi = 0; mi < g.members.size(); mi++) {
                const int m = g.members[mi];
                const pfft_plan_s *p = b->plans[m];
                const auto &list = dir == 0 ? p->fwd : p->bwd;
                std::vector<const void *> srcs;
                std::vector<void *> dsts;
                uint8_t *in = (uint8_t *)b->in + b->in_off[m], *out = (uint8_t *)b->out + b->out_off[m];
                uint8_t *work = (uint8_t *)b->work + b->work_off[m];
                if (dir == 0)
                    assign_buffers(p, list, in, out, work, srcs, dsts);
                else  // the backward reads the forward's output buffer and writes the input buffer
                    assign_buffers(p, list, out, in, work, srcs, dsts);
                const Launch &ln = list[g.k];
                double scale = axis_scale(p, ln.scale_axis, dir == 0);
                StageArgs a = stage_args(p, ln, dev + b->blob_off[m], srcs[g.k], dsts[g.k], scale, 0);
                a.tiles = nullptr;
                a.ntiles = 0;
                args[mi] = a;
            }
        }
    }
}

}  // namespace pfft

// ------------------------------------------------------------------ C ABI --

#define PFFT_GUARD_BEGIN try {
#define PFFT_GUARD_END                                                    \
    }                                                                     \
    catch (const std::bad_alloc &) {                                      \
        return pfft::fail(PFFT_EINTERNAL, "host allocation failed");      \
    }                                                                     \
    catch (...) {                                                         \
        return pfft::fail(PFFT_EINTERNAL, "unexpected exception");        \
    }

extern "C" {

static int create_plan(pfft_plan *out, int ndim, const int64_t *global_shape, int grid_ndim, const int *grid_dims,
                       int precision, int kind, const int *r2r, int norm, const int *chain, int nsteps, unsigned flags)
{
    if (!out) return fail(PFFT_EINVAL, "null plan pointer");
    *out = nullptr;
    if (!global_shape || !grid_dims) return fail(PFFT_EINVAL, "null shape or grid");
    if (ndim < 1 || ndim > PFFT_MAX_DIMS) return fail(PFFT_ESHAPE, "ndim out of range");
    if (grid_ndim < 1 || grid_ndim >= ndim) return fail(PFFT_EGRID, "grid dims must be in [1, ndim)");
    for (int m = 0; m < ndim; m++)
        if (global_shape[m] < 1 || global_shape[m] > (int64_t)1 << 31) return fail(PFFT_ESHAPE, "bad extent");
    int64_t P = 1;
    for (int i = 0; i < grid_ndim; i++) {
        if (grid_dims[i] < 1) return fail(PFFT_EGRID, "grid extent < 1");
        P *= grid_dims[i];
    }
    if (P > (int64_t)1 << 20) return fail(PFFT_EGRID, "too many virtual ranks");
    if (precision != PFFT_F32 && precision != PFFT_F64) return fail(PFFT_EDTYPE, "bad precision");
    if (kind != PFFT_C2C && kind != PFFT_R2C && kind != PFFT_R2R) return fail(PFFT_EDTYPE, "bad kind");
    if (kind == PFFT_R2R) {
        if (!r2r) return fail(PFFT_EINVAL, "real-to-real plans need a transform kind per axis");
        for (int m = 0; m < ndim; m++)
            if (r2r[m] != PFFT_DCT2 && r2r[m] != PFFT_DST2) return fail(PFFT_EDTYPE, "bad real-to-real kind");
    }
    if (norm < PFFT_NORM_FORWARD || norm > PFFT_NORM_NONE) return fail(PFFT_EINVAL, "bad norm");
    if ((flags & ~(PFFT_PATH_MASK | PFFT_LAYOUTS_ONLY | PFFT_PLACE_MASK | PFFT_PLACE_BWD_MASK | PFFT_DESTROY_INPUT |
                   PFFT_TRANSPOSED_OUT)) != 0 ||
        (flags & PFFT_PATH_MASK) == 3u)
        return fail(PFFT_EINVAL, "bad flags");
    if ((flags & PFFT_TRANSPOSED_OUT) && kind == PFFT_R2R && !(flags & PFFT_LAYOUTS_ONLY))
        return fail(PFFT_EUNSUPPORTED, "transposed output is not available for real-to-real plans");
    if (chain && nsteps < 0) return fail(PFFT_EINVAL, "bad nsteps");
    int64_t total = 1;
    for (int m = 0; m < ndim; m++) total *= global_shape[m];
    if (total > ((int64_t)1 << 40)) return fail(PFFT_ESHAPE, "array too large");
    pfft_plan_s *p = new pfft_plan_s();
    p->ndim = ndim;
    for (int m = 0; m < ndim; m++) p->shape[m] = global_shape[m];
    p->ngrid = grid_ndim;
    for (int i = 0; i < grid_ndim; i++) p->grid[i] = grid_dims[i];
    p->precision = precision;
    p->kind = kind;
    p->norm = norm;
    p->flags = flags;
    if (kind == PFFT_R2R)
        for (int m = 0; m < ndim; m++) p->r2r[m] = r2r[m];
    p->tuning = default_tuning();
    if (chain) {
        p->has_chain = true;
        p->chain_in.assign(chain, chain + 2 * nsteps);
    }
    int rc = build_plan(p, chain, chain ? nsteps : 0);
    if (rc != PFFT_OK) {
        delete p;
        return rc;
    }
    *out = p;
    return PFFT_OK;
}

int pfft_plan_create(pfft_plan *out, int ndim, const int64_t *global_shape, int grid_ndim, const int *grid_dims,
                     int precision, int kind, int norm, const int *chain, int nsteps, unsigned flags)
{
    PFFT_GUARD_BEGIN
    if (kind == PFFT_R2R) return fail(PFFT_EDTYPE, "real-to-real plans are created with pfft_plan_create_r2r");
    return create_plan(out, ndim, global_shape, grid_ndim, grid_dims, precision, kind, nullptr, norm, chain, nsteps,
                       flags);
    PFFT_GUARD_END
}

int pfft_plan_create_r2r(pfft_plan *out, int ndim, const int64_t *global_shape, int grid_ndim, const int *grid_dims,
                         int precision, const int *kinds, int norm, const int *chain, int nsteps, unsigned flags)
{
    PFFT_GUARD_BEGIN
    return create_plan(out, ndim, global_shape, grid_ndim, grid_dims, precision, PFFT_R2R, kinds, norm, chain, nsteps,
                       flags);
    PFFT_GUARD_END
}

int pfft_plan_set_tuning(pfft_plan plan, const pfft_tuning *t)
{
    PFFT_GUARD_BEGIN
    if (!plan || !t) return fail(PFFT_EINVAL, "null argument");
    if (t->tile_contig < 0 || t->tile_contig > 5 || t->tile_strided < 0 || t->tile_strided > 7 ||
        t->resident_contig < 0 || t->resident_contig > 1 || t->resident_strided < 0 || t->resident_strided > 1 ||
        t->xcd_order < 0 || t->xcd_order > 2 || t->stream_strided < 0 || t->stream_strided > 4 || t->wide_offsets < 0 ||
        t->wide_offsets > 1 || t->radix_alt < 0 || t->radix_alt > 3 ||
        t->stream_contig < 0 || t->stream_contig > 4)
        return fail(PFFT_EINVAL, "tuning field out of range");
    // rebuild every table with the new kernel shapes; the device state must be bound again
    plan->tuning = *t;
    plan->dirs.clear();
    plan->layouts.clear();
    plan->sched.clear();
    plan->fwd.clear();
    plan->bwd.clear();
    plan->up.clear();
    plan->down.clear();
    plan->blob.clear();
    plan->side_cache.clear();
    plan->tw_cache.clear();
    plan->aux_cache.clear();
    plan->real0 = -1;
    plan->dev = nullptr;
    const int n = (int)plan->chain_in.size() / 2;
    return build_plan(plan, plan->has_chain ? plan->chain_in.data() : nullptr, n);
    PFFT_GUARD_END
}

int pfft_plan_get_tuning(pfft_plan plan, pfft_tuning *t)
{
    if (!plan || !t) return fail(PFFT_EINVAL, "null argument");
    *t = plan->tuning;
    return PFFT_OK;
}

int pfft_plan_destroy(pfft_plan plan)
{
    if (!plan) return fail(PFFT_EINVAL, "null plan");
    for (auto &r : plan->prof) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (hipEvent_t e : plan->pool) hipEventDestroy(e);
    delete plan;
    return PFFT_OK;
}

int pfft_set_profiling(pfft_plan plan, int enable)
{
    if (!plan) return fail(PFFT_EINVAL, "null plan");
    plan->profiling = enable != 0;
    return PFFT_OK;
}

int pfft_profile_read(pfft_plan plan, int max_entries, pfft_profile_entry *entries, int *n)
{
    PFFT_GUARD_BEGIN
    if (!plan || !n || (max_entries > 0 && !entries)) return fail(PFFT_EINVAL, "null argument");
    int k = 0;
    int status = PFFT_OK;
    for (auto &r : plan->prof) {
        if (k < max_entries) {
            float ms = 0.f;
            hipError_t e = hipEventSynchronize(r.b);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
            if (e != hipSuccess) status = fail(PFFT_EHIP, std::string("profile read: ") + hipGetErrorString(e));
            pfft_profile_entry &o = entries[k];
            o.kind = r.kind;
            o.axis = r.axis;
            o.contig = r.contig;
            o.length = r.N;
            o.direction = r.direction;
            o.ms = ms;
            o.bytes = r.bytes;
        }
        k++;
        plan->pool.push_back(r.a);
        plan->pool.push_back(r.b);
    }
    plan->prof.clear();
    *n = k;
    return status;
    PFFT_GUARD_END
}

int pfft_num_layouts(pfft_plan plan, int *n)
{
    if (!plan || !n) return fail(PFFT_EINVAL, "null argument");
    *n = plan->nlayouts;
    return PFFT_OK;
}

int pfft_local_block(pfft_plan plan, int layout, int real, int rank, int64_t *shape, int64_t *start,
                     int64_t *offset)
{
    PFFT_GUARD_BEGIN
    if (!plan || !shape || !start || !offset) return fail(PFFT_EINVAL, "null argument");
    if (layout < 0 || layout >= plan->nlayouts) return fail(PFFT_EINVAL, "layout out of range");
    int lid = layout;
    if (real) {
        if (plan->kind != PFFT_R2C || layout != 0) return fail(PFFT_EINVAL, "only layout 0 of an r2c plan is real");
        lid = plan->real0;
    }
    const Layout &L = plan->layouts[lid];
    if (rank < 0 || rank >= L.P) return fail(PFFT_EINVAL, "rank out of range");
    L.block(rank, shape, start);
    *offset = L.rank_off[rank];
    return PFFT_OK;
    PFFT_GUARD_END
}

int pfft_layout_axis_order(pfft_plan plan, int layout, int *order)
{
    if (!plan || !order) return fail(PFFT_EINVAL, "null argument");
    if (layout < 0 || layout >= plan->nlayouts) return fail(PFFT_EINVAL, "layout out of range");
    for (int k = 0; k < plan->ndim; k++) order[k] = plan->layouts[layout].order[k];
    return PFFT_OK;
}

int pfft_buffer_bytes(pfft_plan plan, int layout, int real, size_t *bytes)
{
    if (!plan || !bytes) return fail(PFFT_EINVAL, "null argument");
    if (layout < 0 || layout >= plan->nlayouts) return fail(PFFT_EINVAL, "layout out of range");
    if (real) {
        if (plan->kind != PFFT_R2C || layout != 0) return fail(PFFT_EINVAL, "only layout 0 of an r2c plan is real");
        *bytes = (size_t)plan->layouts[plan->real0].total() * (plan->elem / 2);
        return PFFT_OK;
    }
    *bytes = (size_t)plan->layouts[layout].total() * plan->elem;
    return PFFT_OK;
}

int pfft_device_state_bytes(pfft_plan plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(PFFT_EINVAL, "null argument");
    *bytes = (plan->blob.size() + 255) & ~(size_t)255;
    return PFFT_OK;
}

int pfft_bind_device_state(pfft_plan plan, void *dev, hipStream_t stream)
{
    if (!plan || !dev) return fail(PFFT_EINVAL, "null argument");
    if (((uintptr_t)dev & 255u) != 0) return fail(PFFT_EINVAL, "device state must be 256-byte aligned");
    hipError_t e = hipMemcpyAsync(dev, plan->blob.data(), plan->blob.size(), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(PFFT_EHIP, std::string("upload: ") + hipGetErrorString(e));
    e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(PFFT_EHIP, std::string("upload sync: ") + hipGetErrorString(e));
    plan->dev = dev;
    return PFFT_OK;
}

int pfft_workspace_bytes(pfft_plan plan, size_t *bytes)
{
    if (!plan || !bytes) return fail(PFFT_EINVAL, "null argument");
    size_t one = (plan->spec_bytes + 255) & ~(size_t)255;
    *bytes = one * (size_t)work_buffers(plan);
    return PFFT_OK;
}

int pfft_redistribute(pfft_plan plan, int layout_from, int layout_to, const void *in, void *out, hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    if (!plan || !in || !out) return fail(PFFT_EINVAL, "null argument");
    int n = plan->nlayouts;
    if (layout_from < 0 || layout_from >= n || layout_to < 0 || layout_to >= n)
        return fail(PFFT_EINVAL, "layout out of range");
    if (overlap(in, layout_bytes(plan, layout_from), out, layout_bytes(plan, layout_to)))
        return fail(PFFT_EINVAL, "in and out must not overlap");
    if (!plan->dev) return fail(PFFT_EWORKSPACE, "device state not bound");
    if (layout_to == layout_from + 1) return run_launch(plan, plan->up[layout_from], in, out, 1.0, -1, 0, stream);
    if (layout_to == layout_from - 1) return run_launch(plan, plan->down[layout_to], in, out, 1.0, -1, 0, stream);
    return fail(PFFT_EINVAL, "layouts must be chain neighbours (one exchange apart)");
    PFFT_GUARD_END
}

int pfft_forward(pfft_plan plan, const void *in, void *out, void *work, hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    if (!plan) return fail(PFFT_EINVAL, "null plan");
    return run_list(plan, plan->fwd, in, out, work, true, -1, 0, stream, 0);
    PFFT_GUARD_END
}

int pfft_backward(pfft_plan plan, const void *in, void *out, void *work, hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    if (!plan) return fail(PFFT_EINVAL, "null plan");
    return run_list(plan, plan->bwd, in, out, work, false, +1, 0, stream, 1);
    PFFT_GUARD_END
}

int pfft_adjoint_forward(pfft_plan plan, const void *in, void *out, void *work, hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    if (!plan) return fail(PFFT_EINVAL, "null plan");
    return run_list(plan, plan->bwd, in, out, work, true, +1, SF_HALVE_INTERIOR, stream, 2);
    PFFT_GUARD_END
}

int pfft_adjoint_backward(pfft_plan plan, const void *in, void *out, void *work, hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    if (!plan) return fail(PFFT_EINVAL, "null plan");
    return run_list(plan, plan->fwd, in, out, work, false, -1, SF_DOUBLE_INTERIOR, stream, 3);
    PFFT_GUARD_END
}

int pfft_validate_plan(pfft_plan plan)
{
    PFFT_GUARD_BEGIN
    if (!plan) return fail(PFFT_EINVAL, "null plan");
    const std::vector<Launch> *lists[4] = {&plan->fwd, &plan->bwd, &plan->up, &plan->down};
    const char *names[4] = {"forward", "backward", "redistribute up", "redistribute down"};
    for (int li = 0; li < 4; li++)
        for (const Launch &ln : *lists[li]) {
            int rc = validate_launch(plan, ln, names[li]);
            if (rc) return rc;
        }
    return PFFT_OK;
    PFFT_GUARD_END
}

int pfft_batch_create(pfft_batch *out, int nplans, const pfft_plan *plans)
{
    PFFT_GUARD_BEGIN
    if (!out || !plans || nplans < 1) return fail(PFFT_EINVAL, "bad batch arguments");
    *out = nullptr;
    pfft_batch_s *b = new pfft_batch_s();
    for (int i = 0; i < nplans; i++) {
        if (!plans[i]) {
            delete b;
            return fail(PFFT_EINVAL, "null plan in batch");
        }
        if (plans[i]->flags & PFFT_LAYOUTS_ONLY) {
            delete b;
            return fail(PFFT_EUNSUPPORTED, "a layouts-only plan cannot join a batch");
        }
        if (i > 0 && plans[i]->precision != plans[0]->precision) {
            delete b;
            return fail(PFFT_EDTYPE, "batch members must share one precision");
        }
        pfft_plan_s *copy = nullptr;
        for (int q = 0; q < i; q++)
            if (plans[q] == plans[i]) copy = b->plans[q];
        if (!copy) {
            copy = new pfft_plan_s(*plans[i]);
            copy->prof.clear();
            copy->pool.clear();
            copy->profiling = false;
            copy->dev = nullptr;
            b->owned.push_back(copy);
        }
        b->plans.push_back(copy);
    }
    b->precision = plans[0]->precision;
    int rc = batch_plan(b);
    if (rc) {
        delete b;
        return rc;
    }
    *out = b;
    return PFFT_OK;
    PFFT_GUARD_END
}

int pfft_batch_destroy(pfft_batch batch)
{
    if (!batch) return fail(PFFT_EINVAL, "null batch");
    delete batch;
    return PFFT_OK;
}

int pfft_batch_buffer_bytes(pfft_batch b, size_t *in_bytes, size_t *out_bytes, size_t *work_bytes)
{
    if (!b || !in_bytes || !out_bytes || !work_bytes) return fail(PFFT_EINVAL, "null argument");
    *in_bytes = std::max<size_t>(b->in_bytes, 256);
    *out_bytes = std::max<size_t>(b->out_bytes, 256);
    *work_bytes = std::max<size_t>(b->work_bytes, 256);
    return PFFT_OK;
}

int pfft_batch_member_offsets(pfft_batch b, int member, size_t *in_offset, size_t *out_offset)
{
    if (!b || !in_offset || !out_offset) return fail(PFFT_EINVAL, "null argument");
    if (member < 0 || member >= (int)b->plans.size()) return fail(PFFT_EINVAL, "member out of range");
    *in_offset = b->in_off[member];
    *out_offset = b->out_off[member];
    return PFFT_OK;
}

static_assert(PFFT_ENERGY_PARTIALS == pfft::kEnergyPartials, "partials buffer size");

// x: always needed (partials / the gradient scalar); y: the loss (always) or
// the gradient (when n > 0)
static int energy_args(int precision, int64_t n, const void *u, const void *w, const void *x, const void *y,
                       size_t xalign, size_t yalign, bool y_always)
{
    if (precision != PFFT_F32 && precision != PFFT_F64) return fail(PFFT_EDTYPE, "bad precision");
    if (n < 0) return fail(PFFT_EINVAL, "negative element count");
    if (!x || (!y && (y_always || n > 0)) || (n > 0 && (!u || !w))) return fail(PFFT_EINVAL, "null buffer");
    const uintptr_t r = precision == PFFT_F32 ? 4 : 8;
    if (((uintptr_t)u % (2 * r)) || ((uintptr_t)w % r) || ((uintptr_t)x % xalign) || ((uintptr_t)y % yalign))
        return fail(PFFT_EINVAL, "misaligned buffer");
    return PFFT_OK;
}

int pfft_weighted_energy(int precision, int64_t n, const void *u, const void *w, double *partials, void *loss,
                         hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    const size_t r = precision == PFFT_F64 ? 8 : 4;
    int rc = energy_args(precision, n, u, w, partials, loss, 8, r, true);
    if (rc) return rc;
    hipError_t e = energy_launch(precision == PFFT_F64 ? 1 : 0, (long)n, u, w, partials, loss, stream);
    if (e != hipSuccess) return fail(PFFT_EHIP, std::string("energy launch: ") + hipGetErrorString(e));
    return PFFT_OK;
    PFFT_GUARD_END
}

int pfft_weighted_energy_noalloc(int precision, int64_t n, const void *u, const void *w, void *loss,
                                 hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    const size_t r = precision == PFFT_F64 ? 8 : 4;
    // (the loss pointer stands in for the absent partials in the null check)
    int rc = energy_args(precision, n, u, w, loss, loss, r, r, true);
    if (rc) return rc;
    hipError_t e = energy_launch_noalloc(precision == PFFT_F64 ? 1 : 0, (long)n, u, w, loss, stream);
    if (e != hipSuccess) return fail(PFFT_EHIP, std::string("energy launch (static scratch): ") + hipGetErrorString(e));
    return PFFT_OK;
    PFFT_GUARD_END
}

int pfft_weighted_energy_grad(int precision, int64_t n, const void *u, const void *w, const void *g_dev, void *grad,
                              hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    const size_t r = precision == PFFT_F64 ? 8 : 4;
    int rc = energy_args(precision, n, u, w, g_dev, grad, r, 2 * r, false);
    if (rc) return rc;
    if (n > 0 && grad == u) return fail(PFFT_EINVAL, "grad overlaps u");
    hipError_t e = energy_grad_launch(precision == PFFT_F64 ? 1 : 0, (long)n, u, w, g_dev, grad, stream);
    if (e != hipSuccess) return fail(PFFT_EHIP, std::string("energy gradient launch: ") + hipGetErrorString(e));
    return PFFT_OK;
    PFFT_GUARD_END
}

int pfft_batch_device_state_bytes(pfft_batch b, size_t *bytes)
{
    if (!b || !bytes) return fail(PFFT_EINVAL, "null argument");
    *bytes = align256(b->blob.size());
    return PFFT_OK;
}

int pfft_batch_bind(pfft_batch b, void *state, void *in, void *out, void *work, hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    if (!b || !state || !in || !out || !work) return fail(PFFT_EINVAL, "null argument");
    if (((uintptr_t)state & 255u) != 0) return fail(PFFT_EINVAL, "device state must be 256-byte aligned");
    if (((uintptr_t)in | (uintptr_t)out | (uintptr_t)work) & 15u)
        return fail(PFFT_EINVAL, "in, out and work must be 16-byte aligned");
    if (overlap(in, b->in_bytes, out, b->out_bytes) || overlap(in, b->in_bytes, work, b->work_bytes) ||
        overlap(out, b->out_bytes, work, b->work_bytes))
        return fail(PFFT_EINVAL, "in, out and work must not overlap");
    b->dev = state;
    b->in = in;
    b->out = out;
    b->work = work;
    batch_fill_args(b);
    hipError_t e = hipMemcpyAsync(state, b->blob.data(), b->blob.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        b->dev = nullptr;
        return fail(PFFT_EHIP, std::string("batch upload: ") + hipGetErrorString(e));
    }
    return PFFT_OK;
    PFFT_GUARD_END
}

int pfft_batch_execute(pfft_batch b, int direction, hipStream_t stream)
{
    PFFT_GUARD_BEGIN
    if (!b) return fail(PFFT_EINVAL, "null batch");
    if (direction != 0 && direction != 1) return fail(PFFT_EINVAL, "direction must be 0 (forward) or 1 (backward)");
    if (!b->dev) return fail(PFFT_EWORKSPACE, "batch not bound");
    const uint8_t *dev = (const uint8_t *)b->dev;
    const int sign = direction == 0 ? -1 : 1;
    for (const auto &g : b->groups[direction]) {
        if (batch_multi(g.kind, g.cfg)) {
            if (g.ntiles == 0) continue;
            const StageArgs *args = (const StageArgs *)(dev + g.off_args);
            const Tile *tiles = (const Tile *)(dev + g.off_tiles);
            hipError_t e = launch_fault_injected() ? hipErrorLaunchFailure
                           : g.kind != KIND_C2C
                               ? real_launch_multi(b->precision, g.N, g.kind, g.cfg, args, tiles, g.ntiles, stream)
                           : b->precision == PFFT_F32
                               ? c2c_launch_multi_f32(g.N, g.contig, sign, g.cfg, args, tiles, g.ntiles, stream)
                               : c2c_launch_multi_f64(g.N, g.contig, sign, g.cfg, args, tiles, g.ntiles, stream);
            if (e != hipSuccess) return fail(PFFT_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
            continue;
        }
        for (int m : g.members) {
            pfft_plan_s *p = b->plans[m];
            const auto &list = direction == 0 ? p->fwd : p->bwd;
            const Launch &ln = list[g.k];
            if (ln.ntiles == 0) continue;
            std::vector<const void *> srcs;
            std::vector<void *> dsts;
            uint8_t *in = (uint8_t *)b->in + b->in_off[m], *out = (uint8_t *)b->out + b->out_off[m];
            uint8_t *work = (uint8_t *)b->work + b->work_off[m];
            if (direction == 0)
                assign_buffers(p, list, in, out, work, srcs, dsts);
            else
                assign_buffers(p, list, out, in, work, srcs, dsts);
            double scale = ln.kind == KIND_COPY ? 1.0 : axis_scale(p, ln.scale_axis, direction == 0);
            StageArgs a = stage_args(p, ln, dev + b->blob_off[m], srcs[g.k], dsts[g.k], scale, stage_flags(ln, sign, 0));
            int rc = launch_fault_injected()
                         ? (int)hipErrorLaunchFailure
                         : launch_stage(ln.kind, p->precision, ln.N, ln.contig, sign, ln.cfg, launch_esize(p, ln), a, stream);
            if (rc != 0) return fail(PFFT_EHIP, std::string("batch launch: ") + hipGetErrorString((hipError_t)rc));
        }
    }
    return PFFT_OK;
    PFFT_GUARD_END
}

const char *pfft_strerror(int status)
{
    switch (status) {
    case PFFT_OK: return "ok";
    case PFFT_EINVAL: return "invalid argument";
    case PFFT_ESHAPE: return "bad global shape";
    case PFFT_EGRID: return "bad virtual process grid or chain";
    case PFFT_EDTYPE: return "bad precision or kind";
    case PFFT_EUNSUPPORTED: return "unsupported transform length";
    case PFFT_EWORKSPACE: return "device state not bound or buffer too small";
    case PFFT_EHIP: return "HIP runtime error";
    case PFFT_EINTERNAL: return "internal error";
    default: return "unknown status";
    }
}

const char *pfft_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
