"""Python side of the CPU FP64 oracle: ctypes binding of ``oracle.c`` plus the
layout chains and transform chains of the paper, written out step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Citations name the paper's sections and equations:
  * Sec. 2, Eqs. 1-2 and Eq. multifft: forward DFT has sign -1 and the factor
    1/N_m per axis; the backward has sign +1 and no factor.
  * Sec. 2, Eq. fftn_forward / fftn_backward: the forward applies the partial
    transforms last axis first, the backward in the opposite order.
  * Sec. 3.1, Eq. decompose: balanced block-contiguous decomposition.
  * Sec. 3.2, Eq. general_gt / Eq. gt: redistribution v -> w inside a group P.
  * Sec. 3.3: row-major rank numbering of a Cartesian grid.
  * Sec. 3.4 (Eqs. pencil0-pencil2) and Sec. 3.5 (Eqs. 4d_fft0-4d_fft3): the
    chain of alignments for a grid of dimension g on a d-dim array.

  * Real-to-real transforms (the "similar" transforms the method also carries,
    Sec. 1 and the conclusions): per axis the quarter-wave cosine or sine
    transform of type II and its inverse of type III, in the unnormalised
    form Y_k = 2 sum_j x_j cos(pi (2j+1) k / 2N) (type II cosine) and the
    standard companions; a forward factor 1/(2N) makes type III undo type II.

Data model: one numpy buffer per alignment holding the rank blocks (C order)
one after another in rank order; complex data is complex128, real float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = [
    "build", "decompose", "Layout", "paper_layouts", "layouts_from_steps",
    "transform_schedule", "scatter_global", "gather_global", "redistribute",
    "redistribute_pairs", "fft_axis", "dft1", "bruteforce_dftn", "forward",
    "backward", "adjoint_forward", "adjoint_backward", "wavenumber_weight",
    "loss_and_grad", "Chain", "dft_bins", "layout_offset",
    "R2R_KINDS", "r2r_matrix", "r2r_axis", "bruteforce_r2rn", "transposed_order", "relayout",
]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP, FP64)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        vp = ctypes.c_void_p
        lib.oracle_decompose.argtypes = [ctypes.c_int64] * 3 + [i64p, i64p]
        lib.oracle_decompose.restype = None
        lib.oracle_block.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p, ip, ctypes.c_int64, i64p, i64p]
        lib.oracle_block.restype = ctypes.c_int64
        lib.oracle_rank_offsets.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p, ip, i64p]
        lib.oracle_rank_offsets.restype = None
        lib.oracle_redistribute_global.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p, ip, ip, vp, vp,
                                                   ctypes.c_int64]
        lib.oracle_redistribute_global.restype = None
        lib.oracle_redistribute_pairs.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p, ip, ip,
                                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp,
                                                  ctypes.c_int64]
        lib.oracle_redistribute_pairs.restype = ctypes.c_int
        lib.oracle_fft_axis.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p, ip, vp, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_double]
        lib.oracle_fft_axis.restype = ctypes.c_int
        lib.oracle_dft1.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int]
        lib.oracle_dft1.restype = None
        lib.oracle_r2c_last.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p, ip, vp, vp, ctypes.c_double]
        lib.oracle_r2c_last.restype = ctypes.c_int
        lib.oracle_c2r_last.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p, ip, vp, vp, ctypes.c_double,
                                        ctypes.c_int]
        lib.oracle_c2r_last.restype = ctypes.c_int
        lib.oracle_bruteforce_dft.argtypes = [ctypes.c_int, i64p, vp, vp, ctypes.c_int, ctypes.c_double]
        lib.oracle_bruteforce_dft.restype = None
        lib.oracle_dft_bins.argtypes = [ctypes.c_int, i64p, vp, ctypes.c_int64, i64p, vp, ctypes.c_int,
                                        ctypes.c_double]
        lib.oracle_dft_bins.restype = None
        _lib = lib
    return _lib


def _i64(seq):
    return (ctypes.c_int64 * max(1, len(seq)))(*[int(x) for x in seq])


def _int(seq):
    return (ctypes.c_int * max(1, len(seq)))(*[int(x) for x in seq])


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------- layouts --


def decompose(N: int, M: int, p: int):
    """Eq. decompose (Sec. 3.1): (n_p, s_p) of part p of N elements in M parts."""
    n = ctypes.c_int64()
    s = ctypes.c_int64()
    _load().oracle_decompose(int(N), int(M), int(p), ctypes.byref(n), ctypes.byref(s))
    return n.value, s.value


@dataclass(frozen=True)
class Layout:
    """One alignment of a d-dim array over a virtual grid (Sec. 3.3).

    ``axis_dir[m]`` is the grid direction distributing axis m, or -1 when axis
    m is whole on every rank.  Rank blocks are C-order and concatenated in
    row-major rank order."""

    shape: tuple
    grid: tuple
    axis_dir: tuple
    order: tuple = None  # storage order of the blocks (axis at each C-order position); None = identity

    @property
    def storage(self) -> tuple:
        return tuple(range(len(self.shape))) if self.order is None else tuple(self.order)

    @property
    def nranks(self) -> int:
        return int(np.prod(self.grid)) if len(self.grid) else 1

    def block(self, rank: int):
        ls = _i64([0] * len(self.shape))
        st = _i64([0] * len(self.shape))
        _load().oracle_block(len(self.shape), _i64(self.shape), len(self.grid), _i64(self.grid),
                             _int(self.axis_dir), int(rank), ls, st)
        return tuple(ls[i] for i in range(len(self.shape))), tuple(st[i] for i in range(len(self.shape)))

    def offsets(self):
        out = _i64([0] * (self.nranks + 1))
        _load().oracle_rank_offsets(len(self.shape), _i64(self.shape), len(self.grid), _i64(self.grid),
                                    _int(self.axis_dir), out)
        return [out[i] for i in range(self.nranks + 1)]

    @property
    def size(self) -> int:
        return int(np.prod(self.shape))

    def with_shape(self, shape):
        return Layout(tuple(shape), self.grid, self.axis_dir, self.order)

    def regular(self):
        """The same alignment with blocks stored in C order of the axes."""
        return Layout(self.shape, self.grid, self.axis_dir)


def transposed_order(axis_dir):
    """Storage order of a transposed-out alignment (Sec. 3.2.1, Eq.
    fftw_transposed_out, where the slab (N0/P, N1, N2) becomes
    (N1/P, N0, N2)): the split axes first, by grid direction, then the whole
    axes in increasing order."""
    nd = len(axis_dir)
    ngrid = max([d for d in axis_dir if d >= 0] + [-1]) + 1
    split = [m for d in range(ngrid) for m in range(nd) if axis_dir[m] == d]
    return tuple(split + [m for m in range(nd) if axis_dir[m] < 0])


def paper_layouts(ndim: int, ngrid: int):
    """Alignments of the paper's rule (Secs. 3.2.1, 3.4, 3.5): grid direction
    i starts on axis i; redistribution t = 1..g moves direction g-t from axis
    g-t to axis g-t+1.  Returns the list of axis_dir tuples."""
    if not (1 <= ngrid < ndim):
        raise ValueError("need 1 <= grid dims < array dims")
    dirs = [-1] * ndim
    for i in range(ngrid):
        dirs[i] = i
    out = [tuple(dirs)]
    for t in range(1, ngrid + 1):
        i = ngrid - t
        dirs[i] = -1
        dirs[i + 1] = i
        out.append(tuple(dirs))
    return out


def layouts_from_steps(ndim: int, ngrid: int, steps):
    """Explicit chain: start like the paper (direction i on axis i), then each
    step (dir, new_axis) moves grid direction ``dir`` onto ``new_axis``."""
    dirs = [-1] * ndim
    for i in range(ngrid):
        dirs[i] = i
    out = [tuple(dirs)]
    for d, new_axis in steps:
        old = dirs.index(d)
        if dirs[new_axis] != -1:
            raise ValueError("target axis already distributed")
        dirs[old] = -1
        dirs[new_axis] = d
        out.append(tuple(dirs))
    return out


def transform_schedule(chain_dirs):
    """Forward order of partial transforms (Eq. fftn_forward): on each
    alignment, transform every axis that is whole there and not yet done,
    highest axis first.  Returns [(layout_index, axis), ...]."""
    ndim = len(chain_dirs[0])
    done = set()
    sched = []
    for li, dirs in enumerate(chain_dirs):
        for m in sorted((m for m in range(ndim) if dirs[m] == -1 and m not in done), reverse=True):
            sched.append((li, m))
            done.add(m)
    if len(done) != ndim:
        raise ValueError("chain leaves an axis untransformed")
    return sched


def scatter_global(glob: np.ndarray, lay: Layout) -> np.ndarray:
    """Cut a global C-order array into the rank blocks of ``lay`` by plain numpy
    slicing (each block's axes permuted into the layout's storage order), and
    concatenate them in rank order."""
    assert tuple(glob.shape) == tuple(lay.shape)
    parts = []
    order = lay.storage
    for r in range(lay.nranks):
        ls, st = lay.block(r)
        sl = tuple(slice(s, s + n) for s, n in zip(st, ls))
        parts.append(np.ascontiguousarray(np.transpose(glob[sl], order)).reshape(-1))
    return np.concatenate(parts) if parts else np.zeros(0, glob.dtype)


def gather_global(buf: np.ndarray, lay: Layout) -> np.ndarray:
    """Inverse of ``scatter_global``."""
    glob = np.empty(lay.shape, dtype=buf.dtype)
    offs = lay.offsets()
    order = lay.storage
    inverse = tuple(int(k) for k in np.argsort(order))
    for r in range(lay.nranks):
        ls, st = lay.block(r)
        sl = tuple(slice(s, s + n) for s, n in zip(st, ls))
        stored = buf[offs[r]:offs[r + 1]].reshape(tuple(ls[m] for m in order))
        glob[sl] = np.transpose(stored, inverse)
    return glob


def relayout(buf: np.ndarray, A: Layout, B: Layout) -> np.ndarray:
    """The buffer of layout A rewritten in layout B (same global array):
    gathered to the global array and cut again."""
    return scatter_global(gather_global(buf, A), B)


def redistribute(buf: np.ndarray, A: Layout, B: Layout) -> np.ndarray:
    """Global-view redistribution (Eq. gt): out[B(g)] = in[A(g)] for every g.
    Layouts with a non-C storage order go through ``relayout``."""
    assert A.shape == B.shape and A.grid == B.grid
    if A.order is not None or B.order is not None:
        return relayout(np.asarray(buf), A, B)
    buf = np.ascontiguousarray(buf)
    out = np.empty_like(buf)
    _load().oracle_redistribute_global(len(A.shape), _i64(A.shape), len(A.grid), _i64(A.grid),
                                       _int(A.axis_dir), _int(B.axis_dir), _ptr(buf), _ptr(out),
                                       buf.dtype.itemsize)
    return out


def redistribute_pairs(buf: np.ndarray, A: Layout, B: Layout) -> np.ndarray:
    """Redistribution as the per-pair subarray exchange of Alg. Exchange."""
    assert A.shape == B.shape and A.grid == B.grid
    diff = [m for m in range(len(A.shape)) if A.axis_dir[m] != B.axis_dir[m]]
    if len(diff) != 2:
        raise ValueError("layouts differ in more than one exchange")
    v = next(m for m in diff if A.axis_dir[m] == -1)
    w = next(m for m in diff if B.axis_dir[m] == -1)
    d = A.axis_dir[w]
    buf = np.ascontiguousarray(buf)
    out = np.empty_like(buf)
    rc = _load().oracle_redistribute_pairs(len(A.shape), _i64(A.shape), len(A.grid), _i64(A.grid),
                                           _int(A.axis_dir), _int(B.axis_dir), d, v, w, _ptr(buf),
                                           _ptr(out), buf.dtype.itemsize)
    if rc != 0:
        raise ValueError("layouts are not related by one exchange")
    return out


def fft_axis(buf: np.ndarray, lay: Layout, axis: int, sign: int, scale: float) -> np.ndarray:
    """Partial transform F_axis (Sec. 2) of every line of every rank block."""
    out = np.array(buf, dtype=np.complex128, copy=True)
    rc = _load().oracle_fft_axis(len(lay.shape), _i64(lay.shape), len(lay.grid), _i64(lay.grid),
                                 _int(lay.axis_dir), _ptr(out), int(axis), int(sign), float(scale))
    if rc != 0:
        raise ValueError("axis %d is distributed in this layout" % axis)
    return out


def dft1(x: np.ndarray, sign: int) -> np.ndarray:
    """Unnormalised 1-D DFT of one line (radix-2 for 2^k, direct sum else)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _load().oracle_dft1(_ptr(x), _ptr(y), x.size, int(sign))
    return y


def bruteforce_dftn(glob: np.ndarray, sign: int, scale: float) -> np.ndarray:
    """Eq. multifft evaluated term by term on a (tiny) global array."""
    x = np.ascontiguousarray(glob, dtype=np.complex128)
    y = np.empty_like(x)
    _load().oracle_bruteforce_dft(x.ndim, _i64(x.shape), _ptr(x), _ptr(y), int(sign), float(scale))
    return y


def dft_bins(glob: np.ndarray, bins, sign: int, scale: float) -> np.ndarray:
    """Selected bins of Eq. multifft, each as the full sum over the array."""
    x = np.ascontiguousarray(glob, dtype=np.complex128)
    ks = np.ascontiguousarray(np.asarray(bins, dtype=np.int64).reshape(-1, x.ndim))
    out = np.empty(len(ks), dtype=np.complex128)
    _load().oracle_dft_bins(x.ndim, _i64(x.shape), _ptr(x), len(ks), ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            _ptr(out), int(sign), float(scale))
    return out


def layout_offset(lay: Layout, g) -> int:
    """Position of global index g in a layout's buffer (found by searching
    each split axis's parts; the local index is taken in the layout's
    storage order)."""
    nd = len(lay.shape)
    coords = [0] * max(1, len(lay.grid))
    loc = [0] * nd
    for m in range(nd):
        d = lay.axis_dir[m]
        if d < 0:
            loc[m] = int(g[m])
            continue
        for p in range(lay.grid[d]):
            n, s = decompose(lay.shape[m], lay.grid[d], p)
            if s <= g[m] < s + n:
                coords[d] = p
                loc[m] = int(g[m]) - s
                break
    rank = 0
    for i, c in enumerate(coords[:len(lay.grid)]):
        rank = rank * lay.grid[i] + c
    ls, _ = lay.block(rank)
    off = 0
    for m in lay.storage:
        off = off * ls[m] + loc[m]
    return lay.offsets()[rank] + off


def _r2c_last(buf, lay_real: Layout, scale):
    h = lay_real.shape[-1] // 2 + 1
    lay_c = lay_real.with_shape(lay_real.shape[:-1] + (h,))
    x = np.ascontiguousarray(buf, dtype=np.float64)
    out = np.empty(lay_c.size, dtype=np.complex128)
    rc = _load().oracle_r2c_last(len(lay_real.shape), _i64(lay_real.shape), len(lay_real.grid),
                                 _i64(lay_real.grid), _int(lay_real.axis_dir), _ptr(x), _ptr(out),
                                 float(scale))
    if rc != 0:
        raise ValueError("last axis must be whole for r2c")
    return out


def _c2r_last(buf, lay_real: Layout, scale, halve_interior=False):
    z = np.ascontiguousarray(buf, dtype=np.complex128)
    out = np.empty(lay_real.size, dtype=np.float64)
    rc = _load().oracle_c2r_last(len(lay_real.shape), _i64(lay_real.shape), len(lay_real.grid),
                                 _i64(lay_real.grid), _int(lay_real.axis_dir), _ptr(z), _ptr(out),
                                 float(scale), int(bool(halve_interior)))
    if rc != 0:
        raise ValueError("last axis must be whole for c2r")
    return out


# ------------------------------------------------- real-to-real (r2r) --

R2R_KINDS = ("dct2", "dst2")


def r2r_matrix(n: int, kind: str, inverse: bool) -> np.ndarray:
    """Matrix (row k = output, column j = input) of one line's unnormalised
    real-to-real transform, from the definitions:
      dct2: Y_k = 2 sum_j x_j cos(pi (2j+1) k / 2n)
      dct3 (inverse of dct2): Y_k = x_0 + 2 sum_{j>=1} x_j cos(pi j (2k+1) / 2n)
      dst2: Y_k = 2 sum_j x_j sin(pi (2j+1) (k+1) / 2n)
      dst3 (inverse of dst2): Y_k = (-1)^k x_{n-1} + 2 sum_{j<n-1} x_j sin(pi (j+1) (2k+1) / 2n)
    Angles are reduced exactly as integers m/(4n) of a full turn before the
    FP64 cos/sin; type III followed by type II gives 2n times the identity."""
    if kind not in R2R_KINDS:
        raise ValueError("kind must be one of %s" % (R2R_KINDS,))
    j = np.arange(n, dtype=np.int64)[None, :]
    k = np.arange(n, dtype=np.int64)[:, None]
    turn = 4 * n
    if kind == "dct2" and not inverse:
        m = ((2 * j + 1) * k) % turn
        return 2.0 * np.cos(2.0 * np.pi * m / turn)
    if kind == "dct2":
        m = (j * (2 * k + 1)) % turn
        M = 2.0 * np.cos(2.0 * np.pi * m / turn)
        M[:, 0] = 1.0
        return M
    if not inverse:
        m = ((2 * j + 1) * (k + 1)) % turn
        return 2.0 * np.sin(2.0 * np.pi * m / turn)
    m = ((j + 1) * (2 * k + 1)) % turn
    M = 2.0 * np.sin(2.0 * np.pi * m / turn)
    M[:, n - 1] = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    return M


def r2r_axis(buf: np.ndarray, lay: Layout, axis: int, kind: str, inverse: bool, scale: float,
             transpose: bool = False) -> np.ndarray:
    """Real-to-real partial transform along ``axis`` of every line of every
    rank block (the axis must be whole in ``lay``): the line matrix (or its
    transpose) applied along the axis (a matrix product), times ``scale``."""
    if lay.axis_dir[axis] != -1:
        raise ValueError("axis %d is distributed in this layout" % axis)
    M = r2r_matrix(lay.shape[axis], kind, inverse)
    if transpose:
        M = M.T
    x = np.ascontiguousarray(buf, dtype=np.float64)
    out = np.empty_like(x)
    offs = lay.offsets()
    for r in range(lay.nranks):
        ls, _ = lay.block(r)
        if offs[r + 1] == offs[r]:
            continue
        blk = x[offs[r]:offs[r + 1]].reshape(ls)
        y = np.moveaxis(np.tensordot(M, blk, axes=([1], [axis])), 0, axis)
        out[offs[r]:offs[r + 1]] = (y * scale).reshape(-1)
    return out


def bruteforce_r2rn(glob: np.ndarray, kinds, inverse: bool, scales) -> np.ndarray:
    """The separable multi-dimensional real-to-real transform evaluated term
    by term on a (tiny) global array: every output element is the full sum
    over every input element of the product of the per-axis coefficients."""
    import itertools
    x = np.asarray(glob, dtype=np.float64)
    mats = [r2r_matrix(n, kd, inverse) * sc for n, kd, sc in zip(x.shape, kinds, scales)]
    out = np.zeros_like(x)
    for kidx in itertools.product(*[range(n) for n in x.shape]):
        acc = 0.0
        for jidx in itertools.product(*[range(n) for n in x.shape]):
            c = 1.0
            for a in range(x.ndim):
                c *= mats[a][kidx[a], jidx[a]]
            acc += c * x[jidx]
        out[kidx] = acc
    return out


# ---------------------------------------------------------------- chains --


@dataclass
class Chain:
    """A full distributed transform: global shape, grid, the alignments it
    passes through, its real/complex kind and normalisation.

    norm: "forward" (the paper: 1/N_m on each forward partial transform),
    "backward" (1/N_m on the backward) or "none"."""

    shape: tuple
    grid: tuple
    dirs: list
    kind: str = "c2c"
    norm: str = "forward"
    r2r: tuple = None  # kind="r2r": the forward transform of each axis (R2R_KINDS)
    transposed_out: bool = False  # last layout stored in the transposed-out order

    @staticmethod
    def paper(shape, grid, kind="c2c", norm="forward", steps=None, r2r=None, transposed_out=False):
        shape = tuple(int(x) for x in shape)
        grid = tuple(int(x) for x in grid)
        dirs = (paper_layouts(len(shape), len(grid)) if steps is None
                else layouts_from_steps(len(shape), len(grid), steps))
        if kind == "r2r":
            r2r = tuple(r2r) if r2r is not None else ("dct2",) * len(shape)
            if len(r2r) != len(shape) or any(k not in R2R_KINDS for k in r2r):
                raise ValueError("one r2r kind per axis")
        return Chain(shape, grid, dirs, kind, norm, r2r, bool(transposed_out))

    def spectral_shape(self):
        if self.kind == "r2c":
            return self.shape[:-1] + (self.shape[-1] // 2 + 1,)
        return self.shape

    def layout(self, li: int, spectral: bool = True) -> Layout:
        """Alignment li as stored (the last one in the transposed-out order
        when the chain has it)."""
        shp = self.spectral_shape() if spectral else self.shape
        order = None
        if self.transposed_out and li == len(self.dirs) - 1 and spectral:
            order = transposed_order(self.dirs[li])
        return Layout(shp, self.grid, tuple(self.dirs[li]), order)

    def input_layout(self) -> Layout:
        return self.layout(0, spectral=(self.kind != "r2c"))

    def output_layout(self) -> Layout:
        return self.layout(len(self.dirs) - 1)

    def scale(self, axis: int, direction: str) -> float:
        # real-to-real: type III undoes type II up to 2N
        n = self.shape[axis] * (2 if self.kind == "r2r" else 1)
        if self.norm == "forward":
            return 1.0 / n if direction == "forward" else 1.0
        if self.norm == "backward":
            return 1.0 if direction == "forward" else 1.0 / n
        return 1.0


def _regular(ch: Chain) -> Chain:
    return Chain(ch.shape, ch.grid, ch.dirs, ch.kind, ch.norm, ch.r2r, False)


def _run_forward(ch: Chain, buf, sign, scale_of, r2c_mode):
    """Shared walk of the forward chain (sign -1).  r2c_mode: "r2c"
    (truncated real transform) or "r2c_double" (r2c with interior bins
    doubled: the adjoint of c2r)."""
    sched = transform_schedule(ch.dirs)
    cur = 0
    data = buf
    first = True
    for li, axis in sched:
        while cur < li:
            data = redistribute(data, ch.layout(cur), ch.layout(cur + 1))
            cur += 1
        if ch.kind == "r2r":
            # the adjoint of the backward walks this chain with the inverse's transpose
            adj = r2c_mode == "r2c_double"
            data = r2r_axis(data, ch.layout(li), axis, ch.r2r[axis], adj, scale_of(axis), transpose=adj)
        elif first and ch.kind == "r2c":
            assert axis == len(ch.shape) - 1, "r2c needs the last axis transformed first"
            data = _r2c_last(data, ch.layout(0, spectral=False), scale_of(axis))
            if r2c_mode == "r2c_double":
                data = data.reshape(-1, ch.spectral_shape()[-1]).copy()
                n = ch.shape[-1]
                k = np.arange(data.shape[1])
                data[:, (k > 0) & (k < n - k)] *= 2.0
                data = data.reshape(-1)
        else:
            data = fft_axis(data, ch.layout(li), axis, sign, scale_of(axis))
        first = False
    while cur < len(ch.dirs) - 1:
        data = redistribute(data, ch.layout(cur), ch.layout(cur + 1))
        cur += 1
    return data


def _run_backward(ch: Chain, buf, sign, scale_of, halve):
    sched = transform_schedule(ch.dirs)
    cur = len(ch.dirs) - 1
    data = buf
    for idx, (li, axis) in enumerate(reversed(sched)):
        while cur > li:
            data = redistribute(data, ch.layout(cur), ch.layout(cur - 1))
            cur -= 1
        last = idx == len(sched) - 1
        if ch.kind == "r2r":
            # the adjoint of the forward walks this chain with the forward's transpose
            data = r2r_axis(data, ch.layout(li), axis, ch.r2r[axis], not halve, scale_of(axis), transpose=halve)
        elif last and ch.kind == "r2c":
            data = _c2r_last(data, ch.layout(0, spectral=False), scale_of(axis), halve_interior=halve)
        else:
            data = fft_axis(data, ch.layout(li), axis, sign, scale_of(axis))
    while cur > 0:
        data = redistribute(data, ch.layout(cur), ch.layout(cur - 1))
        cur -= 1
    return data


def _to_stored(ch: Chain, out):
    # the last layout as stored (transposed-out order) from its C-order form
    if not ch.transposed_out:
        return out
    last = len(ch.dirs) - 1
    return relayout(out, ch.layout(last).regular(), ch.layout(last))


def _from_stored(ch: Chain, buf):
    if not ch.transposed_out:
        return buf
    last = len(ch.dirs) - 1
    return relayout(np.asarray(buf), ch.layout(last), ch.layout(last).regular())


def forward(ch: Chain, buf: np.ndarray) -> np.ndarray:
    """Distributed forward transform (Eq. fftn_forward with the chain's
    redistributions, e.g. Eqs. pencil0-pencil2): input in layout 0, output in
    the last layout (as stored)."""
    reg = _regular(ch)
    return _to_stored(ch, _run_forward(reg, buf, -1, lambda a: ch.scale(a, "forward"), "r2c"))


def backward(ch: Chain, buf: np.ndarray) -> np.ndarray:
    """Distributed backward transform (Eq. fftn_backward): the mirror chain."""
    reg = _regular(ch)
    return _run_backward(reg, _from_stored(ch, buf), +1, lambda a: ch.scale(a, "backward"), False)


def adjoint_forward(ch: Chain, buf: np.ndarray) -> np.ndarray:
    """Adjoint of ``forward`` under the real inner product Re<a, b>: reversed
    chain, inverse redistributions, sign +, the forward's per-axis factors.
    For r2c, Re(F^H S^T z): interior bins halved before the c2r."""
    reg = _regular(ch)
    return _run_backward(reg, _from_stored(ch, buf), +1, lambda a: ch.scale(a, "forward"), True)


def adjoint_backward(ch: Chain, buf: np.ndarray) -> np.ndarray:
    """Adjoint of ``backward``: forward chain with sign -, the backward's
    factors; for r2c the c2r's adjoint is an r2c with interior bins doubled."""
    reg = _regular(ch)
    return _to_stored(ch, _run_forward(reg, buf, -1, lambda a: ch.scale(a, "backward"), "r2c_double"))


def wavenumber_weight(spectral_shape, real_last: bool, real_n: int = None, hermitian: bool = True) -> np.ndarray:
    """w(k) = |k|^2 with signed integer wavenumbers (numpy fftfreq * N) on the
    full axes and 0..N/2 on the half axis of a real transform.

    For a real transform (real_last) with ``hermitian`` set, every half-axis
    bin k that stands for two bins of the full spectrum (k and real_n - k,
    i.e. 0 < k < real_n - k) carries twice the weight, so that the weighted
    sum over the stored half spectrum equals the sum over all k of the full
    spectrum.  real_n is the real length of the last axis (default: the even
    length 2 (h - 1) of a half axis of h bins)."""
    ks = []
    d = len(spectral_shape)
    for m, n in enumerate(spectral_shape):
        if real_last and m == d - 1:
            ks.append(np.arange(n, dtype=np.float64))
        else:
            ks.append(np.fft.fftfreq(n, d=1.0 / n))
    grids = np.meshgrid(*ks, indexing="ij")
    w = sum(g * g for g in grids)
    if real_last and hermitian:
        h = spectral_shape[-1]
        rn = 2 * (h - 1) if real_n is None else int(real_n)
        k = np.arange(h)
        w = w * np.where((k > 0) & (k < rn - k), 2.0, 1.0)
    return w


def loss_and_grad(ch: Chain, u_layout0: np.ndarray, w_out_layout: np.ndarray):
    """L = sum_k w(k) |R u|^2 over the stored (half) spectrum, and its gradient
    2 Re(R^H (w * R u)) in the input layout (with the Hermitian weight of
    ``wavenumber_weight``, L is the sum over the full spectrum)."""
    uh = forward(ch, u_layout0)
    loss = float(np.sum(w_out_layout * np.abs(uh) ** 2))
    grad = 2.0 * adjoint_forward(ch, w_out_layout * uh)
    if ch.kind == "c2c":
        return loss, grad
    return loss, np.real(grad)
