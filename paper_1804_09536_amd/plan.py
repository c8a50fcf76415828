"""Python face of libpfft: a ``Plan`` holding a C plan, its device state and
workspace, with methods that pass torch tensors' device pointers and the
current HIP stream to the C ABI.  PyTorch supplies device memory and streams
only; every step of the transform runs in libpfft's kernels.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import PATHS, NORMS, check

_DT = {
    ("c2c", "f32"): (torch.complex64, torch.complex64),
    ("c2c", "f64"): (torch.complex128, torch.complex128),
    ("r2c", "f32"): (torch.float32, torch.complex64),
    ("r2c", "f64"): (torch.float64, torch.complex128),
    ("r2r", "f32"): (torch.float32, torch.float32),
    ("r2r", "f64"): (torch.float64, torch.float64),
}
R2R_KINDS = {"dct2": 0, "dst2": 1}


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """A distributed multidimensional FFT over a virtual process grid.

    shape: global array shape (the real shape for kind="r2c").
    kind: "c2c", "r2c" or "r2r" (real-to-real: the argument r2r names the
          forward transform of each axis, "dct2" or "dst2"; the backward
          applies the inverse of type III).
    grid: virtual process grid dims (1 <= len(grid) < len(shape)).
    precision: "f32" (complex64) or "f64" (complex128).
    norm: "forward" (the paper's), "backward", "none".
    chain: None for the paper's rule, else [(grid_dir, new_axis), ...].
    path: "fused" (redistribution fused into the transform's load),
          "unfused" (standalone redistribution kernel) or "pack_realign"
          (local transpose + contiguous exchange + realign).
    layouts_only: plan layouts and redistributions only (any lengths); the
          transforms then raise.
    placement: where partial results are stored on the fused path: "gather"
          (in the layout where they were computed; the next stage gathers),
          "scatter" (in the next stage's layout), "direct" (the first in its
          own layout, later ones in the final layout: the chain's middle
          alignments are never stored) or "final" (all in the final layout);
          one name for both chains or a (forward, backward) pair.  Same
          results; different access patterns.  The default pair is the
          fastest measured per kind on the 512^3 pencil workloads.
    destroy_input: the transforms may overwrite a complex input and use it
          for intermediates (no workspace for most c2c plans, one buffer
          instead of two for r2c); a real input is never written.
    transposed_out: the forward output's blocks store their split axes first
          (the paper's transposed-out alignment; see ``axis_order``).
    """

    DEFAULT_PLACEMENT = {"c2c": ("direct", "gather"), "r2c": ("scatter", "gather"), "r2r": ("direct", "gather")}

    def __init__(self, shape: Sequence[int], grid: Sequence[int], precision: str = "f32", kind: str = "c2c",
                 norm: str = "forward", chain=None, path: str = "fused", device=None,
                 layouts_only: bool = False, placement=None, destroy_input: bool = False, r2r=None,
                 transposed_out: bool = False):
        lib = _lib.load()
        self.shape = tuple(int(x) for x in shape)
        self.grid = tuple(int(x) for x in grid)
        self.precision, self.kind, self.norm, self.path = precision, kind, norm, path
        self.destroy_input = bool(destroy_input)
        self.transposed_out = bool(transposed_out)
        if placement is None:
            # with the transposed output on grids of two or more directions, the
            # forward keeps its intermediates (gather) and the backward stores
            # them in the next stage's layout (scatter): every stage then has
            # lines that step alike on both sides or a transposing stage kernel
            placement = (("gather", "scatter") if transposed_out and len(grid) > 1
                         else self.DEFAULT_PLACEMENT[kind])
        self.placement = (placement, placement) if isinstance(placement, str) else tuple(placement)
        if len(self.placement) != 2 or any(p not in _lib.PLACEMENTS for p in self.placement):
            raise ValueError("placement must be one of %s or a pair of them" % sorted(_lib.PLACEMENTS))
        self.chain = None if chain is None else [tuple(int(v) for v in s) for s in chain]
        self.device = torch.device(device if device is not None else "cuda")
        self.in_dtype, self.spec_dtype = _DT[(kind, precision)]
        if kind == "r2r":
            self.r2r = tuple(r2r) if r2r is not None else ("dct2",) * len(self.shape)
            if len(self.r2r) != len(self.shape) or any(k not in R2R_KINDS for k in self.r2r):
                raise ValueError("r2r: one of %s per axis" % sorted(R2R_KINDS))
        else:
            self.r2r = None
        h = ctypes.c_void_p()
        shp = (ctypes.c_int64 * len(self.shape))(*self.shape)
        grd = (ctypes.c_int * len(self.grid))(*self.grid)
        if self.chain is None:
            ch, nsteps = None, 0
        else:
            flat = [v for s in self.chain for v in s]
            ch, nsteps = (ctypes.c_int * max(1, len(flat)))(*flat), len(self.chain)
        flags = (PATHS[path] | (_lib.PFFT_LAYOUTS_ONLY if layouts_only else 0)
                 | (_lib.PLACEMENTS[self.placement[0]] << 3) | (_lib.PLACEMENTS[self.placement[1]] << 5)
                 | (_lib.PFFT_DESTROY_INPUT if self.destroy_input else 0)
                 | (_lib.PFFT_TRANSPOSED_OUT if self.transposed_out else 0))
        prec = 0 if precision == "f32" else 1
        if kind == "r2r":
            kinds = (ctypes.c_int * len(self.shape))(*[R2R_KINDS[k] for k in self.r2r])
            st = lib.pfft_plan_create_r2r(ctypes.byref(h), len(self.shape), shp, len(self.grid), grd, prec, kinds,
                                          NORMS[norm], ch, nsteps, flags)
            check(st, "pfft_plan_create_r2r")
        else:
            st = lib.pfft_plan_create(ctypes.byref(h), len(self.shape), shp, len(self.grid), grd, prec,
                                      {"c2c": 0, "r2c": 1}[kind], NORMS[norm], ch, nsteps, flags)
            check(st, "pfft_plan_create")
        self._h = h
        n = ctypes.c_int()
        check(lib.pfft_num_layouts(h, ctypes.byref(n)), "pfft_num_layouts")
        self.num_layouts = n.value
        self._state = None
        self.tuned = False  # knobs set from the autotuner's table (tune.tuned_plan)
        self._work = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.pfft_plan_destroy(h)
            self._h = None

    # ------------------------------------------------------------ layouts --
    def local_block(self, layout: int, rank: int, real: bool = False):
        lib = _lib.load()
        nd = len(self.shape)
        shp = (ctypes.c_int64 * nd)()
        sta = (ctypes.c_int64 * nd)()
        off = ctypes.c_int64()
        check(lib.pfft_local_block(self._h, layout, int(real), rank, shp, sta, ctypes.byref(off)),
              "pfft_local_block")
        return tuple(shp), tuple(sta), off.value

    def axis_order(self, layout: int):
        """Storage order of the layout's blocks: the axis at each position of
        the block's C-order index."""
        nd = len(self.shape)
        out = (ctypes.c_int * nd)()
        check(_lib.load().pfft_layout_axis_order(self._h, layout, out), "pfft_layout_axis_order")
        return tuple(out)

    def buffer_numel(self, layout: int, real: bool = False) -> int:
        lib = _lib.load()
        b = ctypes.c_size_t()
        check(lib.pfft_buffer_bytes(self._h, layout, int(real), ctypes.byref(b)), "pfft_buffer_bytes")
        esize = torch.empty(0, dtype=self.in_dtype if real else self.spec_dtype).element_size()
        return b.value // esize

    def device_state_bytes(self) -> int:
        b = ctypes.c_size_t()
        check(_lib.load().pfft_device_state_bytes(self._h, ctypes.byref(b)), "pfft_device_state_bytes")
        return b.value

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t()
        check(_lib.load().pfft_workspace_bytes(self._h, ctypes.byref(b)), "pfft_workspace_bytes")
        return b.value

    def validate(self):
        """Host emulation of every kernel's addressing (bounds, write-once)."""
        check(_lib.load().pfft_validate_plan(self._h), "pfft_validate_plan")
        return self

    def tuning(self) -> dict:
        t = _lib.Tuning()
        check(_lib.load().pfft_plan_get_tuning(self._h, ctypes.byref(t)), "pfft_plan_get_tuning")
        return {f: getattr(t, f) for f, _ in _lib.Tuning._fields_}

    def set_tuning(self, **knobs):
        """Change kernel tile shapes / grid policy / radix plan (see
        pfft_tuning); results do not change beyond rounding (bitwise equal
        except for radix_alt).  Drops the bound device state (rebound on next
        use)."""
        cur = self.tuning()
        cur.update(knobs)
        t = _lib.Tuning(**cur)
        check(_lib.load().pfft_plan_set_tuning(self._h, ctypes.byref(t)), "pfft_plan_set_tuning")
        self._state = None
        return self

    def set_profiling(self, enable: bool = True):
        check(_lib.load().pfft_set_profiling(self._h, int(enable)), "pfft_set_profiling")

    def profile_read(self, max_entries: int = 65536):
        """Per-launch records of the calls since the last read (waits for them)."""
        buf = (_lib.ProfileEntry * max_entries)()
        n = ctypes.c_int()
        check(_lib.load().pfft_profile_read(self._h, max_entries, buf, ctypes.byref(n)), "pfft_profile_read")
        kinds = {0: "c2c", 1: "copy", 2: "r2c", 3: "c2r", 4: "r2r"}
        return [dict(kind=kinds.get(e.kind, "?"), axis=e.axis, contig=bool(e.contig), length=e.length,
                     direction=e.direction, ms=e.ms, bytes=e.bytes) for e in buf[:min(n.value, max_entries)]]

    # ----------------------------------------------------- device binding --
    def bind(self):
        """Allocate (through torch) and upload the plan's device tables."""
        if self._state is None:
            nbytes = max(256, self.device_state_bytes())
            self._state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            check(_lib.load().pfft_bind_device_state(self._h, _ptr(self._state), _stream_handle(self.device)),
                  "pfft_bind_device_state")
        return self

    def workspace(self):
        """The plan's workspace tensor (allocated once), or None if the
        transforms need none."""
        if self._work is None:
            nbytes = self.workspace_bytes()
            if nbytes == 0:
                return None
            self._work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._work

    def empty(self, layout: int, real: bool = False) -> torch.Tensor:
        dt = self.in_dtype if real else self.spec_dtype
        return torch.empty(self.buffer_numel(layout, real), dtype=dt, device=self.device)

    # ---------------------------------------------------------- transforms --
    def _check_in(self, x: torch.Tensor, layout: int, real: bool):
        dt = self.in_dtype if real else self.spec_dtype
        if x.dtype != dt:
            raise TypeError("expected %s, got %s" % (dt, x.dtype))
        if not x.is_cuda or not x.is_contiguous():
            raise ValueError("expected a contiguous device tensor")
        if x.numel() != self.buffer_numel(layout, real):
            raise ValueError("expected %d elements, got %d" % (self.buffer_numel(layout, real), x.numel()))

    def _run(self, fn, x, out, work, in_real, out_real, in_layout, out_layout, name):
        self.bind()
        self._check_in(x, in_layout, in_real)
        if out is None:
            out = self.empty(out_layout, out_real)
        else:
            self._check_in(out, out_layout, out_real)
        if work is None:
            work = self.workspace()
        check(fn(self._h, _ptr(x), _ptr(out), _ptr(work), _stream_handle(self.device)), name)
        return out

    def forward(self, x: torch.Tensor, out=None, work=None) -> torch.Tensor:
        lib = _lib.load()
        r = self.kind == "r2c"
        return self._run(lib.pfft_forward, x, out, work, r, False, 0, self.num_layouts - 1, "pfft_forward")

    def backward(self, x: torch.Tensor, out=None, work=None) -> torch.Tensor:
        lib = _lib.load()
        r = self.kind == "r2c"
        return self._run(lib.pfft_backward, x, out, work, False, r, self.num_layouts - 1, 0, "pfft_backward")

    def adjoint_forward(self, x: torch.Tensor, out=None, work=None) -> torch.Tensor:
        lib = _lib.load()
        r = self.kind == "r2c"
        return self._run(lib.pfft_adjoint_forward, x, out, work, False, r, self.num_layouts - 1, 0,
                         "pfft_adjoint_forward")

    def adjoint_backward(self, x: torch.Tensor, out=None, work=None) -> torch.Tensor:
        lib = _lib.load()
        r = self.kind == "r2c"
        return self._run(lib.pfft_adjoint_backward, x, out, work, r, False, 0, self.num_layouts - 1,
                         "pfft_adjoint_backward")

    def redistribute(self, x: torch.Tensor, layout_from: int, layout_to: int, out=None) -> torch.Tensor:
        lib = _lib.load()
        self.bind()
        self._check_in(x, layout_from, False)
        if out is None:
            out = self.empty(layout_to)
        else:
            self._check_in(out, layout_to, False)
        check(lib.pfft_redistribute(self._h, layout_from, layout_to, _ptr(x), _ptr(out),
                                    _stream_handle(self.device)), "pfft_redistribute")
        return out


class Batch:
    """Several plans executed together (see pfft_batch_* in include/pfft.h):
    one launch per (stage, kernel shape) over every member's tiles.  The batch
    owns one input, one output and one workspace buffer; ``inputs[m]`` and
    ``outputs[m]`` are views of member m's regions."""

    def __init__(self, plans, device=None):
        lib = _lib.load()
        self.plans = list(plans)
        self.device = torch.device(device if device is not None else self.plans[0].device)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        check(lib.pfft_batch_create(ctypes.byref(h), len(self.plans), arr), "pfft_batch_create")
        self._h = h
        ib, ob, wb, sb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        check(lib.pfft_batch_buffer_bytes(h, ctypes.byref(ib), ctypes.byref(ob), ctypes.byref(wb)),
              "pfft_batch_buffer_bytes")
        check(lib.pfft_batch_device_state_bytes(h, ctypes.byref(sb)), "pfft_batch_device_state_bytes")
        self.in_buf = torch.empty(ib.value, dtype=torch.uint8, device=self.device)
        self.out_buf = torch.empty(ob.value, dtype=torch.uint8, device=self.device)
        self.work_buf = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        self.state = torch.empty(max(256, sb.value), dtype=torch.uint8, device=self.device)
        check(lib.pfft_batch_bind(h, _ptr(self.state), _ptr(self.in_buf), _ptr(self.out_buf), _ptr(self.work_buf),
                                  _stream_handle(self.device)), "pfft_batch_bind")
        self.inputs, self.outputs = [], []
        for m, p in enumerate(self.plans):
            io, oo = ctypes.c_size_t(), ctypes.c_size_t()
            check(lib.pfft_batch_member_offsets(h, m, ctypes.byref(io), ctypes.byref(oo)), "pfft_batch_member_offsets")
            real = p.kind == "r2c"
            n_in = p.buffer_numel(0, real=real)
            n_out = p.buffer_numel(p.num_layouts - 1)
            isz = torch.empty(0, dtype=p.in_dtype).element_size()
            osz = torch.empty(0, dtype=p.spec_dtype).element_size()
            self.inputs.append(self.in_buf[io.value:io.value + n_in * isz].view(p.in_dtype))
            self.outputs.append(self.out_buf[oo.value:oo.value + n_out * osz].view(p.spec_dtype))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.pfft_batch_destroy(h)
            self._h = None

    def forward(self):
        """Every member's forward transform: inputs[m] -> outputs[m]."""
        check(_lib.load().pfft_batch_execute(self._h, 0, _stream_handle(self.device)), "pfft_batch_execute")

    def backward(self):
        """Every member's backward transform: outputs[m] -> inputs[m]."""
        check(_lib.load().pfft_batch_execute(self._h, 1, _stream_handle(self.device)), "pfft_batch_execute")
