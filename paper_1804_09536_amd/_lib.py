"""ctypes binding of libpfft.so (argument marshalling only).

The library is built in-tree by ``paper_1804_09536_amd.build``; if it is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfft.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pfft.h")

PFFT_C2C, PFFT_R2C = 0, 1
PFFT_F32, PFFT_F64 = 0, 1
NORMS = {"forward": 0, "backward": 1, "none": 2}
PATHS = {"fused": 0, "unfused": 1, "pack_realign": 2}
PFFT_LAYOUTS_ONLY = 4
PFFT_PLACE_SCATTER = 8
PFFT_DESTROY_INPUT = 1 << 8
PFFT_TRANSPOSED_OUT = 1 << 9
ENERGY_PARTIALS = 1024  # PFFT_ENERGY_PARTIALS: FP64 scratch of pfft_weighted_energy
PLACEMENTS = {"gather": 0, "scatter": 1, "direct": 2, "final": 3}

_lib = None


class Tuning(ctypes.Structure):
    _fields_ = [("tile_contig", ctypes.c_int), ("tile_strided", ctypes.c_int),
                ("resident_contig", ctypes.c_int), ("resident_strided", ctypes.c_int),
                ("xcd_order", ctypes.c_int), ("stream_strided", ctypes.c_int), ("wide_offsets", ctypes.c_int),
                ("radix_alt", ctypes.c_int), ("stream_contig", ctypes.c_int)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("axis", ctypes.c_int), ("contig", ctypes.c_int),
                ("length", ctypes.c_int), ("direction", ctypes.c_int), ("ms", ctypes.c_float),
                ("bytes", ctypes.c_double)]


class PfftError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        msg = "%s failed: %s (%d)" % (where, strerror(status), status)
        if detail:
            msg += ": " + detail
        super().__init__(msg)


def load():
    """Load libpfft.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError("libpfft.so not found at %s; build it with `python -m paper_1804_09536_amd.build`"
                      % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64p, ip, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int), ctypes.c_size_t
    c_int = ctypes.c_int
    sigs = {
        "pfft_plan_create": [ctypes.POINTER(vp), c_int, i64p, c_int, ip, c_int, c_int, c_int, ip, c_int,
                             ctypes.c_uint],
        "pfft_plan_create_r2r": [ctypes.POINTER(vp), c_int, i64p, c_int, ip, c_int, ip, c_int, ip, c_int,
                                 ctypes.c_uint],
        "pfft_plan_destroy": [vp],
        "pfft_plan_set_tuning": [vp, ctypes.POINTER(Tuning)],
        "pfft_plan_get_tuning": [vp, ctypes.POINTER(Tuning)],
        "pfft_validate_plan": [vp],
        "pfft_num_layouts": [vp, ip],
        "pfft_local_block": [vp, c_int, c_int, c_int, i64p, i64p, i64p],
        "pfft_layout_axis_order": [vp, c_int, ip],
        "pfft_buffer_bytes": [vp, c_int, c_int, ctypes.POINTER(sz)],
        "pfft_device_state_bytes": [vp, ctypes.POINTER(sz)],
        "pfft_bind_device_state": [vp, vp, vp],
        "pfft_workspace_bytes": [vp, ctypes.POINTER(sz)],
        "pfft_redistribute": [vp, c_int, c_int, vp, vp, vp],
        "pfft_batch_create": [ctypes.POINTER(vp), c_int, ctypes.POINTER(vp)],
        "pfft_batch_destroy": [vp],
        "pfft_batch_buffer_bytes": [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "pfft_batch_member_offsets": [vp, c_int, ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "pfft_batch_device_state_bytes": [vp, ctypes.POINTER(sz)],
        "pfft_batch_bind": [vp, vp, vp, vp, vp, vp],
        "pfft_batch_execute": [vp, c_int, vp],
        "pfft_forward": [vp, vp, vp, vp, vp],
        "pfft_backward": [vp, vp, vp, vp, vp],
        "pfft_adjoint_forward": [vp, vp, vp, vp, vp],
        "pfft_adjoint_backward": [vp, vp, vp, vp, vp],
        "pfft_weighted_energy": [c_int, ctypes.c_int64, vp, vp, vp, vp, vp],
        "pfft_weighted_energy_grad": [c_int, ctypes.c_int64, vp, vp, vp, vp, vp],
        "pfft_weighted_energy_noalloc": [c_int, ctypes.c_int64, vp, vp, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c_int
    lib.pfft_set_profiling.argtypes = [vp, c_int]
    lib.pfft_set_profiling.restype = c_int
    lib.pfft_profile_read.argtypes = [vp, c_int, ctypes.POINTER(ProfileEntry), ip]
    lib.pfft_profile_read.restype = c_int
    lib.pfft_strerror.argtypes = [c_int]
    lib.pfft_strerror.restype = ctypes.c_char_p
    lib.pfft_last_error.argtypes = []
    lib.pfft_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().pfft_strerror(int(status)).decode()


def check(status: int, where: str):
    if status != 0:
        raise PfftError(status, where, load().pfft_last_error().decode())


def header_functions():
    """Names of the functions declared in include/pfft.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pfft_[a-z_0-9]+)\s*\(", text)))
