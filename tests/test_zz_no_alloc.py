"""The allocation-free energy entry point (pfft_weighted_energy_noalloc,
partial sums in the library's static device scratch) through the C ABI
against pfft_weighted_energy with caller scratch: the same kernels in the same
order, so the losses agree bit for bit, on two calls in a row (the second
with fewer elements, so fewer partial sums than the first call left in the
scratch), and both lie within the FP64 tolerance of numpy."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1804_09536_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_energy_equals_scratch_variant(prec):
    lib = _lib.load()
    cdt, rdt = (np.complex64, np.float32) if prec == "f32" else (np.complex128, np.float64)
    tdt = torch.float32 if prec == "f32" else torch.float64
    pcode = 0 if prec == "f32" else 1
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n in (1_000_003, 4_097):   # 1024 partial sums, then 17
        print("case", prec, n, flush=True)
        u0 = inputs.uniform_complex(n, [41, n], cdt)
        w0 = np.abs(inputs.gaussian_real(n, [42, n], rdt))
        u = torch.from_numpy(u0).cuda()
        w = torch.from_numpy(w0).cuda()
        partials = torch.empty(_lib.ENERGY_PARTIALS, dtype=torch.float64, device="cuda")
        ref = torch.empty((), dtype=tdt, device="cuda")
        got = torch.full((), float("nan"), dtype=tdt, device="cuda")
        _lib.check(lib.pfft_weighted_energy(pcode, n, _p(u), _p(w), _p(partials), _p(ref), stream),
                   "pfft_weighted_energy")
        _lib.check(lib.pfft_weighted_energy_noalloc(pcode, n, _p(u), _p(w), _p(got), stream),
                   "pfft_weighted_energy_noalloc")
        torch.cuda.synchronize()
        assert got.item() == ref.item()
        expect = float(np.sum(w0.astype(np.float64) * np.abs(u0.astype(np.complex128)) ** 2))
        tol = 1e-6 if prec == "f32" else 1e-13
        assert abs(got.item() - expect) <= tol * expect


def test_noalloc_energy_argument_checks():
    lib = _lib.load()
    v = ctypes.c_void_p
    a16 = v(4096)
    assert lib.pfft_weighted_energy_noalloc(2, 4, a16, a16, a16, None) == -4    # bad precision
    assert lib.pfft_weighted_energy_noalloc(0, -1, a16, a16, a16, None) == -1   # negative count
    assert lib.pfft_weighted_energy_noalloc(0, 4, a16, a16, None, None) == -1   # null loss
