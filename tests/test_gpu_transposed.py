"""Transposed output (Sec. 3.2.1, Eq. fftw_transposed_out) on the GPU against
the oracle: the forward output stored with its split axes first, for slabs,
pencils and a 4-D grid, complex and real input, every placement of
intermediates, the backward and both adjoints, and the standalone
redistribution into the transposed layout bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09536_amd import inputs
from paper_1804_09536_amd.plan import Plan

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [
    ((32, 48, 16), (4,), "c2c", "f64", None),
    ((64, 32, 128), (4,), "c2c", "f32", None),
    ((32, 64, 48), (2, 4), "c2c", "f32", None),
    ((16, 24, 32), (3, 2), "c2c", "f64", ("gather", "gather")),
    ((16, 24, 32), (3, 2), "c2c", "f32", ("scatter", "scatter")),
    ((16, 24, 32), (3, 2), "c2c", "f32", ("final", "final")),
    ((8, 16, 12, 32), (2, 2, 3), "c2c", "f32", None),
    ((24, 16, 32), (4,), "r2c", "f32", None),
    ((24, 16, 32), (2, 4), "r2c", "f64", ("scatter", "gather")),
    ((128, 128, 128), (4, 4), "c2c", "f32", None),
    ((96, 48, 40), (4, 2), "c2c", "f32", None),      # 3*2^a lines into the transposed layout
    ((384, 24, 20), (2, 2), "c2c", "f64", None),
    ((2048, 6, 16), (2, 2), "c2c", "f32", None),     # long lines: slot-group shapes (stores point by point)
]


@pytest.mark.parametrize("shape,grid,kind,prec,placement", CASES)
def test_transposed_out_matches_oracle(shape, grid, kind, prec, placement):
    print("case", shape, grid, kind, prec, placement, flush=True)
    p = Plan(shape, grid, kind=kind, precision=prec, placement=placement, transposed_out=True)
    p.validate()
    ch = oracle.Chain.paper(shape, grid, kind=kind, transposed_out=True)
    assert p.axis_order(p.num_layouts - 1) == ch.output_layout().storage
    n = p.buffer_numel(0, real=(kind == "r2c"))
    if kind == "c2c":
        u = inputs.uniform_complex(n, [52, n], np.complex64 if prec == "f32" else np.complex128)
        u64 = u.astype(np.complex128)
    else:
        u = inputs.gaussian_real(n, [52, n], np.float32 if prec == "f32" else np.float64)
        u64 = u.astype(np.float64)
    y = p.forward(torch.from_numpy(u).cuda())
    got = _host(y)
    assert relerr(got, oracle.forward(ch, u64)) <= TOL[prec]
    g = got.astype(np.complex128)
    assert relerr(_host(p.backward(y)), oracle.backward(ch, g)) <= TOL[prec]
    assert relerr(_host(p.adjoint_forward(y)), oracle.adjoint_forward(ch, g)) <= TOL[prec]
    assert relerr(_host(p.adjoint_backward(torch.from_numpy(u).cuda())), oracle.adjoint_backward(ch, u64)) <= TOL[prec]


@pytest.mark.parametrize("shape,grid", [((12, 8, 10), (4,)), ((10, 12, 14), (2, 3)), ((6, 8, 4, 10), (2, 2, 2))])
def test_redistribute_into_transposed_layout_bit_exact(shape, grid):
    print("case", shape, grid, flush=True)
    p = Plan(shape, grid, transposed_out=True, layouts_only=True)
    ch = oracle.Chain.paper(shape, grid, transposed_out=True)
    last = p.num_layouts - 1
    payload = inputs.index_payload(p.buffer_numel(last - 1), np.complex64)
    out = p.empty(last)
    out.fill_(complex(float("nan"), float("nan")))
    y = p.redistribute(torch.from_numpy(payload).cuda(), last - 1, last, out=out)
    expect = oracle.redistribute(payload, ch.layout(last - 1), ch.layout(last))
    assert _host(y).tobytes() == expect.tobytes()
    back = _host(p.redistribute(y, last, last - 1))
    assert back.tobytes() == payload.tobytes()
