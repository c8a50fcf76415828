"""GPU parity of the real-input path (r2c forward, c2r backward) and of the
adjoint chains against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09536_amd import inputs
from paper_1804_09536_amd.plan import Plan

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}
RDT = {"f32": np.float32, "f64": np.float64}
CDT = {"f32": np.complex64, "f64": np.complex128}


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


R2C = [
    ((16, 16, 16), (4, 4), "f64"),
    ((64, 32, 512), (8, 8), "f32"),      # 257 bins over 8: 33 + 7 x 32
    ((8, 16, 4, 32), (3, 1, 5), "f32"),  # 4-D, uneven
    ((6, 12, 8), (2,), "f64"),           # slab, radix-3 lengths
    ((4, 2, 8), (8, 3), "f32"),          # empty blocks
    ((32, 24, 96), (4, 2), "f32"),
]


@pytest.mark.parametrize("shape,grid,prec", R2C)
def test_r2c_c2r_match_oracle(shape, grid, prec):
    print("case", shape, grid, prec, flush=True)
    p = Plan(shape, grid, precision=prec, kind="r2c")
    ch = oracle.Chain.paper(shape, grid, kind="r2c")
    x = inputs.gaussian_real(p.buffer_numel(0, real=True), [20, 1], RDT[prec])
    y = p.forward(_dev(x))
    got = _host(y)
    assert relerr(got, oracle.forward(ch, x.astype(np.float64))) <= TOL[prec]
    back = _host(p.backward(y))
    assert relerr(back, oracle.backward(ch, got.astype(np.complex128))) <= TOL[prec]
    assert relerr(back, x.astype(np.float64)) <= TOL[prec]


def test_c2r_ignores_imaginary_dc_and_nyquist():
    shape, grid = (8, 8, 16), (2, 2)
    p = Plan(shape, grid, precision="f64", kind="r2c")
    ch = oracle.Chain.paper(shape, grid, kind="r2c")
    z = inputs.uniform_complex(p.buffer_numel(p.num_layouts - 1), [21], np.complex128)  # not Hermitian
    got = _host(p.backward(_dev(z)))
    assert relerr(got, oracle.backward(ch, z)) <= 1e-12


ADJ = [
    ((16, 8, 32), (2, 4), "c2c", "f64", "forward"),
    ((16, 8, 32), (2, 4), "c2c", "f32", "backward"),
    ((16, 16, 16), (4, 4), "r2c", "f64", "forward"),
    ((32, 24, 96), (4, 2), "r2c", "f32", "forward"),
    ((8, 16, 4, 32), (3, 1, 5), "r2c", "f64", "none"),
]


@pytest.mark.parametrize("shape,grid,kind,prec,norm", ADJ)
def test_adjoints_match_oracle(shape, grid, kind, prec, norm):
    print("case", shape, grid, kind, prec, norm, flush=True)
    p = Plan(shape, grid, precision=prec, kind=kind, norm=norm)
    ch = oracle.Chain.paper(shape, grid, kind=kind, norm=norm)
    last = p.num_layouts - 1
    z = inputs.uniform_complex(p.buffer_numel(last), [22, 0], CDT[prec])
    got = _host(p.adjoint_forward(_dev(z)))
    assert relerr(got, oracle.adjoint_forward(ch, z.astype(np.complex128))) <= TOL[prec]
    if kind == "c2c":
        x = inputs.uniform_complex(p.buffer_numel(0), [22, 1], CDT[prec])
    else:
        x = inputs.gaussian_real(p.buffer_numel(0, real=True), [22, 1], RDT[prec])
    got = _host(p.adjoint_backward(_dev(x)))
    expect = oracle.adjoint_backward(ch, x.astype(np.complex128 if kind == "c2c" else np.float64))
    assert relerr(got, expect) <= TOL[prec]


@pytest.mark.parametrize("kind", ["c2c", "r2c"])
def test_gpu_dot_product_identity(kind):
    # <F x, z> = <x, F^H z> (real part for r2c) on the GPU's own outputs
    shape, grid = (16, 32, 16), (4, 2)
    p = Plan(shape, grid, precision="f64", kind=kind)
    last = p.num_layouts - 1
    z = inputs.uniform_complex(p.buffer_numel(last), [23, 0], np.complex128)
    if kind == "c2c":
        x = inputs.uniform_complex(p.buffer_numel(0), [23, 1], np.complex128)
    else:
        x = inputs.gaussian_real(p.buffer_numel(0, real=True), [23, 1], np.float64)
    fx = _host(p.forward(_dev(x)))
    fhz = _host(p.adjoint_forward(_dev(z)))
    lhs = np.vdot(fx, z)
    rhs = np.vdot(x, fhz)
    if kind == "r2c":
        lhs, rhs = lhs.real, rhs.real
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
