"""Lengths without a register radix plan run through the LDS mixed-radix
kernel (radix 2/3/4/5/7 butterflies, a direct butterfly for other small
primes, Bluestein's convolution for lines with a prime factor above 32): the
paper's two appendix programs on the GPU (42x127x256 on 2-D grids and
16x17x18x19 on 3-D grids, complex128, filled with j + j*I, forward then
backward to 1e-8), their forward results against the oracle, odd-length real
transforms, and long or prime lengths on strided and contiguous axes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09536_amd import inputs
from paper_1804_09536_amd.plan import Plan

pytestmark = pytest.mark.gpu


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("shape,grid", [((42, 127, 256), (2, 2)), ((42, 127, 256), (3, 4)),
                                        ((16, 17, 18, 19), (2, 2, 2)), ((16, 17, 18, 19), (1, 2, 3))])
def test_appendix_programs_on_gpu(shape, grid):
    print("case", shape, grid, flush=True)
    p = Plan(shape, grid, precision="f64")
    ch = oracle.Chain.paper(shape, grid)
    P = int(np.prod(grid))
    sizes = [int(np.prod(p.local_block(0, r)[0])) for r in range(P)]
    a = inputs.local_index_fill(sizes)
    y = p.forward(torch.from_numpy(a).cuda())
    z = _host(p.backward(y))
    j = a.real
    assert np.all(np.abs(z.real - j) < 1e-8) and np.all(np.abs(z.imag - j) < 1e-8)
    got = _host(y)
    expect = oracle.forward(ch, a)
    assert np.linalg.norm(got - expect) / np.linalg.norm(expect) <= 1e-12


@pytest.mark.parametrize("shape,grid,prec", [((9, 10, 15), (2, 2), "f64"), ((8, 6, 7), (2,), "f64"),
                                             ((12, 20, 14), (3, 2), "f32"), ((5, 7, 6), (2, 3), "f32")])
def test_general_length_real_and_complex(shape, grid, prec):
    print("case", shape, grid, prec, flush=True)
    tol = 1e-12 if prec == "f64" else 1e-5
    for kind in ("c2c", "r2c"):
        p = Plan(shape, grid, precision=prec, kind=kind)
        ch = oracle.Chain.paper(shape, grid, kind=kind)
        if kind == "c2c":
            x = inputs.uniform_complex(p.buffer_numel(0), [40], np.complex64 if prec == "f32" else np.complex128)
            x64 = x.astype(np.complex128)
        else:
            x = inputs.gaussian_real(p.buffer_numel(0, real=True), [40], np.float32 if prec == "f32" else np.float64)
            x64 = x.astype(np.float64)
        y = p.forward(torch.from_numpy(x).cuda())
        got = _host(y)
        e = oracle.forward(ch, x64)
        assert np.linalg.norm(got - e) / np.linalg.norm(e) <= tol
        back = _host(p.backward(y))
        e = oracle.backward(ch, got.astype(np.complex128))
        assert np.linalg.norm(back - e) / np.linalg.norm(e) <= tol
        adj = _host(p.adjoint_forward(y))
        e = oracle.adjoint_forward(ch, got.astype(np.complex128))
        assert np.linalg.norm(adj - e) / np.linalg.norm(e) <= tol


# (length, precision): 5- and 7-smooth lengths, small primes (direct
# butterfly), primes and lengths with a prime factor above 32 (Bluestein),
# powers of two and 3 * 2^a past the register kernels
MIXED = [(5, "f64"), (7, "f32"), (25, "f32"), (35, "f64"), (49, "f32"), (125, "f64"), (1000, "f32"),
         (1000, "f64"), (1001, "f32"), (2310, "f32"), (127, "f64"), (127, "f32"), (1009, "f32"), (74, "f64"),
         (4099, "f32"), (2053, "f64"), (8192, "f32"), (6144, "f32")]


@pytest.mark.parametrize("mode", ["strided", "contig"])
@pytest.mark.parametrize("N,prec", MIXED)
def test_mixed_radix_and_bluestein_lengths(N, prec, mode):
    shape, grid = ((N, 4, 6), (2, 2)) if mode == "strided" else ((4, 6, N), (2, 2))
    print("case", shape, grid, prec, flush=True)
    tol = 1e-12 if prec == "f64" else 1e-5
    p = Plan(shape, grid, precision=prec)
    p.validate()
    ch = oracle.Chain.paper(shape, grid)
    x = inputs.uniform_complex(p.buffer_numel(0), [43, N], np.complex64 if prec == "f32" else np.complex128)
    y = p.forward(torch.from_numpy(x).cuda())
    got = _host(y)
    e = oracle.forward(ch, x.astype(np.complex128))
    assert np.linalg.norm(got - e) / np.linalg.norm(e) <= tol
    back = _host(p.backward(y))
    e = oracle.backward(ch, got.astype(np.complex128))
    assert np.linalg.norm(back - e) / np.linalg.norm(e) <= tol


@pytest.mark.parametrize("N,prec", [(127, "f64"), (1000, "f32"), (254, "f32"), (1009, "f64"), (75, "f32")])
def test_mixed_radix_real_transforms(N, prec):
    # r2c / c2r and their adjoints along a last axis without a radix plan
    shape, grid = (6, 4, N), (2, 2)
    print("case", shape, grid, prec, flush=True)
    tol = 1e-12 if prec == "f64" else 1e-5
    p = Plan(shape, grid, precision=prec, kind="r2c")
    p.validate()
    ch = oracle.Chain.paper(shape, grid, kind="r2c")
    x = inputs.gaussian_real(p.buffer_numel(0, real=True), [44, N], np.float32 if prec == "f32" else np.float64)
    y = p.forward(torch.from_numpy(x).cuda())
    got = _host(y)
    e = oracle.forward(ch, x.astype(np.float64))
    assert np.linalg.norm(got - e) / np.linalg.norm(e) <= tol
    g = got.astype(np.complex128)
    for fn, ref in ((p.backward, oracle.backward), (p.adjoint_forward, oracle.adjoint_forward)):
        out = _host(fn(y))
        e = ref(ch, g)
        assert np.linalg.norm(out - e) / np.linalg.norm(e) <= tol
    adj = _host(p.adjoint_backward(torch.from_numpy(x).cuda()))
    e = oracle.adjoint_backward(ch, x.astype(np.float64))
    assert np.linalg.norm(adj - e) / np.linalg.norm(e) <= tol
