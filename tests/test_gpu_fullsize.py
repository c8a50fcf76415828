"""Parity at the full workload sizes, in the launch configuration the bench
times (default tiles, placements and XCD tile order): every output element of
the forward against the oracle (Eq. multifft through the chain of Eqs.
pencil0-pencil2 / 4d_fft0-4d_fft3), the backward against the oracle on the
GPU's own forward output (Eq. fftn_backward), the round trip, and a few bins
against direct sums of the definition that do not go through the oracle's
chain at all."""
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


FULL = [
    ((512, 512, 512), (8, 8), "c2c", "f32", 4),       # the metric workload (seed as in the bench)
    ((256, 256, 256), (4, 4), "c2c", "f32", 1),
    ((512, 512, 512), (8, 8), "r2c", "f32", 2),
    ((64, 64, 64, 64), (2, 2, 4), "c2c", "f32", 3),
    ((512, 512, 512), (8, 8), "c2c", "f64", 4),
]


@pytest.mark.parametrize("shape,grid,kind,prec,seed", FULL)
def test_full_size_matches_oracle(shape, grid, kind, prec, seed):
    print("case", shape, grid, kind, prec, flush=True)
    p = Plan(shape, grid, kind=kind, precision=prec)
    ch = oracle.Chain.paper(shape, grid, kind=kind)
    n = p.buffer_numel(0, real=(kind == "r2c"))
    if kind == "c2c":
        u = inputs.uniform_complex(n, [seed], np.complex64 if prec == "f32" else np.complex128)
        u64 = u.astype(np.complex128)
    else:
        u = inputs.gaussian_real(n, [seed], np.float32 if prec == "f32" else np.float64)
        u64 = u.astype(np.float64)
    x = torch.from_numpy(u).to("cuda")
    del u
    y = p.forward(x)
    yh = _host(y)
    print("  forward done", flush=True)
    expect = oracle.forward(ch, u64)
    assert relerr(yh, expect) <= TOL[prec]
    # a few bins straight from the definition (independent of the oracle's chain)
    G = oracle.gather_global(u64, ch.layout(0, spectral=(kind == "c2c")))
    rng = np.random.default_rng(seed + 100)
    spec = ch.spectral_shape()
    bins = [tuple(int(rng.integers(0, s)) for s in spec) for _ in range(3)] + [tuple(0 for _ in spec)]
    direct = oracle.dft_bins(G, bins, -1, 1.0 / float(np.prod(shape)))
    del G
    lay = ch.output_layout()
    got = np.array([yh[oracle.layout_offset(lay, b)] for b in bins])
    assert relerr(got, direct) <= TOL[prec]
    del expect
    # the backward alone, on the GPU's own forward output
    z = p.backward(y)
    zh = _host(z)
    print("  backward done", flush=True)
    expect_b = oracle.backward(ch, yh.astype(np.complex128))
    assert relerr(zh, expect_b) <= TOL[prec]
    del expect_b
    assert relerr(zh, u64) <= TOL[prec]


@pytest.mark.parametrize("shape,grid,kind", [((512, 512, 512), (8, 8), "c2c"), ((512, 512, 512), (8, 8), "r2c")])
def test_full_size_tile_order_and_placement_are_result_neutral(shape, grid, kind):
    # at 1 GiB per buffer the forward axis-1 stage of the default c2c placement
    # (stores straight into the next layout) hands each XCD a contiguous range
    # of tiles; the gather placement and the order forced off keep the
    # round-robin order: every line sees the same arithmetic, so the outputs
    # agree bit for bit
    print("case", shape, grid, kind, flush=True)
    a = Plan(shape, grid, kind=kind)
    b = Plan(shape, grid, kind=kind, placement=("gather", "gather"))
    c = Plan(shape, grid, kind=kind)
    c.set_tuning(xcd_order=2)
    if kind == "c2c":
        x = inputs.uniform_complex_device(a.buffer_numel(0), 4, torch.complex64, torch.device("cuda"))
    else:
        g = torch.Generator(device="cuda")
        g.manual_seed(2)
        x = torch.randn(a.buffer_numel(0, real=True), dtype=torch.float32, device="cuda", generator=g)
    ya = a.forward(x)
    for other in (b, c):
        assert torch.equal(ya, other.forward(x))
    za = a.backward(ya)
    for other in (b, c):
        assert torch.equal(za, other.backward(ya))
