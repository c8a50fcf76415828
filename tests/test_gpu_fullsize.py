"""Parity at the full workload sizes, in the launch configuration the bench
times: sampled output bins against the oracle's direct sums of Eq. multifft,
plus properties that hold at any size (round trip, Parseval)."""
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


FULL = [
    ((512, 512, 512), (8, 8), "c2c", 4),       # the metric workload (seed as in the bench)
    ((256, 256, 256), (4, 4), "c2c", 1),
    ((512, 512, 512), (8, 8), "r2c", 2),
    ((64, 64, 64, 64), (2, 2, 4), "c2c", 3),
]


@pytest.mark.parametrize("shape,grid,kind,seed", FULL)
def test_full_size_sampled_bins_and_properties(shape, grid, kind, seed):
    print("case", shape, grid, kind, flush=True)
    p = Plan(shape, grid, kind=kind)
    ch = oracle.Chain.paper(shape, grid, kind=kind)
    n = p.buffer_numel(0, real=(kind == "r2c"))
    if kind == "c2c":
        u = inputs.uniform_complex(n, [seed], np.complex64)
    else:
        u = inputs.gaussian_real(n, [seed], np.float32)
    x = torch.from_numpy(u).to("cuda")
    y = p.forward(x)
    z = p.backward(y)
    yh = _host(y)
    zh = _host(z)
    # round trip and Parseval over the whole array
    u64 = u.astype(np.complex128 if kind == "c2c" else np.float64)
    assert np.linalg.norm(zh - u64) / np.linalg.norm(u64) <= 1e-5
    if kind == "c2c":
        total = float(np.prod(shape))
        lhs = float(np.sum(np.abs(u64) ** 2))
        rhs = total * float(np.sum(np.abs(yh.astype(np.complex128)) ** 2))
        assert abs(lhs - rhs) <= 1e-5 * lhs
    # sampled bins against direct sums of the definition
    G = oracle.gather_global(u64, ch.layout(0, spectral=(kind == "c2c")))
    rng = np.random.default_rng(seed + 100)
    spec = ch.spectral_shape()
    bins = [tuple(int(rng.integers(0, s)) for s in spec) for _ in range(6)]
    bins.append(tuple(0 for _ in spec))
    expect = oracle.dft_bins(G, bins, -1, 1.0 / float(np.prod(shape)))
    lay = ch.output_layout()
    got = np.array([yh[oracle.layout_offset(lay, b)] for b in bins])
    assert np.linalg.norm(got - expect) / np.linalg.norm(expect) <= 1e-5


def test_full_size_tile_order_and_placement_are_result_neutral():
    # at 1 GiB per buffer the forward axis-1 stage of the default placement
    # (stores straight into the next layout) hands each XCD a contiguous range
    # of tiles; the gather placement keeps the round-robin order: every line
    # sees the same arithmetic, so the outputs agree bit for bit
    shape, grid = (512, 512, 512), (8, 8)
    print("case", shape, grid, flush=True)
    a = Plan(shape, grid)
    b = Plan(shape, grid, placement=("gather", "gather"))
    x = inputs.uniform_complex_device(a.buffer_numel(0), 4, torch.complex64, torch.device("cuda"))
    ya = a.forward(x)
    yb = b.forward(x)
    assert torch.equal(ya, yb)
    del yb
    za = a.backward(ya)
    zb = b.backward(ya)
    assert torch.equal(za, zb)
