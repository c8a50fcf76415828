"""64-bit element offsets: the kernels' wide variants forced onto small plans
against the oracle (results must not depend on the offset width), and the
paper's largest 3-D size, 2048^3 complex64 (2^33 elements, 64 GiB per buffer)
on the 8x8 grid, checked against closed forms over every output element: a
separable plane wave e^{2 pi i m.j / N} transforms to a unit delta at k = m
(Eq. multifft with the paper's 1/N_m factors), and the backward returns the
wave."""
import math

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


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


SMALL = [((16, 24, 32), (2, 3), "c2c", "f32", False), ((32, 16, 64), (4, 2), "c2c", "f64", False),
         ((8, 12, 6, 10), (2, 2, 3), "c2c", "f32", False), ((12, 16, 20), (4,), "r2c", "f32", False),
         ((16, 24, 32), (2, 3), "c2c", "f32", True), ((20, 14, 10), (2, 2), "c2c", "f64", False)]


@pytest.mark.parametrize("shape,grid,kind,prec,tr", SMALL)
def test_forced_wide_offsets_match_oracle(shape, grid, kind, prec, tr):
    print("case", shape, grid, kind, prec, tr, flush=True)
    tol = 1e-12 if prec == "f64" else 1e-5
    p = Plan(shape, grid, kind=kind, precision=prec, transposed_out=tr)
    p.set_tuning(wide_offsets=1)
    p.validate()
    ch = oracle.Chain.paper(shape, grid, kind=kind, transposed_out=tr)
    n = p.buffer_numel(0, real=(kind == "r2c"))
    if kind == "c2c":
        u = inputs.uniform_complex(n, [60, n], np.complex64 if prec == "f32" else np.complex128)
        u64 = u.astype(np.complex128)
    else:
        u = inputs.gaussian_real(n, [60, n], np.float32 if prec == "f32" else np.float64)
        u64 = u.astype(np.float64)
    y = p.forward(torch.from_numpy(u).cuda())
    got = _host(y)
    assert relerr(got, oracle.forward(ch, u64)) <= tol
    assert relerr(_host(p.backward(y)), oracle.backward(ch, got.astype(np.complex128))) <= tol
    # the standalone redistribution with the wide copy kernel, bit for bit
    payload = inputs.index_payload(p.buffer_numel(0), p.spec_dtype == torch.complex64 and np.complex64
                                   or np.complex128)
    r = _host(p.redistribute(torch.from_numpy(payload).cuda(), 0, 1))
    assert r.tobytes() == oracle.redistribute(payload, ch.layout(0), ch.layout(1)).tobytes()


SHAPE, GRID, MODE = (2048, 2048, 2048), (8, 8), (37, 1000, 2045)


def _wave_block(p, layout, r):
    """The plane wave on rank r's block of `layout` (complex64, C order of
    the block's axes), or None for an empty block."""
    shp, st, off = p.local_block(layout, r)
    if shp[0] * shp[1] * shp[2] == 0:
        return None, off
    ph = []
    for a in range(3):
        j = torch.arange(st[a], st[a] + shp[a], device="cuda", dtype=torch.float64)
        ang = 2.0 * math.pi * ((MODE[a] * j) % SHAPE[a]) / SHAPE[a]
        ph.append(torch.polar(torch.ones_like(ang), ang))
    blk = (ph[0][:, None, None] * ph[1][None, :, None] * ph[2][None, None, :]).to(torch.complex64)
    return blk.reshape(-1), off


def test_2048_cubed_plane_wave_closed_form():
    print("case", SHAPE, GRID, MODE, flush=True)
    p = Plan(SHAPE, GRID)
    assert p.buffer_numel(0) == 2 ** 33
    P = GRID[0] * GRID[1]
    x = p.empty(0)
    for r in range(P):
        blk, off = _wave_block(p, 0, r)
        if blk is not None:
            x[off:off + blk.numel()] = blk
            del blk
    y = p.forward(x)
    del x
    torch.cuda.synchronize()
    print("  forward done", flush=True)
    # the delta's position in the output layout, and the largest other magnitude
    last = p.num_layouts - 1
    pos = None
    for r in range(P):
        shp, st, off = p.local_block(last, r)
        if all(st[a] <= MODE[a] < st[a] + shp[a] for a in range(3)):
            loc = [MODE[a] - st[a] for a in range(3)]
            pos = off + (loc[0] * shp[1] + loc[1]) * shp[2] + loc[2]
    assert pos is not None
    peak = y[pos].item()
    assert abs(peak - 1.0) <= 1e-5
    y[pos] = 0
    chunk = 1 << 28
    worst = max(torch.max(torch.abs(y[i:i + chunk])).item() for i in range(0, y.numel(), chunk))
    assert worst <= 1e-5
    y[pos] = 1.0
    z = p.backward(y)
    del y
    torch.cuda.synchronize()
    print("  backward done", flush=True)
    err = 0.0
    for r in range(P):
        blk, off = _wave_block(p, 0, r)
        if blk is not None:
            err = max(err, torch.max(torch.abs(z[off:off + blk.numel()] - blk)).item())
            del blk
    assert err <= 1e-5
