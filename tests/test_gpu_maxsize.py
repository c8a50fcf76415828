"""The largest buffers of the 32-bit-offset kernels (just under 2^31 elements:
1536x1024x1024 complex64, 12 GiB per buffer) on the metric's 8x8 grid, checked
against closed forms over every output element: a separable plane wave
e^{2 pi i m.j / N} transforms to a unit delta at k = m (Eq. multifft with the
paper's 1/N_m factors), and the backward returns the wave."""
import math

import pytest
import torch

from paper_1804_09536_amd.plan import Plan

pytestmark = pytest.mark.gpu

SHAPE, GRID, MODE = (1536, 1024, 1024), (8, 8), (37, 1000, 5)


def _plane_wave(p, layout):
    """The wave in `layout`, rank block by rank block (outer products of
    per-axis phases over each block's global index range)."""
    buf = p.empty(layout)
    P = GRID[0] * GRID[1]
    for r in range(P):
        shp, st, off = p.local_block(layout, r)
        cnt = shp[0] * shp[1] * shp[2]
        if cnt == 0:
            continue
        ph = []
        for a in range(3):
            j = torch.arange(st[a], st[a] + shp[a], device="cuda", dtype=torch.float64)
            ang = 2.0 * math.pi * ((MODE[a] * j) % SHAPE[a]) / SHAPE[a]
            ph.append(torch.polar(torch.ones_like(ang), ang))
        blk = ph[0][:, None, None] * ph[1][None, :, None] * ph[2][None, None, :]
        buf[off:off + cnt] = blk.reshape(-1).to(torch.complex64)
        del blk
    return buf


def test_largest_buffers_plane_wave_closed_form():
    print("case", SHAPE, GRID, MODE, flush=True)
    p = Plan(SHAPE, GRID)
    assert p.buffer_numel(0) < 2 ** 31
    x = _plane_wave(p, 0)
    y = p.forward(x)
    # the delta's position in the output layout
    last = p.num_layouts - 1
    P = GRID[0] * GRID[1]
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
    assert torch.max(torch.abs(y)).item() <= 1e-5
    y[pos] = 1.0
    z = p.backward(y)
    err = torch.max(torch.abs(z - x)).item()
    assert err <= 1e-5
    torch.cuda.synchronize()
