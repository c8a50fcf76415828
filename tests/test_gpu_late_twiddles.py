"""The twiddle staging order of the stage kernels: plans on buffers beyond the
last-level cache stage each workgroup's twiddle table while its first loads
are in flight (the kernels' SF_LATE_TWIDDLES path), smaller plans first.  With
PFFT_LATE_TWIDDLES=1 at plan creation every stage takes the late order, so
small plans of every kernel family that reads the flag (strided and
contiguous complex stages in both precisions, stages whose sides step
differently, resident grids, 64-bit offsets, real-to-complex and
complex-to-real stages, batches) must give bitwise the results of the default
order, and the oracle's within tolerance."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09536_amd import inputs
from paper_1804_09536_amd.plan import Batch, Plan

pytestmark = pytest.mark.gpu

CASES = [
    dict(shape=(64, 32, 128), grid=(4, 4)),
    dict(shape=(64, 32, 128), grid=(4, 4), precision="f64"),
    dict(shape=(96, 64, 128), grid=(2, 4), transposed_out=True),
    dict(shape=(48, 40, 96), grid=(2, 3), tuning=dict(resident_contig=1, resident_strided=1)),
    dict(shape=(64, 24, 48), grid=(2, 2), tuning=dict(wide_offsets=1)),
    dict(shape=(1024, 4, 32), grid=(2, 2)),
    dict(shape=(32, 16, 512), grid=(2, 4), kind="r2c"),
    dict(shape=(32, 16, 512), grid=(2, 4), kind="r2c", precision="f64"),
    dict(shape=(12, 10, 96), grid=(2, 3), kind="r2c", tuning=dict(tile_contig=2)),
]


def _plan(c):
    p = Plan(c["shape"], c["grid"], kind=c.get("kind", "c2c"), precision=c.get("precision", "f32"),
             transposed_out=c.get("transposed_out", False))
    if "tuning" in c:
        p.set_tuning(**c["tuning"])
    return p


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("c", CASES, ids=[str(i) for i in range(len(CASES))])
def test_late_twiddle_order_gives_identical_results(c, monkeypatch):
    print("case", c, flush=True)
    kind, prec = c.get("kind", "c2c"), c.get("precision", "f32")
    ref = _plan(c)
    monkeypatch.setenv("PFFT_LATE_TWIDDLES", "1")
    late = _plan(c)
    late.validate()
    monkeypatch.delenv("PFFT_LATE_TWIDDLES")
    n = ref.buffer_numel(0, real=(kind == "r2c"))
    if kind == "c2c":
        u = inputs.uniform_complex(n, [61], np.complex64 if prec == "f32" else np.complex128)
    else:
        u = inputs.gaussian_real(n, [61], np.float32 if prec == "f32" else np.float64)
    x = torch.from_numpy(u).cuda()
    y0, y1 = _host(ref.forward(x)), _host(late.forward(x))
    assert y1.tobytes() == y0.tobytes()
    yd = torch.from_numpy(y0).cuda()
    assert _host(late.backward(yd)).tobytes() == _host(ref.backward(yd)).tobytes()
    ch = oracle.Chain.paper(c["shape"], c["grid"], kind=kind, transposed_out=c.get("transposed_out", False))
    e = oracle.forward(ch, u.astype(np.float64 if kind == "r2c" else np.complex128))
    tol = 1e-5 if prec == "f32" else 1e-12
    assert np.linalg.norm(y1 - e) / np.linalg.norm(e) <= tol


def test_late_twiddle_order_in_batches(monkeypatch):
    members = [((32, 16, 64), (2, 4), "c2c"), ((16, 12, 64), (2, 2), "r2c"), ((24, 8, 64), (2, 2), "r2c")]

    def make():
        return Batch([Plan(s, g, kind=k) for s, g, k in members])

    ref = make()
    monkeypatch.setenv("PFFT_LATE_TWIDDLES", "1")
    late = make()
    monkeypatch.delenv("PFFT_LATE_TWIDDLES")
    for b in (ref, late):
        for m, (s, g, k) in enumerate(members):
            n = b.inputs[m].numel()
            u = (inputs.uniform_complex(n, [62, m], np.complex64) if k == "c2c"
                 else inputs.gaussian_real(n, [62, m], np.float32))
            b.inputs[m].copy_(torch.from_numpy(u))
        b.forward()
    torch.cuda.synchronize()
    for m in range(len(members)):
        print("member", m, members[m], flush=True)
        assert _host(late.outputs[m]).tobytes() == _host(ref.outputs[m]).tobytes()
    ref.backward()
    late.backward()
    torch.cuda.synchronize()
    for m in range(len(members)):
        assert _host(late.inputs[m]).tobytes() == _host(ref.inputs[m]).tobytes()
