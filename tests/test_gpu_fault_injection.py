"""The launch error path, forced from the host: with PFFT_FAULT_INJECT=launch
every stage launch reports a failure without launching anything, so the
chains, redistributions and batches must return PFFT_EHIP with a message
(PfftError in Python) and leave the plan usable; without it the same calls
give correct results again."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09536_amd import _lib, inputs
from paper_1804_09536_amd.plan import Batch, Plan

pytestmark = pytest.mark.gpu

PFFT_EHIP = -7


def test_injected_launch_failures_are_reported_and_recoverable(monkeypatch):
    shape, grid = (32, 16, 64), (2, 4)
    p = Plan(shape, grid)
    n = p.buffer_numel(0)
    u = inputs.uniform_complex(n, [50], np.complex64)
    x = torch.from_numpy(u).cuda()
    b = Batch([p, Plan((16, 32, 8), (3, 5))])
    monkeypatch.setenv("PFFT_FAULT_INJECT", "launch")
    for call in (lambda: p.forward(x), lambda: p.backward(x[:p.buffer_numel(p.num_layouts - 1)]),
                 lambda: p.redistribute(x, 0, 1), b.forward, b.backward):
        with pytest.raises(_lib.PfftError) as e:
            call()
        assert e.value.status == PFFT_EHIP
        assert "launch" in str(e.value)
    monkeypatch.delenv("PFFT_FAULT_INJECT")
    y = p.forward(x)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    ch = oracle.Chain.paper(shape, grid)
    expect = oracle.forward(ch, u.astype(np.complex128))
    assert np.linalg.norm(got - expect) / np.linalg.norm(expect) <= 1e-5
    b.forward()
    torch.cuda.synchronize()
