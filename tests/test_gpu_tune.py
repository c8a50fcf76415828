"""The autotuner: it times the result-neutral knobs of a small workload,
caches its choice, and the tuned plan computes exactly what the default
plan computes."""
import json

import numpy as np
import pytest
import torch

from paper_1804_09536_amd import inputs, tune
from paper_1804_09536_amd.plan import Plan

pytestmark = pytest.mark.gpu


def test_autotune_choice_is_cached_and_result_neutral(tmp_path):
    cache = str(tmp_path / "tune.json")
    shape, grid = (32, 16, 64), (2, 4)
    best = tune.autotune(shape, grid, steps=2, cache=cache)
    assert set(best) == {"placement", "tuning", "ms"}
    assert all(p in tune.PLACEMENTS for p in best["placement"])
    with open(cache) as f:
        assert len(json.load(f)) == 1
    assert tune.autotune(shape, grid, steps=2, cache=cache) == best   # served from the cache
    tuned = tune.tuned_plan(shape, grid, cache=cache)
    plain = Plan(shape, grid)
    u = torch.from_numpy(inputs.uniform_complex(plain.buffer_numel(0), [31], np.complex64)).cuda()
    a = plain.forward(u)
    b = tuned.forward(u)
    torch.cuda.synchronize()
    assert a.cpu().numpy().tobytes() == b.cpu().numpy().tobytes()
