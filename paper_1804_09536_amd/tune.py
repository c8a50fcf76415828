"""Autotuner: picks, per workload, the kernel tile shapes, grid policy and the
placement of intermediates (all result-neutral knobs of a plan) by timing
forward+backward on the device with HIP events, and caches the choice in a
JSON file (``$PFFT_TUNE_CACHE``, default ``~/.cache/paper_1804_09536_amd/tune.json``).

The search is coordinate-wise: strided-stage knobs first (with the library
defaults for the contiguous stages), then contiguous-stage knobs, for each
placement; about 30 timed configurations per workload.
"""
from __future__ import annotations

import json
import os
from typing import Optional

import numpy as np
import torch

from . import inputs
from .plan import Plan

TILES = (0, 1, 2, 3)
RESIDENT = (0, 1)


def cache_path() -> str:
    return os.environ.get("PFFT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1804_09536_amd", "tune.json"))


def _key(shape, grid, kind, precision, chain, path) -> str:
    return json.dumps({"shape": list(shape), "grid": list(grid), "kind": kind, "precision": precision,
                       "chain": chain, "path": path, "device": torch.cuda.get_device_name(0)}, sort_keys=True)


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time(plan: Plan, x, y, z, work, steps: int) -> float:
    for _ in range(2):
        plan.forward(x, out=y, work=work)
        plan.backward(y, out=z, work=work)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        plan.forward(x, out=y, work=work)
        plan.backward(y, out=z, work=work)
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / steps


def autotune(shape, grid, kind: str = "c2c", precision: str = "f32", chain=None, path: str = "fused",
             steps: int = 5, cache: Optional[str] = None, force: bool = False, verbose: bool = False) -> dict:
    """Best {"placement", "tuning", "ms"} for the workload (cached)."""
    cache = cache or cache_path()
    key = _key(shape, grid, kind, precision, chain, path)
    table = _load_cache(cache)
    if key in table and not force:
        return table[key]
    best = None
    for placement in ("gather", "scatter", "direct", "final"):
        plan = Plan(shape, grid, precision=precision, kind=kind, chain=chain, path=path, placement=placement)
        real = kind == "r2c"
        n = plan.buffer_numel(0, real=real)
        if real:
            rdt = np.float32 if plan.in_dtype == torch.float32 else np.float64
            x = torch.from_numpy(inputs.gaussian_real(n, [0], rdt)).to(plan.device)
        else:
            x = inputs.uniform_complex_device(n, 0, plan.spec_dtype, plan.device)
        y = plan.empty(plan.num_layouts - 1)
        z = plan.empty(0, real=real)
        work = plan.workspace()
        cur = plan.tuning()

        def run(t):
            plan.set_tuning(**t)
            plan.bind()
            ms = _time(plan, x, y, z, work, steps)
            if verbose:
                print("  %s %s %.4f ms" % (placement, t, ms), flush=True)
            return ms

        ms_cur = run(cur)
        for fields in (("tile_strided", "resident_strided"), ("tile_contig", "resident_contig")):
            for tile in TILES:
                for res in RESIDENT:
                    t = dict(cur, **{fields[0]: tile, fields[1]: res})
                    if t == cur:
                        continue
                    ms = run(t)
                    if ms < ms_cur:
                        cur, ms_cur = t, ms
        if best is None or ms_cur < best["ms"]:
            best = {"placement": placement, "tuning": cur, "ms": ms_cur}
        del plan, x, y, z, work
        torch.cuda.empty_cache()
    table = _load_cache(cache)
    table[key] = best
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    tmp = cache + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, cache)
    return best


def tuned_plan(shape, grid, kind: str = "c2c", precision: str = "f32", chain=None, path: str = "fused",
               **kw) -> Plan:
    """A plan with the cached (or freshly tuned) best knobs."""
    best = autotune(shape, grid, kind=kind, precision=precision, chain=chain, path=path, **kw)
    plan = Plan(shape, grid, precision=precision, kind=kind, chain=chain, path=path, placement=best["placement"])
    plan.set_tuning(**best["tuning"])
    return plan
