"""Autotuner: picks, per workload, the kernel tile shapes, grid policy and the
placement of intermediates (all result-neutral knobs of a plan) by timing
forward+backward on the device with HIP events, and caches the choice in a
JSON file (``$PFFT_TUNE_CACHE``, default ``~/.cache/paper_1804_09536_amd/tune.json``).

The search is coordinate-wise: strided-stage knobs first (with the library
defaults for the contiguous stages), then contiguous-stage knobs, then the
XCD tile order, streaming loads/stores and the radix plan of the complex
stages, then the forward and the backward placement; about 40 timed
configurations per workload.
"""
from __future__ import annotations

import json
import os
from typing import Optional

import numpy as np
import torch

from . import inputs
from .plan import Plan

TILES = {"tile_strided": (0, 1, 2, 3, 4, 5, 6, 7), "tile_contig": (0, 1, 2, 3, 4, 5)}
RESIDENT = (0, 1)
PLACEMENTS = ("gather", "scatter", "direct", "final")
# single knobs searched one at a time after the tile shapes
KNOBS = (("xcd_order", (0, 1, 2)), ("stream_strided", (0, 1, 2, 3, 4)), ("stream_contig", (0, 1, 2, 3, 4)),
         ("radix_alt", (0, 1, 2, 3)))


# Choices measured on MI355X for the workloads of the bench (written by
# `python -m paper_1804_09536_amd.tune --out <this file> --case ...`, each
# kept where the bench measured it faster than the library defaults), used
# where the user cache has no entry.
SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def cache_path() -> str:
    return os.environ.get("PFFT_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1804_09536_amd", "tune.json"))


def device_id(dev: int = 0) -> str:
    """The device's instruction set and compute-unit count, e.g.
    "gfx950/256cu" (the marketing name comes from name tables that are not
    found in every process, e.g. under a profiler)."""
    p = torch.cuda.get_device_properties(dev)
    arch = (getattr(p, "gcnArchName", "") or p.name).split(":")[0]
    return "%s/%dcu" % (arch, p.multi_processor_count)


def _key(shape, grid, kind, precision, chain, path) -> str:
    return json.dumps({"shape": list(shape), "grid": list(grid), "kind": kind, "precision": precision,
                       "chain": chain, "path": path, "device": device_id(0)}, sort_keys=True)


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _time(fn, steps: int) -> float:
    for _ in range(2):
        fn()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / steps


class _Case:
    """A plan of the workload with its buffers, for timing."""

    def __init__(self, shape, grid, kind, precision, chain, path, placement):
        self.plan = Plan(shape, grid, precision=precision, kind=kind, chain=chain, path=path, placement=placement)
        real = kind == "r2c"
        n = self.plan.buffer_numel(0, real=real)
        if real:
            rdt = np.float32 if self.plan.in_dtype == torch.float32 else np.float64
            self.x = torch.from_numpy(inputs.gaussian_real(n, [0], rdt)).to(self.plan.device)
        else:
            self.x = inputs.uniform_complex_device(n, 0, self.plan.spec_dtype, self.plan.device)
        self.y = self.plan.empty(self.plan.num_layouts - 1)
        self.z = self.plan.empty(0, real=real)
        self.work = self.plan.workspace()

    def fwd(self):
        self.plan.forward(self.x, out=self.y, work=self.work)

    def bwd(self):
        self.plan.backward(self.y, out=self.z, work=self.work)

    def both(self):
        self.fwd()
        self.bwd()


def lookup(shape, grid, kind: str = "c2c", precision: str = "f32", chain=None, path: str = "fused",
           cache: Optional[str] = None) -> Optional[dict]:
    """The cached choice for the workload on this device (the user cache
    first, then the shipped table), or None."""
    key = _key(shape, grid, kind, precision, chain, path)
    for path_ in (cache or cache_path(), SHIPPED):
        table = _load_cache(path_)
        if key in table:
            return table[key]
    return None


def autotune(shape, grid, kind: str = "c2c", precision: str = "f32", chain=None, path: str = "fused",
             steps: int = 5, cache: Optional[str] = None, force: bool = False, verbose: bool = False) -> dict:
    """Best {"placement": [forward, backward], "tuning", "ms"} for the
    workload (cached).  Tile knobs are searched with the default placement
    pair; then each chain's placement is chosen by timing that chain alone
    (the forward placement changes only forward launches, and likewise)."""
    cache = cache or cache_path()
    key = _key(shape, grid, kind, precision, chain, path)
    if not force:
        hit = lookup(shape, grid, kind, precision, chain, path, cache)
        if hit is not None:
            return hit
    case = _Case(shape, grid, kind, precision, chain, path, None)
    plan = case.plan
    cur = plan.tuning()

    def run(t):
        plan.set_tuning(**t)
        plan.bind()
        ms = _time(case.both, steps)
        if verbose:
            print("  tiles %s %.4f ms" % (t, ms), flush=True)
        return ms

    ms_cur = run(cur)
    for fields in (("tile_strided", "resident_strided"), ("tile_contig", "resident_contig")):
        for tile in TILES[fields[0]]:
            for res in RESIDENT:
                t = dict(cur, **{fields[0]: tile, fields[1]: res})
                if t == cur:
                    continue
                ms = run(t)
                if ms < ms_cur:
                    cur, ms_cur = t, ms
    for name, values in KNOBS:
        for v in values:
            t = dict(cur, **{name: v})
            if t == cur:
                continue
            ms = run(t)
            if ms < ms_cur:
                cur, ms_cur = t, ms
    del case, plan
    chosen = []
    for side in (0, 1):
        best_p, best_ms = None, None
        for p in PLACEMENTS:
            c = _Case(shape, grid, kind, precision, chain, path, (p, p))
            c.plan.set_tuning(**cur)
            c.plan.bind()
            if side == 1:
                c.fwd()
            ms = _time(c.fwd if side == 0 else c.bwd, steps)
            if verbose:
                print("  %s placement %s %.4f ms" % ("forward" if side == 0 else "backward", p, ms), flush=True)
            if best_ms is None or ms < best_ms:
                best_p, best_ms = p, ms
            del c
            torch.cuda.empty_cache()
        chosen.append(best_p)
    final = _Case(shape, grid, kind, precision, chain, path, tuple(chosen))
    final.plan.set_tuning(**cur)
    final.plan.bind()
    best = {"placement": chosen, "tuning": cur, "ms": _time(final.both, steps)}
    del final
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
               tune_missing: bool = True, device=None, **kw) -> Plan:
    """A plan with the cached (or, with tune_missing, freshly tuned) best
    knobs; the library defaults where there is none."""
    best = (autotune(shape, grid, kind=kind, precision=precision, chain=chain, path=path, **kw) if tune_missing
            else lookup(shape, grid, kind, precision, chain, path, kw.get("cache")))
    if best is None:
        return Plan(shape, grid, precision=precision, kind=kind, chain=chain, path=path, device=device)
    plan = Plan(shape, grid, precision=precision, kind=kind, chain=chain, path=path,
                placement=tuple(best["placement"]), device=device)
    plan.set_tuning(**best["tuning"])
    plan.tuned = True
    return plan


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="tune workloads on this device and write the choices to a table")
    ap.add_argument("--out", required=True, help="JSON table to write (entries are added or replaced)")
    ap.add_argument("--case", action="append", required=True,
                    help='JSON [shape, grid] or [shape, grid, kind, precision], e.g. "[[384,384,384],[8,8]]"')
    ap.add_argument("--steps", type=int, default=5)
    args = ap.parse_args(argv)
    for c in args.case:
        spec = json.loads(c)
        shape, grid = tuple(spec[0]), tuple(spec[1])
        kind = spec[2] if len(spec) > 2 else "c2c"
        prec = spec[3] if len(spec) > 3 else "f32"
        best = autotune(shape, grid, kind=kind, precision=prec, steps=args.steps, cache=args.out, force=True)
        print(json.dumps({"shape": shape, "grid": grid, "kind": kind, "precision": prec, **best}), flush=True)


if __name__ == "__main__":
    main()
