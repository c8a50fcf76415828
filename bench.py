"""Benchmark of the distributed FFT hot path on one MI355X.

A step is one forward plus one backward transform (every partial transform
and every fused redistribution of both chains) of the workload's array, with
the input already resident in HBM.  Default workload: 512^3 complex64, pencil
decomposition on an 8x8 virtual-rank grid (two redistributions per direction,
each fused into the next partial transform's kernel).

Prints ONE JSON line.  `value` is milliseconds per forward+backward (lower is
better); `pct_hbm_peak` is the algorithmic traffic of a step (each partial
transform reads and writes the array once) over the step time, as a fraction
of the MI355X's 8 TB/s.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # bytes/s, MI355X published peak

WORKLOADS = {
    # name: (shape, grid, kind, precision, chain)
    "pencil512": ((512, 512, 512), (8, 8), "c2c", "f32", None),
    # the same array over other virtual grids: slab, coarser and finer pencils,
    # and the thin-slab limit (one plane per rank)
    "slab512": ((512, 512, 512), (8,), "c2c", "f32", None),
    "pencil512_4x4": ((512, 512, 512), (4, 4), "c2c", "f32", None),
    "pencil512_32x16": ((512, 512, 512), (32, 16), "c2c", "f32", None),
    "slab512_thin": ((512, 512, 512), (512,), "c2c", "f32", None),
    # long lines: 1024^3, and the largest buffers of 32-bit offsets (just
    # under 2^31 elements, 12 GiB each)
    "c2c1024": ((1024, 1024, 1024), (8, 8), "c2c", "f32", None),
    "max1536": ((1536, 1024, 1024), (8, 8), "c2c", "f32", None),
    # the paper's largest 3-D size: 2^33 elements, 64 GiB per buffer (64-bit offsets)
    "c2c2048": ((2048, 2048, 2048), (8, 8), "c2c", "f32", None),
    "pencil256": ((256, 256, 256), (4, 4), "c2c", "f32", None),
    "slab32_f64": ((32, 32, 32), (4,), "c2c", "f64", [(0, 2)]),
    "pencil512_f64": ((512, 512, 512), (8, 8), "c2c", "f64", None),
    "r2c512": ((512, 512, 512), (8, 8), "r2c", "f32", None),
    # real-to-real: type II cosine transform on every axis (type III back)
    "dct512": ((512, 512, 512), (8, 8), "r2r", "f32", None),
    "c2c4d64": ((64, 64, 64, 64), (2, 2, 4), "c2c", "f32", None),
    # the transposed-out alignment of the output (split axes stored first)
    "slab512_tr": ((512, 512, 512), (8,), "c2c", "f32", None, {"transposed_out": True}),
    "pencil512_tr": ((512, 512, 512), (8, 8), "c2c", "f32", None, {"transposed_out": True}),
}

KIND_NAMES = {"c2c": "c2c_stage", "copy": "redistribute_copy", "r2c": "r2c_stage", "c2r": "c2r_stage",
              "r2r": "r2r_stage"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="pencil512", choices=sorted(WORKLOADS) + ["batch168", "grad256"])
    ap.add_argument("--path", default="fused", choices=["fused", "unfused", "pack_realign"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip per-launch events in the timed region")
    ap.add_argument("--placement", default=None,
                    help="gather|scatter|direct|final, or FWD,BWD (default: the library's default pair)")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload only: skip the FP64, real-input, 4-D, batch and autograd sub-benches")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, copy one buffer of the workload's size with torch (a "
                         "known-size reference for hardware byte counters)")
    return ap.parse_args()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None if there is none or the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pencil512_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for src in rec.get("kernel_sources", []):
        with open(os.path.join(ROOT, "paper_1804_09536_amd", "csrc", src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec.get("kernel_sources_sha256"):
        return None
    return rec.get("traffic_bytes_per_launch", {}).get(kernel)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_name(rec):
    base = KIND_NAMES.get(rec["kind"], rec["kind"])
    mode = "contig" if rec["contig"] else "strided"
    return "%s_%s_n%d" % (base, mode, rec["length"])


def cpu_baseline(shape, grid, kind, chain, u_np):
    """The FP64 oracle on the host cores: one forward + backward of the same
    workload (the full array: ~10-40 s of CPU work)."""
    import numpy as np
    import oracle

    ch = oracle.Chain.paper(shape, grid, kind=kind, steps=chain)
    x = u_np.astype(np.complex128 if kind == "c2c" else np.float64)
    t0 = time.perf_counter()
    y = oracle.forward(ch, x)
    oracle.backward(ch, y)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": round(dt * 1e3, 1), "unit": "ms per forward+backward", "cores": cores, "kind": "oracle",
           "sample": "one full forward+backward of the same workload in FP64 (OpenMP over lines)",
           "cpu_model": cpu_model()}
    # the same oracle on one thread, on a bounded sample: the 256^3 pencil on
    # 4x4 ranks, in a child process so that its OpenMP runtime starts with one thread
    import subprocess
    code = ("import time, numpy as np, oracle\n"
            "ch = oracle.Chain.paper((256, 256, 256), (4, 4))\n"
            "x = np.random.default_rng(1).uniform(-1, 1, 2 * 256 ** 3).view(np.complex128)\n"
            "t = time.perf_counter(); oracle.backward(ch, oracle.forward(ch, x)); print(time.perf_counter() - t)\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT,
                           timeout=300)
        t1 = float(r.stdout.strip().splitlines()[-1])
        out["single_thread"] = {"value": round(t1 * 1e3, 1), "unit": "ms per forward+backward", "cores": 1,
                                "sample": "256x256x256 complex128 on a 4x4 virtual-rank grid, one thread"}
    except (subprocess.SubprocessError, ValueError, IndexError):
        out["single_thread"] = None
    return out


BATCH_SHAPES = [
    # (shape, grid): the mixed workload of many uneven transforms, 8 instances x 3 field components each
    ((64, 64, 64), (4,)),
    ((96, 96, 96), (8,)),
    ((128, 128, 128), (4, 4)),
    ((192, 192, 192), (4, 4)),
    ((256, 256, 256), (4, 4)),
    ((384, 384, 384), (8, 8)),
    ((128, 256, 512), (4, 8)),
]


def _timeit(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def bench_batch(steps, warmup):
    """168 complex64 transforms (7 shapes x 8 instances x 3 components): the
    batch (one launch per stage and kernel shape, captured in a HIP graph)
    against one call per transform, the latter both with the library
    defaults and with each shape's autotuned knobs (the user cache, else the
    shipped table for this device).  The batch keeps the defaults: members
    with their own tuned knobs split the grouped launches (measured slower).
    Returns a record."""
    import torch

    from paper_1804_09536_amd import inputs, tune
    from paper_1804_09536_amd.plan import Batch, Plan

    dev = torch.device("cuda:0")
    uniq = [Plan(s, g, device=dev).bind() for s, g in BATCH_SHAPES]
    tuned = [tune.tuned_plan(s, g, tune_missing=False, device=dev).bind() for s, g in BATCH_SHAPES]
    n_tuned = sum(1 for p in tuned if p.tuned)
    members = [p for p in uniq for _ in range(24)]
    tuned_members = [p for p in tuned for _ in range(24)]
    batch = Batch(members, device=dev)
    for m, x in enumerate(batch.inputs):
        x.copy_(inputs.uniform_complex_device(x.numel(), 1000 + m, torch.complex64, dev))
    total_bytes = 0.0
    for p in members:
        total_bytes += 2 * 3 * 2 * p.buffer_numel(0) * 8  # fwd+bwd, 3 stages, read+write
    work = {id(p): p.workspace() for p in uniq + tuned}

    def per_transform(plans):
        def step():
            for m, p in enumerate(plans):
                p.forward(batch.inputs[m], out=batch.outputs[m], work=work[id(p)])
            for m, p in enumerate(plans):
                p.backward(batch.outputs[m], out=batch.inputs[m], work=work[id(p)])
        return step

    def batched():
        batch.forward()
        batch.backward()

    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        batched()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(graph, stream=stream):
            batched()
    torch.cuda.synchronize()

    t_graph = _timeit(graph.replay, steps, warmup)
    t_batch = _timeit(batched, steps, warmup)
    t_plain = _timeit(per_transform(tuned_members), steps, warmup)
    t_plain_default = _timeit(per_transform(members), steps, warmup)
    # the same transforms one shape at a time (tuned knobs): 24 calls of each plan
    per_shape = {}
    for i, p in enumerate(tuned):
        idx = [m for m, q in enumerate(members) if q is uniq[i]]

        def shape_step(p=p, idx=idx):
            for m in idx:
                p.forward(batch.inputs[m], out=batch.outputs[m], work=work[id(p)])
            for m in idx:
                p.backward(batch.outputs[m], out=batch.inputs[m], work=work[id(p)])
        per_shape["x".join(map(str, p.shape))] = round(_timeit(shape_step, steps, warmup), 3)
    del graph, batch, work
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return {"workload": "7 shapes x 8 instances x 3 components c2c complex64, mixed slab/pencil grids",
            "shapes": [[list(s), list(g)] for s, g in BATCH_SHAPES],
            "batched_graph_ms": round(t_graph, 3), "batched_eager_ms": round(t_batch, 3),
            "per_transform_ms": round(t_plain, 3), "per_transform_tuned_shapes": n_tuned,
            "per_transform_default_knobs_ms": round(t_plain_default, 3), "per_shape_ms": per_shape,
            "algorithmic_bytes": total_bytes,
            "pct_hbm_peak": round(100.0 * total_bytes / (t_graph * 1e-3) / HBM_PEAK, 2),
            "per_transform_pct_hbm_peak": round(100.0 * total_bytes / (t_plain * 1e-3) / HBM_PEAK, 2)}


def bench_grad(steps, warmup):
    """The differentiation workload: loss = sum_k |k|^2 |FFT(u)(k)|^2 on a
    256^3 float32 field (r2c, 4x4 pencil); one autograd step (forward, loss,
    backward through the adjoint kernels) against one plain forward+backward
    of the same plan.  Returns a record."""
    import numpy as np
    import torch

    from paper_1804_09536_amd import autograd as pad
    from paper_1804_09536_amd import inputs
    from paper_1804_09536_amd.plan import Plan

    dev = torch.device("cuda:0")
    shape, grid = (256, 256, 256), (4, 4)
    from paper_1804_09536_amd import tune
    plan = tune.tuned_plan(shape, grid, kind="r2c", tune_missing=False, device=dev).bind()
    w = pad.wavenumber_weight(plan).to(torch.float32)
    u0 = torch.from_numpy(inputs.gaussian_real(plan.buffer_numel(0, real=True), [5], np.float32)).to(dev)
    u = u0.clone().requires_grad_()

    def grad_step():
        u.grad = None
        uh = pad.forward(u, plan)
        loss = pad.weighted_energy(uh, w)
        loss.backward()

    y = plan.empty(plan.num_layouts - 1)
    z = plan.empty(0, real=True)

    def plain_step():
        plan.forward(u0, out=y)
        plan.backward(y, out=z)

    t_grad = _timeit(grad_step, steps, warmup)
    t_plain = _timeit(plain_step, steps, warmup)
    spec = plan.buffer_numel(plan.num_layouts - 1) * 8
    real = plan.buffer_numel(0, real=True) * 4
    # r2c stage: real in + spectrum out; two complex stages: spectrum in + out; same for the adjoint
    step_bytes = 2 * ((real + spec) + 2 * (2 * spec))
    return {"workload": "256x256x256 r2c float32, 4x4 pencil, loss sum |k|^2 |u_hat|^2",
            "autograd_step_ms": round(t_grad, 4), "plain_fwd_bwd_ms": round(t_plain, 4),
            "transform_bytes_per_step": step_bytes,
            "plain_pct_hbm_peak": round(100.0 * step_bytes / (t_plain * 1e-3) / HBM_PEAK, 2)}


def measure_plain(name, steps, warmup, path="fused", placement=None, profile=True, traffic=False):
    """Forward+backward of one WORKLOADS entry: ms per step (mean over the
    timed steps), per-launch HIP-event averages per kernel, the dominant
    kernel's roofline record, and the round trip's relative error."""
    import numpy as np
    import torch

    from paper_1804_09536_amd import inputs
    from paper_1804_09536_amd.plan import Plan

    shape, grid, kind, prec, chain = WORKLOADS[name][:5]
    extra = WORKLOADS[name][5] if len(WORKLOADS[name]) > 5 else {}
    from paper_1804_09536_amd import tune

    dev = torch.device("cuda:0")
    if placement is None and not extra:
        # the autotuner's choice for this workload on this device where it
        # has one (the user cache, else the shipped table), else the defaults
        plan = tune.tuned_plan(shape, grid, kind=kind, precision=prec, chain=chain, path=path, tune_missing=False,
                               device=dev).bind()
    else:
        plan = Plan(shape, grid, precision=prec, kind=kind, chain=chain, path=path, device=dev,
                    placement=placement, **extra).bind()
    n_in = plan.buffer_numel(0, real=(kind == "r2c"))
    # arrays beyond 2^28 elements are drawn on the device (no host copy, no CPU baseline)
    big = n_in > (1 << 28)
    if big and kind == "c2c":
        u_np = None
        x = inputs.uniform_complex_device(n_in, 4, plan.spec_dtype, dev)
    else:
        if kind == "c2c":
            u_np = inputs.uniform_complex(n_in, [4], np.complex64 if prec == "f32" else np.complex128)
        else:
            u_np = inputs.gaussian_real(n_in, [2], np.float32 if prec == "f32" else np.float64)
        x = torch.from_numpy(u_np).to(dev)
    y = plan.empty(plan.num_layouts - 1)
    # buffers beyond 32 GiB (2048^3 complex64: 64 GiB each): the backward
    # writes into the input buffer, so three buffers fit one device
    huge = x.numel() * x.element_size() > (32 << 30)
    z = x if huge else plan.empty(0, real=(kind == "r2c"))
    work = plan.workspace()

    def step():
        plan.forward(x, out=y, work=work)
        plan.backward(y, out=z, work=work)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.profile_read()
    if profile:
        plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.set_profiling(False)
    recs = plan.profile_read() if profile else []
    ms_per_step = (t1 - t0) * 1e3 / steps

    # algorithmic bytes of one step: every launch of forward and backward
    step_bytes = 0.0
    per_kernel = {}
    for r in recs:
        k = kernel_name(r)
        d = per_kernel.setdefault(k, {"ms": 0.0, "n": 0, "bytes": 0.0})
        d["ms"] += r["ms"]
        d["n"] += 1
        d["bytes"] += r["bytes"]
        step_bytes += r["bytes"]
    step_bytes /= max(1, steps)
    roofline = None
    if per_kernel:
        dom = max(per_kernel, key=lambda k: per_kernel[k]["ms"])
        d = per_kernel[dom]
        avg_ms = d["ms"] / d["n"]
        per_launch = d["bytes"] / d["n"]
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": 8000.0,
                    "unit": "GB/s", "frac": round(achieved / 8000.0, 4),
                    "traffic": measured_traffic(dom) if traffic else None,
                    "avg_launch_ms": round(avg_ms, 4), "bytes_per_launch": per_launch}
    # round-trip sanity on the last step (not for the huge buffers, whose
    # input is overwritten; the tests check those against closed forms)
    rt = None if huge else float(torch.linalg.vector_norm((z - x).flatten()) / torch.linalg.vector_norm(x.flatten()))
    return {"plan": plan, "step": step, "x": x, "y": y, "u_np": u_np, "shape": shape, "grid": grid, "kind": kind,
            "prec": prec, "chain": chain, "ms": ms_per_step, "step_bytes": step_bytes, "per_kernel": per_kernel,
            "roofline": roofline, "roundtrip": rt, "huge": huge}


def plain_record(name, steps, warmup):
    """A compact record of a WORKLOADS entry for the sub-benches of the default run."""
    import torch
    r = measure_plain(name, steps, warmup)
    shape, grid, kind, prec = r["shape"], r["grid"], r["kind"], r["prec"]
    out = {"workload": "%s %s %s on a %s virtual-rank grid" % ("x".join(map(str, shape)), kind,
                                                              ("complex64" if prec == "f32" else "complex128")
                                                              if kind != "r2c" else
                                                              ("float32" if prec == "f32" else "float64"),
                                                              "x".join(map(str, grid))),
           "ms_per_step": round(r["ms"], 4), "step_bytes": r["step_bytes"],
           "pct_hbm_peak": round(100.0 * r["step_bytes"] / (r["ms"] * 1e-3) / HBM_PEAK, 2),
           "per_kernel_avg_ms": {k: round(v["ms"] / v["n"], 4) for k, v in r["per_kernel"].items()},
           "roofline": r["roofline"], "roundtrip_rel_l2": r["roundtrip"],
           "placement": list(r["plan"].placement), "autotuned": r["plan"].tuned}
    del r
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the virtual ranks of the decomposition share one device; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.workload in ("batch168", "grad256"):
        rec = bench_batch(args.steps, args.warmup) if args.workload == "batch168" else bench_grad(args.steps,
                                                                                                     args.warmup)
        ms = rec["batched_graph_ms"] if args.workload == "batch168" else rec["autograd_step_ms"]
        metric = ("fwd+bwd ms, 168 mixed complex64 transforms; batched vs per-transform" if args.workload == "batch168"
                  else "autograd step (forward + loss + adjoint) vs plain fwd+bwd, 256^3 r2c float32")
        out = {"metric": metric, "value": ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": ms, "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
               "data": "synthetic", "config": {"workload": rec["workload"]}}
        out.update(rec)
        print(json.dumps(out), flush=True)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    placement = tuple(args.placement.split(",")) if args.placement else None
    if placement is not None and len(placement) == 1:
        placement = placement * 2
    r = measure_plain(args.workload, args.steps, args.warmup, path=args.path, placement=placement,
                      profile=not args.no_profile,
                      traffic=(args.workload == "pencil512" and args.placement is None and args.path == "fused"))
    plan, step, x, y = r["plan"], r["step"], r["x"], r["y"]
    shape, grid, kind, prec, chain, u_np = r["shape"], r["grid"], r["kind"], r["prec"], r["chain"], r["u_np"]
    ms_per_step, step_bytes, per_kernel, roofline = r["ms"], r["step_bytes"], r["per_kernel"], r["roofline"]

    # The paper's statistic (outside the timed region, Sec. 4): 50 blocks of 3
    # uninterrupted forward+backward pairs, each block bracketed by events on
    # the stream; the fastest block (and the median) divided by 3.
    outer, inner = (10 if r["huge"] else 50), 3
    blocks = []
    for _ in range(outer):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(inner):
            step()
        e1.record()
        blocks.append((e0, e1))
    torch.cuda.synchronize()
    per_pair = sorted(a.elapsed_time(b) / inner for a, b in blocks)
    paper_stat = {"outer": outer, "inner": inner, "min_ms": round(per_pair[0], 4),
                  "median_ms": round(per_pair[len(per_pair) // 2], 4)}

    # Copy ceiling: a device-to-device copy of one buffer of the workload's
    # size (read + write), the practical bound of any pass over the array.
    src_c = y[: 1 << 27] if r["huge"] else y  # (a 1 GiB piece of the huge buffers)
    dst_c = torch.empty_like(src_c)
    for _ in range(2):
        dst_c.copy_(src_c)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(10):
        dst_c.copy_(src_c)
    c1.record()
    c1.synchronize()
    copy_ms = c0.elapsed_time(c1) / 10
    copy_gbps = 2 * src_c.numel() * src_c.element_size() / (copy_ms * 1e-3) / 1e9
    del dst_c
    copy_probe = {"bytes": 2 * src_c.numel() * src_c.element_size(), "ms": round(copy_ms, 4), "gbps": round(copy_gbps, 1),
                  "dominant_kernel_frac_of_copy": round(roofline["achieved"] / copy_gbps, 4) if roofline else None}

    if args.copy_calibration:
        ref = torch.empty_like(y)
        for _ in range(3):
            ref.copy_(y)
        torch.cuda.synchronize()
        del ref

    out = {
        "metric": "fwd+bwd 3D FFT ms & %HBM peak, 512^3 c2c FP32; batched/adjoint vs plain path",
        "value": round(ms_per_step, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": "%s %s %s on a %s virtual-rank grid, forward+backward, %s path"
                               % ("x".join(map(str, shape)), kind,
                                  ("float32" if prec == "f32" else "float64") if kind == "r2r"
                                  else ("complex64" if prec == "f32" else "complex128"),
                                  "x".join(map(str, grid)), args.path),
                   "shape": list(shape), "grid": list(grid), "kind": kind, "path": args.path,
                   "placement": list(plan.placement), "tuning": plan.tuning(),
                   "autotuned": plan.tuned},
        "step_bytes": step_bytes,
        "pct_hbm_peak": round(100.0 * step_bytes / (ms_per_step * 1e-3) / HBM_PEAK, 2) if step_bytes else None,
        "roundtrip_rel_l2": r["roundtrip"],
        "per_kernel_avg_ms": {k: round(v["ms"] / v["n"], 4) for k, v in per_kernel.items()},
        "roofline": roofline,
        "paper_statistic": paper_stat,
        "copy_probe": copy_probe,
    }
    del r, plan, step, x, y, src_c
    torch.cuda.synchronize()
    torch.cuda.empty_cache()

    # The metric's other half, measured in the same run on the same GPU: the
    # paper's precision (FP64), the real-input and 4-D configurations, the
    # batched form against per-transform calls and the autograd step against
    # plain forward+backward.
    if not args.no_extras and args.workload == "pencil512" and args.path == "fused" and args.placement is None:
        xs, xw = max(5, args.steps), max(2, args.warmup)
        print("extras: fp64", file=sys.stderr, flush=True)
        out["fp64"] = plain_record("pencil512_f64", xs, xw)
        print("extras: r2c", file=sys.stderr, flush=True)
        out["r2c"] = plain_record("r2c512", xs, xw)
        print("extras: c2c4d", file=sys.stderr, flush=True)
        out["c2c4d"] = plain_record("c2c4d64", xs, xw)
        print("extras: batched", file=sys.stderr, flush=True)
        out["batched"] = bench_batch(xs, xw)
        print("extras: autograd", file=sys.stderr, flush=True)
        out["autograd"] = bench_grad(xs, xw)

    cpu = None
    if not args.no_cpu_baseline and u_np is not None:
        print("cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(shape, grid, kind, chain, u_np)
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
