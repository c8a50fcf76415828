"""Batched execution: several plans of different shapes and grids in one
batch give the same results as their own per-transform launches (the same
kernels, bit for bit) and as the oracle; a captured graph replays them."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09536_amd import inputs
from paper_1804_09536_amd.plan import Batch, Plan

pytestmark = pytest.mark.gpu

MEMBERS = [
    ((16, 32, 8), (3, 5), "c2c"),
    ((32, 16, 64), (2, 4), "c2c"),
    ((24, 12, 48), (2, 2), "c2c"),       # radix-3 lengths
    ((32, 32, 32), (4,), "c2c"),         # slab
    ((8, 16, 4, 32), (3, 1, 5), "c2c"),  # 4-D
    ((16, 16, 32), (4, 2), "r2c"),       # real input (its r2c/c2r stages run the multi-transform kernel)
    ((12, 16, 24), (2, 3), "r2r"),       # cosine/sine transforms (per-member launches)
]
R2R = ("dst2", "dct2", "dst2")


def _plan(s, g, k, **kw):
    return Plan(s, g, kind=k, r2r=R2R if k == "r2r" else None, **kw)


def _fill(batch):
    data = []
    for m, p in enumerate(batch.plans):
        n = batch.inputs[m].numel()
        if p.kind == "c2c":
            u = inputs.uniform_complex(n, [30, m], np.complex64)
        else:
            u = inputs.gaussian_real(n, [30, m], np.float32)
        batch.inputs[m].copy_(torch.from_numpy(u))
        data.append(u)
    return data


def test_batch_equals_per_transform_and_oracle():
    plans = [_plan(s, g, k) for s, g, k in MEMBERS]
    plans.append(plans[1])  # the same plan twice shares its tables
    plans.append(_plan((32, 16, 64), (2, 4), "c2c", destroy_input=True))  # no workspace
    b = Batch(plans)
    data = _fill(b)
    b.forward()
    torch.cuda.synchronize()
    for m, p in enumerate(b.plans):
        print("member", m, p.shape, p.grid, p.kind, flush=True)
        ref = p.forward(torch.from_numpy(data[m]).cuda())
        torch.cuda.synchronize()
        assert b.outputs[m].cpu().numpy().tobytes() == ref.cpu().numpy().tobytes()
        ch = oracle.Chain.paper(p.shape, p.grid, kind=p.kind, r2r=p.r2r)
        expect = oracle.forward(ch, data[m].astype(np.complex128 if p.kind == "c2c" else np.float64))
        got = b.outputs[m].cpu().numpy()
        assert np.linalg.norm(got - expect) / np.linalg.norm(expect) <= 1e-5
    b.backward()
    torch.cuda.synchronize()
    for m in range(len(b.plans)):
        back = b.inputs[m].cpu().numpy()
        assert np.linalg.norm(back - data[m]) / np.linalg.norm(data[m]) <= 1e-5


def test_batch_graph_replay():
    plans = [_plan(s, g, k) for s, g, k in MEMBERS[:3]]
    b = Batch(plans)
    data = _fill(b)
    b.forward()
    torch.cuda.synchronize()
    eager = [o.clone() for o in b.outputs]
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            b.forward()
    torch.cuda.current_stream().wait_stream(stream)
    for rep in range(3):
        for o in b.outputs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for m in range(len(plans)):
            assert torch.equal(b.outputs[m], eager[m]), (rep, m)
        # eager work between replays
        for m in range(len(plans)):
            b.inputs[m].copy_(torch.from_numpy(data[m]))
        torch.cuda.synchronize()


# The mixed batch of the batching workload: one instance of each shape, three
# field components each (seeds [6, shape, instance, component]), on the grids
# the bench uses; 384^3 and 128x256x512 run the radix-3 and the 512-point
# strided kernels inside the multi-transform launches.
CONFIG5 = [((64, 64, 64), (4,)), ((96, 96, 96), (8,)), ((128, 128, 128), (4, 4)), ((192, 192, 192), (4, 4)),
           ((256, 256, 256), (4, 4)), ((384, 384, 384), (8, 8)), ((128, 256, 512), (4, 8))]


@pytest.fixture(scope="module")
def config5_batch():
    plans = [Plan(s, g) for s, g in CONFIG5]
    members = [p for p in plans for _ in range(3)]
    print("config5 batch of", len(members), "members", flush=True)
    b = Batch(members)
    data = []
    for m, x in enumerate(b.inputs):
        u = inputs.uniform_complex(x.numel(), [6, m // 3, 0, m % 3], np.complex64)
        x.copy_(torch.from_numpy(u))
        data.append(u)
    b.forward()
    torch.cuda.synchronize()
    eager = [o.clone() for o in b.outputs]
    outs = [o.cpu().numpy() for o in b.outputs]
    # the same batch captured in a graph replays to the same bits
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            b.forward()
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    for rep in range(2):
        for o in b.outputs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        replay_equal = all(torch.equal(b.outputs[m], eager[m]) for m in range(len(members)))
        assert replay_equal, rep
    del eager
    b.backward()
    torch.cuda.synchronize()
    backs = [i.cpu().numpy() for i in b.inputs]
    print("config5 batch done", flush=True)
    return members, data, outs, backs


@pytest.mark.parametrize("sid", range(len(CONFIG5)), ids=["x".join(map(str, s)) for s, _ in CONFIG5])
def test_config5_batch_matches_oracle(config5_batch, sid):
    members, data, outs, backs = config5_batch
    shape, grid = CONFIG5[sid]
    ch = oracle.Chain.paper(shape, grid)
    for c in range(3):
        m = 3 * sid + c
        expect = oracle.forward(ch, data[m].astype(np.complex128))
        assert np.linalg.norm(outs[m] - expect) / np.linalg.norm(expect) <= 1e-5, (shape, c)
        expect_b = oracle.backward(ch, outs[m].astype(np.complex128))
        assert np.linalg.norm(backs[m] - expect_b) / np.linalg.norm(expect_b) <= 1e-5, (shape, c)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_batch_real_members_share_launches(prec):
    # real-input members of one line length (and of two shapes of tile) in
    # one batch: the grouped r2c / c2r launches give each member's own
    # results bit for bit, and the oracle's
    specs = [((16, 16, 32), (4, 2)), ((8, 24, 32), (2, 3)), ((32, 8, 32), (2, 2)), ((16, 16, 32), (4, 2)),
             ((12, 10, 96), (3, 2))]
    plans = [Plan(s, g, kind="r2c", precision=prec) for s, g in specs]
    b = Batch(plans)
    rdt = np.float32 if prec == "f32" else np.float64
    data = []
    for m, p in enumerate(b.plans):
        u = inputs.gaussian_real(b.inputs[m].numel(), [31, m], rdt)
        b.inputs[m].copy_(torch.from_numpy(u))
        data.append(u)
    b.forward()
    torch.cuda.synchronize()
    outs = []
    for m, p in enumerate(b.plans):
        print("member", m, p.shape, p.grid, flush=True)
        ref = p.forward(torch.from_numpy(data[m]).cuda())
        torch.cuda.synchronize()
        got = b.outputs[m].cpu().numpy()
        assert got.tobytes() == ref.cpu().numpy().tobytes()
        ch = oracle.Chain.paper(p.shape, p.grid, kind="r2c")
        expect = oracle.forward(ch, data[m].astype(np.float64))
        assert np.linalg.norm(got - expect) / np.linalg.norm(expect) <= (1e-5 if prec == "f32" else 1e-12)
        outs.append(got)
    b.backward()
    torch.cuda.synchronize()
    for m, p in enumerate(b.plans):
        ref = p.backward(torch.from_numpy(outs[m]).cuda())
        torch.cuda.synchronize()
        assert b.inputs[m].cpu().numpy().tobytes() == ref.cpu().numpy().tobytes()
        assert np.linalg.norm(b.inputs[m].cpu().numpy() - data[m]) / np.linalg.norm(data[m]) <= \
            (1e-5 if prec == "f32" else 1e-12)
