"""The alternative radix plan of the complex stage kernels (tuning field
radix_alt: 16 points per thread instead of 8, 8 instead of 16, and the other
power-of-two part for 3 * 2^a lengths) against the FP64 oracle, for every
length that has one, along a strided axis and along the contiguous last axis,
in both precisions; with differently stepping sides (transposed output),
where the stages keep their own kernels; and inside a batch, whose members
then leave the multi-transform kernel but give their own plans' results bit
for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_1804_09536_amd import inputs
from paper_1804_09536_amd.plan import Batch, Plan

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}
NPDT = {"f32": np.complex64, "f64": np.complex128}
# (strided length along axis 0, contiguous length along axis 2): each
# length with an alternative plan appears once in each role
PAIRS = [(32, 4096), (4096, 32), (48, 3072), (3072, 48), (64, 2048), (2048, 64), (96, 1536), (1536, 96),
         (128, 1024), (1024, 128), (192, 768), (768, 192), (256, 512), (512, 256), (384, 384)]


def relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("pair", PAIRS)
def test_radix_alt_matches_oracle(pair, prec):
    shape, grid = (pair[0], 4, pair[1]), (2, 2)
    print("case", shape, grid, prec, flush=True)
    p = Plan(shape, grid, precision=prec)
    p.set_tuning(radix_alt=3)
    p.validate()
    ch = oracle.Chain.paper(shape, grid)
    n = p.buffer_numel(0)
    u = inputs.uniform_complex(n, [41, pair[0], pair[1]], NPDT[prec])
    y = p.forward(_dev(u))
    got = _host(y)
    assert relerr(got, oracle.forward(ch, u.astype(np.complex128))) <= TOL[prec]
    z = _host(p.backward(y))
    assert relerr(z, oracle.backward(ch, got.astype(np.complex128))) <= TOL[prec]


@pytest.mark.parametrize("alt", [1, 2])
def test_radix_alt_per_mode_and_transposed(alt):
    # one mode at a time on the pencil workload's lengths, and a transposed
    # output whose last stage steps its sides differently
    for shape, grid, tr in [((64, 128, 512), (4, 2), False), ((96, 64, 128), (2, 4), True)]:
        print("case", shape, grid, alt, tr, flush=True)
        p = Plan(shape, grid, transposed_out=tr)
        p.set_tuning(radix_alt=alt)
        p.validate()
        ch = oracle.Chain.paper(shape, grid, transposed_out=tr)
        n = p.buffer_numel(0)
        u = inputs.uniform_complex(n, [42, alt], np.complex64)
        y = p.forward(_dev(u))
        got = _host(y)
        assert relerr(got, oracle.forward(ch, u.astype(np.complex128))) <= 1e-5
        z = _host(p.backward(y))
        assert relerr(z, oracle.backward(ch, got.astype(np.complex128))) <= 1e-5


def test_radix_alt_batch_members_match_their_plans():
    members = [((32, 16, 64), (2, 4)), ((48, 24, 96), (2, 2)), ((64, 64, 64), (4, 2))]
    plans = []
    for i, (s, g) in enumerate(members):
        p = Plan(s, g)
        p.set_tuning(radix_alt=3 if i != 1 else 0)
        plans.append(p)
    b = Batch(plans)
    data = []
    for m, p in enumerate(b.plans):
        u = inputs.uniform_complex(b.inputs[m].numel(), [43, m], np.complex64)
        b.inputs[m].copy_(torch.from_numpy(u))
        data.append(u)
    b.forward()
    torch.cuda.synchronize()
    for m, p in enumerate(b.plans):
        print("member", m, p.shape, p.grid, flush=True)
        ref = _host(p.forward(_dev(data[m])))
        assert _host(b.outputs[m]).tobytes() == ref.tobytes()
        ch = oracle.Chain.paper(p.shape, p.grid)
        assert relerr(ref, oracle.forward(ch, data[m].astype(np.complex128))) <= 1e-5
    b.backward()
    torch.cuda.synchronize()
    for m in range(len(b.plans)):
        assert relerr(_host(b.inputs[m]), data[m]) <= 1e-5
