"""Host-side property checks of the plan engine over random shapes, grids,
chains, kinds, placements and paths (no GPU): every plan's layouts equal the
oracle's, and the emulation of every kernel's address arithmetic stays in
bounds and writes every destination element exactly once."""
import os

import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_1804_09536_amd import _lib
from paper_1804_09536_amd.plan import Plan

LENGTHS = st.sampled_from([1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 17, 24, 32, 48, 64])


@st.composite
def plan_cases(draw):
    ndim = draw(st.integers(2, 4))
    shape = tuple(draw(LENGTHS) for _ in range(ndim))
    ngrid = draw(st.integers(1, ndim - 1))
    grid = tuple(draw(st.integers(1, 5)) for _ in range(ngrid))
    kind = draw(st.sampled_from(["c2c", "r2c"]))
    names = ["gather", "scatter", "direct", "final"]
    placement = (draw(st.sampled_from(names)), draw(st.sampled_from(names)))
    path = draw(st.sampled_from(["fused", "unfused", "pack_realign"]))
    chain = None
    if draw(st.booleans()) and ngrid == 1:
        # slab moved onto another whole axis
        chain = [(0, draw(st.integers(1, ndim - 1)))]
    transposed = draw(st.booleans())
    return shape, grid, kind, placement, path, chain, transposed


@settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(plan_cases())
def test_random_plans_validate_and_match_oracle_layouts(case):
    shape, grid, kind, placement, path, chain, transposed = case
    try:
        p = Plan(shape, grid, kind=kind, placement=placement, path=path, chain=chain, transposed_out=transposed)
    except _lib.PfftError as e:
        # only legitimate refusals: r2c needs the last axis whole in layout 0
        assert e.status == -3 and kind == "r2c"
        return
    p.validate()
    ch = oracle.Chain.paper(shape, grid, kind=kind, steps=chain, transposed_out=transposed)
    assert p.num_layouts == len(ch.dirs)
    for li in range(p.num_layouts):
        lay = ch.layout(li)
        offs = lay.offsets()
        assert p.axis_order(li) == lay.storage
        for r in range(lay.nranks):
            shp, sta, off = p.local_block(li, r)
            assert (shp, sta, off) == (lay.block(r)[0], lay.block(r)[1], offs[r])


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(os.path.dirname(_lib.LIB_PATH), "nonexistent.so"))
    with pytest.raises(OSError):
        Plan((8, 8, 8), (2, 2))
