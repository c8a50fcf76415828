"""Host emulation of every kernel launch of the full-size plans, in the launch
configuration the bench times (default tiles, placements and XCD tile order):
each access stays inside its rank block and buffer, every destination element
is written exactly once, the XCD tile order is a permutation, and source and
destination of every position are the same global element (Eq. gt)."""
import pytest

from paper_1804_09536_amd.plan import Plan

FULL = [
    ((512, 512, 512), (8, 8), "c2c", None),        # the metric workload
    ((512, 512, 512), (8, 8), "c2c", ("gather", "gather")),
    ((512, 512, 512), (8, 8), "r2c", None),
    ((64, 64, 64, 64), (2, 2, 4), "c2c", None),
    ((256, 256, 256), (4, 4), "r2c", None),        # the differentiation workload
    # the mixed batch's shapes and grids
    ((64, 64, 64), (4,), "c2c", None),
    ((96, 96, 96), (8,), "c2c", None),
    ((192, 192, 192), (4, 4), "c2c", None),
    ((384, 384, 384), (8, 8), "c2c", None),
    ((128, 256, 512), (4, 8), "c2c", None),
]


@pytest.mark.parametrize("shape,grid,kind,placement", FULL)
def test_full_size_plans_validate(shape, grid, kind, placement):
    p = Plan(shape, grid, kind=kind, placement=placement, device="cpu")
    p.validate()


def test_forced_xcd_order_validates():
    # the XCD tile order forced onto every complex strided stage (wrapped
    # tiles and gathering stages included) stays a permutation of the tiles
    p = Plan((24, 48, 96), (2, 3), device="cpu")
    p.set_tuning(xcd_order=1)
    p.validate()
