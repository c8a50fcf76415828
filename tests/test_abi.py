"""Host-side checks of libpfft (no GPU needed): the library loads and exports
every function include/pfft.h declares, plans describe the same layouts as
the oracle, and bad arguments come back as error codes."""
import ctypes

import pytest

import oracle
from paper_1804_09536_amd import _lib


def test_library_exports_every_header_function():
    lib = _lib.load()
    names = _lib.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


LAYOUT_CASES = [
    ((512, 512, 512), (8, 8), None, "c2c"),
    ((256, 256, 256), (4, 4), None, "c2c"),
    ((32, 32, 32), (4,), [(0, 2)], "c2c"),
    ((64, 64, 64, 64), (2, 2, 4), None, "c2c"),
    ((512, 512, 512), (8, 8), None, "r2c"),
    ((42, 127, 256), (3, 4), None, "c2c"),
    ((5, 7, 6), (2, 3), None, "c2c"),
    ((3, 2, 4), (4, 3), None, "c2c"),
    ((16, 32, 8), (3, 5), None, "c2c"),       # uneven splits, power-of-two lengths
    ((4, 2, 8), (8, 3), None, "c2c"),         # empty blocks
    ((8, 16, 4, 32), (3, 1, 5), None, "c2c"),
]


@pytest.mark.parametrize("shape,grid,chain,kind", LAYOUT_CASES)
def test_plan_layouts_match_oracle(shape, grid, chain, kind):
    from paper_1804_09536_amd.plan import Plan
    p = Plan(shape, grid, kind=kind, chain=chain, layouts_only=True)
    ch = oracle.Chain.paper(shape, grid, kind=kind, steps=chain)
    assert p.num_layouts == len(ch.dirs)
    for li in range(p.num_layouts):
        lay = ch.layout(li)
        offs = lay.offsets()
        for r in range(lay.nranks):
            shp, st, off = p.local_block(li, r)
            assert (shp, st) == lay.block(r)
            assert off == offs[r]
        assert p.buffer_numel(li) == offs[-1]
    if kind == "r2c":
        lay = ch.layout(0, spectral=False)
        for r in range(lay.nranks):
            shp, st, off = p.local_block(0, r, real=True)
            assert (shp, st) == lay.block(r)


def _create(shape, grid, prec=0, kind=0, norm=0, chain=None, flags=0):
    lib = _lib.load()
    h = ctypes.c_void_p()
    shp = (ctypes.c_int64 * len(shape))(*shape)
    grd = (ctypes.c_int * max(1, len(grid)))(*grid)
    ch, n = None, 0
    if chain is not None:
        flat = [v for s in chain for v in s]
        ch, n = (ctypes.c_int * max(1, len(flat)))(*flat), len(chain)
    st = lib.pfft_plan_create(ctypes.byref(h), len(shape), shp, len(grid), grd, prec, kind, norm, ch, n, flags)
    if st == 0:
        lib.pfft_plan_destroy(h)
    return st


def test_error_codes():
    assert _create((16, 16, 16), (2, 2)) == 0
    assert _create((16, 16, 16), (2, 2, 2)) == -3        # grid dims must be < ndim
    assert _create((16, 0, 16), (2, 2)) == -2           # empty axis
    assert _create((16, 16, 16), (2, 0)) == -3          # empty grid direction
    assert _create((16, 16, 16), (2, 2), prec=7) == -4
    assert _create((16, 16, 16), (2, 2), kind=9) == -4
    assert _create((16, 16, 16), (2, 2), norm=5) == -1
    assert _create((16, 16, 16), (2, 2), flags=3) == -1
    assert _create((16, 16, 16), (2,), chain=[(0, 0)]) == -3   # onto a distributed axis
    assert _create((16, 16, 16), (2,), chain=[(3, 1)]) == -3   # no such direction
    assert _create((16, 16, 16), (4,), chain=[]) == -3          # axis 0 never whole
    assert _create((16, 16, 17), (2, 2)) == 0                   # direct-sum DFT kernel
    assert _create((4, 4, 10247), (2, 2)) == -5                 # prime: its Bluestein convolution (20580) exceeds the LDS
    assert _create((4, 4, 10247), (2, 2), flags=4) == 0         # layouts only: any length
    assert _create((16, 16, 16), (2, 2), flags=1 << 7) == -1    # unknown flag bit


def test_calls_before_binding_fail_cleanly():
    lib = _lib.load()
    from paper_1804_09536_amd.plan import Plan
    p = Plan((16, 16, 16), (2, 2))
    v = ctypes.c_void_p
    a, b, c = v(1 << 20), v(1 << 24), v(1 << 28)   # stand-in addresses, never dereferenced
    assert lib.pfft_forward(p._h, a, b, c, None) == -6
    assert lib.pfft_forward(None, None, None, None, None) == -1
    assert lib.pfft_redistribute(p._h, 0, 2, a, b, None) == -6
    assert _lib.strerror(-5) == "unsupported transform length"


def test_overlapping_buffers_are_refused():
    # checked before anything touches the device: a stage reading and writing
    # overlapping buffers would race
    lib = _lib.load()
    from paper_1804_09536_amd.plan import Plan
    p = Plan((16, 16, 16), (2, 2))   # 16^3 complex64: 32 KiB per buffer
    nb = 16 ** 3 * 8
    v = ctypes.c_void_p
    base = 1 << 24
    far = v(base + 4 * nb)
    for fn in (lib.pfft_forward, lib.pfft_backward, lib.pfft_adjoint_forward, lib.pfft_adjoint_backward):
        assert fn(p._h, v(base), v(base), far, None) == -1                  # in == out
        assert fn(p._h, v(base), v(base + nb - 16), far, None) == -1        # out starts inside in
        assert fn(p._h, v(base), v(base + nb), v(base + nb + 4096), None) == -1   # work inside out
        assert fn(p._h, v(base), v(base + nb), far, None) == -6             # disjoint: not bound yet
        # disjoint, with `out` right after the workspace (where a second workspace
        # buffer would start): still disjoint
        assert fn(p._h, v(base), v(base + 2 * nb), v(base + nb), None) == -6
    assert lib.pfft_redistribute(p._h, 0, 1, v(base), v(base + 256), None) == -1
    assert lib.pfft_redistribute(p._h, 0, 1, v(base), v(base + nb), None) == -6


@pytest.mark.parametrize("shape,grid,kind,placement,path,plain,destroyed", [
    ((64, 32, 16), (4, 4), "c2c", None, "fused", 1, 0),                          # 3 transforms: odd
    ((8, 8, 8, 8), (2, 2, 2), "c2c", None, "fused", 1, 0),                       # 4: the first runs in place
    ((8, 8, 8, 8), (2, 2, 2), "c2c", ("scatter", "gather"), "fused", 1, 1),      # first one leaves its layout
    ((16, 16, 16), (2, 2), "r2c", None, "fused", 2, 1),
    ((16, 16, 16), (2, 2), "c2c", None, "unfused", 1, 0),
    ((16, 16, 16), (2, 2), "c2c", None, "pack_realign", 1, 0),
])
def test_destroy_input_workspace(shape, grid, kind, placement, path, plain, destroyed):
    # the two-largest-buffers scheme: intermediates reuse a complex input
    from paper_1804_09536_amd.plan import Plan
    a = Plan(shape, grid, kind=kind, placement=placement, path=path)
    b = Plan(shape, grid, kind=kind, placement=placement, path=path, destroy_input=True)
    one = (a.buffer_numel(a.num_layouts - 1) * 8 + 255) // 256 * 256
    assert a.workspace_bytes() == plain * one
    assert b.workspace_bytes() == destroyed * one
    b.validate()


def test_r2r_plan_creation_checks():
    lib = _lib.load()
    h = ctypes.c_void_p()
    shp = (ctypes.c_int64 * 3)(16, 12, 8)
    grd = (ctypes.c_int * 2)(2, 2)
    ok = (ctypes.c_int * 3)(0, 1, 0)
    bad = (ctypes.c_int * 3)(0, 7, 0)
    assert lib.pfft_plan_create_r2r(ctypes.byref(h), 3, shp, 2, grd, 0, ok, 0, None, 0, 0) == 0
    lib.pfft_plan_destroy(h)
    assert lib.pfft_plan_create_r2r(ctypes.byref(h), 3, shp, 2, grd, 0, bad, 0, None, 0, 0) == -4
    assert lib.pfft_plan_create_r2r(ctypes.byref(h), 3, shp, 2, grd, 0, None, 0, None, 0, 0) == -1
    assert lib.pfft_plan_create(ctypes.byref(h), 3, shp, 2, grd, 0, 2, 0, None, 0, 0) == -4
    # no transposed output for real-to-real plans
    assert lib.pfft_plan_create_r2r(ctypes.byref(h), 3, shp, 2, grd, 0, ok, 0, None, 0, 1 << 9) == -5
    odd = (ctypes.c_int64 * 3)(16, 5, 8)   # length 5 has no radix plan for the cosine stage
    assert lib.pfft_plan_create_r2r(ctypes.byref(h), 3, odd, 2, grd, 0, ok, 0, None, 0, 0) == -5


def test_r2r_layouts_match_oracle_and_validate():
    from paper_1804_09536_amd.plan import Plan
    shape, grid = (24, 12, 48), (3, 2)
    p = Plan(shape, grid, kind="r2r", r2r=("dst2", "dct2", "dst2"))
    ch = oracle.Chain.paper(shape, grid, kind="r2r", r2r=("dst2", "dct2", "dst2"))
    for li in range(p.num_layouts):
        lay = ch.layout(li)
        offs = lay.offsets()
        for r in range(lay.nranks):
            assert p.local_block(li, r) == (lay.block(r)[0], lay.block(r)[1], offs[r])
    assert p.buffer_numel(0) == 24 * 12 * 48
    p.validate()


def test_buffers_of_2_31_elements_take_wide_offsets():
    # from 2^31 elements on, plans use the kernels' 64-bit-offset variants;
    # real-to-real plans have none and are refused
    from paper_1804_09536_amd.plan import Plan
    p = Plan((2048, 1024, 1024), (8, 8), device="cpu")
    assert p.buffer_numel(0) == 2 ** 31
    lib = _lib.load()
    h = ctypes.c_void_p()
    shp = (ctypes.c_int64 * 3)(2048, 1024, 1024)
    grd = (ctypes.c_int * 2)(8, 8)
    kinds = (ctypes.c_int * 3)(0, 0, 0)
    assert lib.pfft_plan_create_r2r(ctypes.byref(h), 3, shp, 2, grd, 0, kinds, 0, None, 0, 0) == -5


@pytest.mark.parametrize("shape,grid,kind", [((16, 24, 32), (2, 3), "c2c"), ((12, 16, 20), (4,), "r2c"),
                                             ((8, 12, 6, 10), (2, 2, 3), "c2c"), ((16, 24, 32), (2, 3), "c2c_tr")])
def test_forced_wide_offsets_validate(shape, grid, kind):
    from paper_1804_09536_amd.plan import Plan
    p = Plan(shape, grid, kind=kind[:3], transposed_out=kind.endswith("_tr"), device="cpu")
    p.set_tuning(wide_offsets=1)
    p.validate()


@pytest.mark.parametrize("alt", [1, 2, 3])
@pytest.mark.parametrize("shape,grid,tr", [((32, 48, 4096), (2, 3), False), ((3072, 4, 64), (4, 2), False),
                                           ((96, 128, 192), (2, 2), True), ((512, 512, 512), (8, 8), False)])
def test_radix_alt_plans_validate(shape, grid, tr, alt):
    # the alternative radix plan changes the stage kernels' tile shapes only
    # through their thread counts: the address emulation still covers every
    # destination element once
    from paper_1804_09536_amd.plan import Plan
    p = Plan(shape, grid, transposed_out=tr, device="cpu")
    p.set_tuning(radix_alt=alt)
    assert p.tuning()["radix_alt"] == alt
    p.validate()
    with pytest.raises(_lib.PfftError):
        p.set_tuning(radix_alt=4)


def test_weighted_energy_argument_checks():
    # checked before anything is launched, so no device is needed
    lib = _lib.load()
    v = ctypes.c_void_p
    a16, a8 = v(4096), v(4104)   # stand-in addresses: 16-byte and 8-byte aligned
    assert lib.pfft_weighted_energy(2, 4, a16, a16, a16, a16, None) == -4       # bad precision
    assert lib.pfft_weighted_energy(0, -1, a16, a16, a16, a16, None) == -1      # negative count
    assert lib.pfft_weighted_energy(0, 4, None, a16, a16, a16, None) == -1      # null input
    assert lib.pfft_weighted_energy(0, 4, a16, a16, None, a16, None) == -1      # null partials
    assert lib.pfft_weighted_energy(1, 4, a8, a16, a16, a16, None) == -1        # complex128 needs 16 bytes
    assert lib.pfft_weighted_energy_grad(0, 4, a16, a16, a16, a16, None) == -1  # grad overlaps u
    assert lib.pfft_weighted_energy_grad(0, 4, a16, a16, None, a8, None) == -1  # null gradient scalar
