"""Pins for the oracle's transforms (Sec. 2, Eqs. 1-2, Eq. multifft,
Eq. fftn_forward/fftn_backward) against closed forms, brute force and a
library special case."""
import cmath
import math

import numpy as np
import pytest

import oracle
from paper_1804_09536_amd import inputs


def _direct_line(x, sign):
    # Eq. 1 without the 1/N, written as a plain double loop.
    n = len(x)
    out = []
    for k in range(n):
        acc = 0j
        for j in range(n):
            acc += x[j] * cmath.exp(sign * 2j * math.pi * ((j * k) % n) / n)
        out.append(acc)
    return np.array(out)


# composite lengths run the mixed-radix recursion (factors 2, 3, 5, 7, 11 and
# their products, several levels deep), primes the direct sum, powers of two
# the radix-2 passes
@pytest.mark.parametrize("n", list(range(1, 21)) + [21, 24, 25, 27, 30, 32, 35, 36, 45, 48, 49, 55, 63, 64, 77,
                                                    96, 105, 121])
@pytest.mark.parametrize("sign", [-1, 1])
def test_dft1_equals_direct_sum(n, sign):
    x = inputs.uniform_complex(n, [10, n], np.complex128)
    assert np.allclose(oracle.dft1(x, sign), _direct_line(x, sign), rtol=0, atol=1e-12 * n)


@pytest.mark.parametrize("n", [192, 384, 768, 1000, 1536, 2048, 3072, 6144, 4099, 10247, 2 * 3 * 5 * 7 * 11])
def test_dft1_long_lines_equal_numpy_fft(n):
    # library special case: numpy's unnormalised fft / ifft are Eq. 1 and Eq. 2
    # without the factor; rounding grows like log n (mixed radix, radix 2) or
    # sqrt(n) (direct sum of a prime length)
    x = inputs.uniform_complex(n, [13, n], np.complex128)
    for sign, ref in ((-1, np.fft.fft(x)), (1, np.fft.ifft(x) * n)):
        got = oracle.dft1(x, sign)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13


@pytest.mark.parametrize("shape", [(4, 6, 5), (3, 5, 7, 2), (2, 1, 8), (9,), (3, 4)])
def test_bruteforce_equals_numpy_fftn(shape):
    # Library special case: numpy's fftn with norm="forward" is Eq. multifft.
    n = int(np.prod(shape))
    G = inputs.uniform_complex(n, [11, n], np.complex128).reshape(shape)
    got = oracle.bruteforce_dftn(G, -1, 1.0 / n)
    assert np.allclose(got, np.fft.fftn(G, norm="forward"), rtol=0, atol=1e-13)
    got_b = oracle.bruteforce_dftn(G, +1, 1.0)
    assert np.allclose(got_b, np.fft.ifftn(G, norm="forward"), rtol=0, atol=1e-12)


CHAINS = [
    ((4, 6, 5), (2,), None),
    ((6, 4, 8), (3,), None),
    ((5, 7, 6), (2, 3), None),
    ((3, 2, 4), (4, 3), None),          # empty blocks
    ((4, 6, 5, 3), (2, 2, 3), None),    # 4-D
    ((8, 6, 10), (4,), [(0, 2)]),       # slab, axis 0 -> axis 2
    ((8, 8, 8), (2, 2), None),
]


@pytest.mark.parametrize("shape,grid,steps", CHAINS)
def test_forward_chain_equals_bruteforce(shape, grid, steps):
    ch = oracle.Chain.paper(shape, grid, steps=steps)
    n = int(np.prod(shape))
    u0 = inputs.uniform_complex(n, [12, n], np.complex128)
    uh = oracle.forward(ch, u0)
    G = oracle.gather_global(u0, ch.input_layout())
    expect = oracle.bruteforce_dftn(G, -1, 1.0 / n)
    assert np.allclose(oracle.gather_global(uh, ch.output_layout()), expect, rtol=0, atol=1e-13)
    back = oracle.backward(ch, uh)
    assert np.allclose(back, u0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape,grid", [((4, 6, 5), (2, 3)), ((8, 4, 6), (2,))])
def test_delta_closed_form(shape, grid):
    ch = oracle.Chain.paper(shape, grid)
    jstar = tuple(min(2, s - 1) for s in shape)
    G = np.zeros(shape, np.complex128)
    G[jstar] = 1.0
    uh = oracle.gather_global(oracle.forward(ch, oracle.scatter_global(G, ch.input_layout())),
                              ch.output_layout())
    k = np.indices(shape)
    phase = sum(k[m] * jstar[m] / shape[m] for m in range(len(shape)))
    expect = np.exp(-2j * np.pi * phase) / np.prod(shape)
    assert np.allclose(uh, expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("shape,grid", [((4, 6, 5), (2, 3)), ((8, 4, 6), (2,)), ((4, 4, 3, 5), (2, 2, 1))])
def test_plane_wave_gives_unit_delta(shape, grid):
    ch = oracle.Chain.paper(shape, grid)
    m = tuple((2 * i + 1) % s for i, s in enumerate(shape))
    j = np.indices(shape)
    G = np.exp(2j * np.pi * sum(m[a] * j[a] / shape[a] for a in range(len(shape))))
    uh = oracle.gather_global(oracle.forward(ch, oracle.scatter_global(G, ch.input_layout())),
                              ch.output_layout())
    expect = np.zeros(shape, np.complex128)
    expect[m] = 1.0
    assert np.allclose(uh, expect, rtol=0, atol=1e-14)


def test_parseval_and_linearity():
    shape, grid = (6, 8, 10), (2, 2)
    ch = oracle.Chain.paper(shape, grid)
    n = int(np.prod(shape))
    a = inputs.uniform_complex(n, [13, 0], np.complex128)
    b = inputs.uniform_complex(n, [13, 1], np.complex128)
    fa, fb = oracle.forward(ch, a), oracle.forward(ch, b)
    assert math.isclose(np.sum(np.abs(a) ** 2), n * np.sum(np.abs(fa) ** 2), rel_tol=1e-13)
    fab = oracle.forward(ch, 2.0 * a - 3j * b)
    assert np.allclose(fab, 2.0 * fa - 3j * fb, rtol=0, atol=1e-14)


@pytest.mark.parametrize("norm", ["backward", "none"])
def test_other_normalisations(norm):
    shape, grid = (4, 6, 8), (2, 2)
    ch = oracle.Chain.paper(shape, grid, norm=norm)
    n = int(np.prod(shape))
    u0 = inputs.uniform_complex(n, [14], np.complex128)
    G = oracle.gather_global(u0, ch.input_layout())
    got = oracle.gather_global(oracle.forward(ch, u0), ch.output_layout())
    assert np.allclose(got, np.fft.fftn(G), rtol=0, atol=1e-11)
    back = oracle.backward(ch, oracle.forward(ch, u0))
    scale = 1.0 if norm == "backward" else float(n)
    assert np.allclose(back, scale * u0, rtol=0, atol=1e-10)


@pytest.mark.parametrize("shape", [(4, 6, 5), (3, 5, 7, 2), (8, 1, 6)])
def test_dft_bins_equal_bruteforce(shape):
    n = int(np.prod(shape))
    G = inputs.uniform_complex(n, [15, n], np.complex128).reshape(shape)
    full = oracle.bruteforce_dftn(G, -1, 1.0 / n)
    rng = np.random.default_rng(3)
    bins = [tuple(int(rng.integers(0, s)) for s in shape) for _ in range(6)]
    got = oracle.dft_bins(G, bins, -1, 1.0 / n)
    assert np.allclose(got, [full[b] for b in bins], rtol=0, atol=1e-14)


def test_layout_offset_matches_scatter():
    shape, grid = (5, 7, 6), (2, 3)
    ch = oracle.Chain.paper(shape, grid)
    G = np.arange(np.prod(shape)).reshape(shape).astype(np.complex128)
    for li in range(len(ch.dirs)):
        lay = ch.layout(li)
        buf = oracle.scatter_global(G, lay)
        for g in [(0, 0, 0), (4, 6, 5), (2, 3, 1), (1, 5, 4)]:
            assert buf[oracle.layout_offset(lay, g)] == G[g]
