"""Pins of the oracle's real-to-real transforms (the cosine/sine transforms
the method carries as "similar" transforms): library special cases, the
inverse relation, closed forms, brute force on tiny arrays, and the chain's
round trip."""
import numpy as np
import pytest
import scipy.fft as sf

import oracle

LIB = {("dct2", False): lambda x: sf.dct(x, type=2), ("dct2", True): lambda x: sf.dct(x, type=3),
       ("dst2", False): lambda x: sf.dst(x, type=2), ("dst2", True): lambda x: sf.dst(x, type=3)}


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 12, 17, 64])
@pytest.mark.parametrize("kind", oracle.R2R_KINDS)
@pytest.mark.parametrize("inverse", [False, True])
def test_matrix_equals_library_unnormalised_transform(n, kind, inverse):
    # scipy's unnormalised types 2 and 3 have the same definitions
    x = np.random.default_rng(n).standard_normal(n)
    got = oracle.r2r_matrix(n, kind, inverse) @ x
    ref = LIB[(kind, inverse)](x)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n", [1, 2, 7, 16, 30])
@pytest.mark.parametrize("kind", oracle.R2R_KINDS)
def test_type3_undoes_type2_up_to_2n(n, kind):
    F = oracle.r2r_matrix(n, kind, False)
    B = oracle.r2r_matrix(n, kind, True)
    assert np.abs(B @ F - 2 * n * np.eye(n)).max() < 1e-11 * n
    assert np.abs(F @ B - 2 * n * np.eye(n)).max() < 1e-11 * n


@pytest.mark.parametrize("n,m", [(8, 0), (8, 3), (13, 12), (16, 5)])
def test_cosine_and_sine_modes_are_deltas(n, m):
    j = np.arange(n)
    c = np.cos(np.pi * (2 * j + 1) * m / (2 * n))
    y = oracle.r2r_matrix(n, "dct2", False) @ c
    ref = np.zeros(n)
    ref[m] = 2 * n if m == 0 else n
    assert np.abs(y - ref).max() < 1e-11 * n
    s = np.sin(np.pi * (2 * j + 1) * (m + 1) / (2 * n))
    y = oracle.r2r_matrix(n, "dst2", False) @ s
    ref = np.zeros(n)
    ref[m] = 2 * n if m == n - 1 else n
    assert np.abs(y - ref).max() < 1e-11 * n


@pytest.mark.parametrize("shape,grid,kinds", [
    ((4, 6, 5), (2, 3), ("dct2", "dst2", "dct2")),
    ((3, 4, 2), (2,), ("dst2", "dst2", "dct2")),
    ((2, 3, 2, 3), (2, 1, 2), ("dct2", "dst2", "dst2", "dct2")),
])
@pytest.mark.parametrize("norm", ["forward", "none"])
def test_chain_equals_bruteforce(shape, grid, kinds, norm):
    ch = oracle.Chain.paper(shape, grid, kind="r2r", norm=norm, r2r=kinds)
    glob = np.random.default_rng(3).standard_normal(shape)
    x = oracle.scatter_global(glob, ch.input_layout())
    y = oracle.forward(ch, x)
    scales = [ch.scale(a, "forward") for a in range(len(shape))]
    ref = oracle.bruteforce_r2rn(glob, kinds, False, scales)
    got = oracle.gather_global(y, ch.output_layout())
    assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
    # the backward chain against brute force of the inverse transforms
    yb = oracle.backward(ch, oracle.scatter_global(glob, ch.output_layout()))
    refb = oracle.bruteforce_r2rn(glob, kinds, True, [ch.scale(a, "backward") for a in range(len(shape))])
    assert np.abs(oracle.gather_global(yb, ch.input_layout()) - refb).max() < 1e-12 * max(1.0, np.abs(refb).max())


def test_one_rank_equals_library_nd_transform():
    shape = (6, 4, 10)
    ch = oracle.Chain.paper(shape, (1, 1), kind="r2r", norm="none", r2r=("dct2", "dct2", "dct2"))
    glob = np.random.default_rng(5).standard_normal(shape)
    y = oracle.gather_global(oracle.forward(ch, oracle.scatter_global(glob, ch.input_layout())),
                             ch.output_layout())
    ref = sf.dctn(glob, type=2)
    assert np.abs(y - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("norm", ["forward", "backward", "none"])
def test_round_trip(norm):
    shape, grid = (12, 10, 16), (3, 2)
    ch = oracle.Chain.paper(shape, grid, kind="r2r", norm=norm, r2r=("dst2", "dct2", "dst2"))
    x = np.random.default_rng(8).standard_normal(int(np.prod(shape)))
    back = oracle.backward(ch, oracle.forward(ch, x))
    f = 1.0 if norm != "none" else float(np.prod([2 * n for n in shape]))
    assert np.abs(back - f * x).max() < 1e-11 * f


@pytest.mark.parametrize("kinds", [("dct2", "dst2", "dct2"), ("dst2", "dst2", "dst2")])
@pytest.mark.parametrize("norm", ["forward", "backward"])
def test_adjoints_satisfy_dot_product_identity(kinds, norm):
    # <F x, y> = <x, F^T y> and <B y, x> = <y, B^T x> in FP64
    shape, grid = (6, 8, 10), (2, 3)
    ch = oracle.Chain.paper(shape, grid, kind="r2r", norm=norm, r2r=kinds)
    rng = np.random.default_rng(11)
    n = int(np.prod(shape))
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    lhs = np.dot(oracle.forward(ch, x), y)
    rhs = np.dot(x, oracle.adjoint_forward(ch, y))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))
    lhs = np.dot(oracle.backward(ch, y), x)
    rhs = np.dot(y, oracle.adjoint_backward(ch, x))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_adjoint_is_the_inverse_with_the_special_element_reweighted():
    # type II transposed = type III with its special input doubled (cosine: first, sine: last)
    n = 9
    for kind, sp in (("dct2", 0), ("dst2", n - 1)):
        F = oracle.r2r_matrix(n, kind, False)
        B = oracle.r2r_matrix(n, kind, True)
        D = np.eye(n)
        D[sp, sp] = 2.0
        assert np.abs(F.T - B @ D).max() < 1e-12 * n
