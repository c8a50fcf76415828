"""Pins for the oracle's real transforms (footnote of Sec. 2: half index set
for real input), its adjoints and the differentiation workload's gradient."""
import numpy as np
import pytest

import oracle
from paper_1804_09536_amd import inputs

SHAPES = [((6, 4, 8), (2,)), ((5, 6, 9), (2, 3)), ((4, 6, 4, 6), (2, 1, 3)), ((8, 8, 8), (2, 2))]


def _cdot(a, b):
    return np.vdot(a, b)  # sum conj(a) * b


@pytest.mark.parametrize("shape,grid", SHAPES)
def test_r2c_is_truncated_c2c(shape, grid):
    ch_r = oracle.Chain.paper(shape, grid, kind="r2c")
    ch_c = oracle.Chain.paper(shape, grid, kind="c2c")
    n = int(np.prod(shape))
    x = inputs.gaussian_real(n, [20, n], np.float64)
    G = oracle.gather_global(x, ch_r.layout(0, spectral=False))
    full = oracle.gather_global(oracle.forward(ch_c, oracle.scatter_global(G.astype(np.complex128),
                                                                           ch_c.input_layout())),
                                ch_c.output_layout())
    half = oracle.gather_global(oracle.forward(ch_r, x), ch_r.output_layout())
    h = shape[-1] // 2 + 1
    assert np.allclose(half, full[..., :h], rtol=0, atol=1e-14)
    # Hermitian symmetry of the full spectrum of a real array
    idx = tuple((-np.arange(s)) % s for s in shape)
    mirrored = full[np.ix_(*idx)]
    assert np.allclose(full, np.conj(mirrored), rtol=0, atol=1e-14)
    # library special case
    assert np.allclose(half, np.fft.rfftn(G, norm="forward"), rtol=0, atol=1e-14)


@pytest.mark.parametrize("shape,grid", SHAPES)
def test_c2r_inverts_r2c(shape, grid):
    ch = oracle.Chain.paper(shape, grid, kind="r2c")
    n = int(np.prod(shape))
    x = inputs.gaussian_real(n, [21, n], np.float64)
    back = oracle.backward(ch, oracle.forward(ch, x))
    assert np.allclose(back, x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape,grid", SHAPES)
@pytest.mark.parametrize("norm", ["forward", "backward"])
def test_adjoint_dot_product_c2c(shape, grid, norm):
    ch = oracle.Chain.paper(shape, grid, norm=norm)
    n = int(np.prod(shape))
    x = inputs.uniform_complex(n, [22, 0], np.complex128)
    z = inputs.uniform_complex(n, [22, 1], np.complex128)
    lhs = _cdot(oracle.forward(ch, x), z)
    rhs = _cdot(x, oracle.adjoint_forward(ch, z))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    lhs = _cdot(oracle.backward(ch, z), x)
    rhs = _cdot(z, oracle.adjoint_backward(ch, x))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("shape,grid", SHAPES)
def test_adjoint_dot_product_r2c(shape, grid):
    # real inner product Re<a, b>
    ch = oracle.Chain.paper(shape, grid, kind="r2c")
    n = int(np.prod(shape))
    m = int(np.prod(ch.spectral_shape()))
    x = inputs.gaussian_real(n, [23, 0], np.float64)
    z = inputs.uniform_complex(m, [23, 1], np.complex128)
    lhs = np.real(_cdot(oracle.forward(ch, x), z))
    rhs = float(np.dot(x, oracle.adjoint_forward(ch, z)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
    # adjoint of the c2r backward
    y = inputs.gaussian_real(n, [23, 2], np.float64)
    lhs = float(np.dot(oracle.backward(ch, z), y))
    rhs = np.real(_cdot(z, oracle.adjoint_backward(ch, y)))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_loss_gradient_exact_central_differences():
    # L(u) is a quadratic form, so (L(u+h e) - L(u-h e)) / 2h is exact for any
    # h; h = 1 leaves only rounding error.
    shape, grid = (16, 16, 16), (4, 4)
    ch = oracle.Chain.paper(shape, grid, kind="r2c")
    n = int(np.prod(shape))
    u = inputs.gaussian_real(n, [24], np.float64)
    wg = oracle.wavenumber_weight(ch.spectral_shape(), real_last=True)
    w = np.real(oracle.scatter_global(wg.astype(np.complex128), ch.output_layout()))
    loss, grad = oracle.loss_and_grad(ch, u, w)
    rng = np.random.default_rng(7)
    for i in rng.choice(n, size=48, replace=False):
        e = np.zeros(n)
        e[i] = 1.0
        lp, _ = oracle.loss_and_grad(ch, u + e, w)
        lm, _ = oracle.loss_and_grad(ch, u - e, w)
        fd = (lp - lm) / 2.0
        assert abs(fd - grad[i]) <= 1e-9 * max(1.0, abs(fd)), (i, fd, grad[i])


def test_wavenumber_weight_values():
    w = oracle.wavenumber_weight((4, 6, 4), real_last=True, hermitian=False)
    assert w.shape == (4, 6, 4)
    # axis 0 wavenumbers 0,1,-2,-1; axis 1 0,1,2,-3,-2,-1; half axis 0..3
    assert w[2, 3, 3] == 4 + 9 + 9
    assert w[3, 5, 1] == 1 + 1 + 1
    # Hermitian weight of the half axis of a real length 6: bins 1 and 2 stand
    # for two bins each, bins 0 and 3 (the Nyquist bin) for one
    wh = oracle.wavenumber_weight((4, 6, 4), real_last=True)
    assert wh[2, 3, 3] == 4 + 9 + 9
    assert wh[3, 5, 1] == 2 * (1 + 1 + 1)
    assert wh[1, 1, 0] == 1 + 1
    # an odd real length 7 has no Nyquist bin: bins 1..3 all double
    wo = oracle.wavenumber_weight((2, 2, 4), real_last=True, real_n=7)
    assert wo[0, 0, 3] == 2 * 9


@pytest.mark.parametrize("shape,grid", [((8, 6, 10), (2, 3)), ((6, 4, 7), (2,)), ((4, 6, 4, 6), (2, 1, 3))])
def test_hermitian_loss_equals_full_spectrum_sum(shape, grid):
    # the half-spectrum loss with the Hermitian weight equals sum over ALL k
    # of |k|^2 |FFT(u)(k)|^2, computed from the full complex transform of the
    # same real field (numpy's fftn, a library special case of Eq. multifft)
    ch = oracle.Chain.paper(shape, grid, kind="r2c")
    n = int(np.prod(shape))
    u = inputs.gaussian_real(n, [25], np.float64)
    wg = oracle.wavenumber_weight(ch.spectral_shape(), real_last=True, real_n=shape[-1])
    w = np.real(oracle.scatter_global(wg.astype(np.complex128), ch.output_layout()))
    loss, _ = oracle.loss_and_grad(ch, u, w)
    G = oracle.gather_global(u, ch.layout(0, spectral=False))
    full = np.fft.fftn(G, norm="forward")
    wf = oracle.wavenumber_weight(shape, real_last=False)
    assert abs(loss - float(np.sum(wf * np.abs(full) ** 2))) <= 1e-12 * abs(loss)
