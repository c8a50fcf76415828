"""The paper's two appendix programs as oracle tests: every rank fills its
local input array with j + j*I (j = local linear index), a forward and a
backward transform follow, and every value must come back to within 1e-8
(App. A: 42x127x256 on a 2-D grid; App. B: 16x17x18x19 on a 3-D grid; the 4-D
program's ndims=3 argument to exchange is read as 4)."""
import numpy as np
import pytest

import oracle
from paper_1804_09536_amd import inputs


def _roundtrip(shape, grid):
    ch = oracle.Chain.paper(shape, grid)
    lay = ch.input_layout()
    sizes = [int(np.prod(lay.block(r)[0])) for r in range(lay.nranks)]
    a = inputs.local_index_fill(sizes)
    back = oracle.backward(ch, oracle.forward(ch, a))
    j = np.real(a)
    assert np.all(np.abs(back.real - j) < 1e-8)
    assert np.all(np.abs(back.imag - j) < 1e-8)


@pytest.mark.parametrize("grid", [(2, 2), (3, 4)])
def test_appendix_a_pencil_c2c(grid):
    _roundtrip((42, 127, 256), grid)


@pytest.mark.parametrize("grid", [(2, 2, 2), (1, 2, 3)])
def test_appendix_b_4d_c2c(grid):
    _roundtrip((16, 17, 18, 19), grid)
