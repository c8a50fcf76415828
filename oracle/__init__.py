"""CPU FP64 oracle for the transpose-based parallel multidimensional FFT
(Dalcin, Mortensen & Keyes, arXiv:1804.09536).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_1804_09536_amd``) and never imports it.

Every function here is pinned by the ``tests/test_oracle_*.py`` checks
(brute force, closed forms, library special cases, two independent
redistribution formulations, dot-product adjoint tests, exact finite
differences); none is left "parity unpinned".
"""
from .core import *  # noqa: F401,F403
from .core import build  # noqa: F401
