"""paper_1804_09536_amd: the transpose-based parallel multidimensional FFT of
Dalcin, Mortensen & Keyes (arXiv:1804.09536) for one AMD Instinct MI355X.

Virtual ranks of a Cartesian process grid keep their local blocks in one HBM
allocation per alignment; each global redistribution is fused into the HIP
kernel of the next partial transform.  See ``include/pfft.h`` for the C ABI.

Importing this package loads nothing; ``Plan`` loads ``libpfft.so`` on first
use and raises if it has not been built.
"""
from __future__ import annotations

__all__ = ["Plan", "PfftError", "build"]


def __getattr__(name):
    if name == "Plan":
        from .plan import Plan
        return Plan
    if name == "PfftError":
        from ._lib import PfftError
        return PfftError
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
