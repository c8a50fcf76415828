"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module draws random numbers and nothing else: it holds none of the
transform's arithmetic and imports neither the HIP binding nor the oracle.
Every generator returns a flat buffer of ``n`` elements.  Because the values
are independent and identically distributed, the flat buffer is used directly
as the rank-blocked buffer of a transform's input layout.

Recipes (stated once here, used everywhere):
  * complex uniform: real and imaginary parts i.i.d. U[-1, 1], drawn in FP64
    from ``numpy.random.default_rng(seed)`` (real parts first, then imaginary
    parts), then rounded to the requested complex dtype;
  * real Gaussian: i.i.d. N(0, 1) in FP64 from ``default_rng(seed)``, rounded
    to the requested real dtype;
  * index payload: element i holds the value i encoded exactly (complex64:
    real = i mod 2^20, imag = i div 2^20, both exact in FP32), which makes any
    misplaced, lost or duplicated element visible after a permutation.
"""
from __future__ import annotations

import numpy as np

_REAL_OF = {np.dtype(np.complex64): np.float32, np.dtype(np.complex128): np.float64}


def uniform_complex(n: int, seed, dtype=np.complex64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=n)
    im = rng.uniform(-1.0, 1.0, size=n)
    out = np.empty(n, dtype=dtype)
    out.real = re.astype(_REAL_OF[np.dtype(dtype)])
    out.imag = im.astype(_REAL_OF[np.dtype(dtype)])
    return out


def gaussian_real(n: int, seed, dtype=np.float32) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=n).astype(dtype)


def index_payload(n: int, dtype=np.complex64) -> np.ndarray:
    i = np.arange(n, dtype=np.int64)
    out = np.empty(n, dtype=dtype)
    out.real = (i % (1 << 20)).astype(np.float64)
    out.imag = (i // (1 << 20)).astype(np.float64)
    return out


def decode_index_payload(buf: np.ndarray) -> np.ndarray:
    return buf.real.astype(np.int64) + (buf.imag.astype(np.int64) << 20)


def local_index_fill(block_sizes) -> np.ndarray:
    """The appendix programs' fill: every rank's local array holds
    j + j*I at local linear index j.  ``block_sizes`` lists the element count
    of each rank block in rank order; returns complex128."""
    parts = [np.arange(int(c), dtype=np.float64) for c in block_sizes]
    j = np.concatenate(parts) if parts else np.zeros(0)
    return (j + 1j * j).astype(np.complex128)


def uniform_complex_device(n: int, seed: int, dtype, device):
    """Device-side variant for multi-gigabyte timing inputs: real and
    imaginary parts i.i.d. U[-1, 1] from torch's generator seeded with
    `seed` (a different stream from the numpy recipe above; used only where
    values are not compared with the oracle)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    buf = torch.rand(2 * n, dtype=rdt, device=device, generator=g).mul_(2.0).sub_(1.0)
    return torch.view_as_complex(buf.view(n, 2))
