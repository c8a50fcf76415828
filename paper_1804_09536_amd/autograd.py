"""Differentiable forward / backward transforms for torch.autograd.

The gradient of a transform is its adjoint under the real inner product
(``pfft_adjoint_forward`` / ``pfft_adjoint_backward``: reversed chain, inverse
redistributions, conjugate sign, the same per-axis factors; for real input the
half-spectrum adjoint), which is exactly torch's convention for complex
gradients: for y = A x the incoming gradient g maps to A^H g, and for a real
input the real part.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import check
from .plan import Plan, _ptr, _stream_handle


class _Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.forward(x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.adjoint_forward(g.contiguous()), None


class _Backward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.backward(x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.adjoint_backward(g.contiguous()), None


def _check(plan: Plan):
    if plan.destroy_input:
        raise ValueError("autograd needs a plan that leaves its inputs intact (destroy_input=False)")


def forward(x: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Distributed forward FFT of the rank-blocked buffer x (input layout),
    differentiable."""
    _check(plan)
    return _Forward.apply(x, plan)


def backward(x: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Distributed backward FFT (output layout -> input layout), differentiable."""
    _check(plan)
    return _Backward.apply(x, plan)


def global_indices(plan: Plan, layout: int, real: bool = False, device=None):
    """Per-axis global index of every element of a layout's buffer, as a list
    of int64 tensors (one per axis), from the plan's block descriptions."""
    device = device if device is not None else plan.device
    P = 1
    for g in plan.grid:
        P *= g
    nd = len(plan.shape)
    parts = [[] for _ in range(nd)]
    for r in range(P):
        shp, st, _ = plan.local_block(layout, r, real=real)
        if any(s == 0 for s in shp):
            continue
        axes = [torch.arange(st[m], st[m] + shp[m], dtype=torch.int64) for m in range(nd)]
        grids = torch.meshgrid(*axes, indexing="ij")
        for m in range(nd):
            parts[m].append(grids[m].reshape(-1))
    return [torch.cat(p).to(device) for p in parts]


_ENERGY = {torch.complex64: (0, torch.float32), torch.complex128: (1, torch.float64)}


def _energy_args(uh, w):
    if uh.dtype not in _ENERGY:
        raise TypeError("expected complex64 or complex128, got %s" % uh.dtype)
    prec, rdt = _ENERGY[uh.dtype]
    if w.dtype != rdt or w.numel() != uh.numel() or not (uh.is_cuda and w.is_cuda):
        raise ValueError("the weight must be a %s device tensor with one value per element" % rdt)
    return prec, rdt, uh.contiguous(), w.contiguous()


class _WeightedEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, uh, w):
        prec, rdt, uh, w = _energy_args(uh, w)
        lib = _lib.load()
        partials = torch.empty(_lib.ENERGY_PARTIALS, dtype=torch.float64, device=uh.device)
        loss = torch.empty((), dtype=rdt, device=uh.device)
        check(lib.pfft_weighted_energy(prec, uh.numel(), _ptr(uh), _ptr(w), _ptr(partials), _ptr(loss),
                                       _stream_handle(uh.device)), "pfft_weighted_energy")
        ctx.prec = prec
        ctx.save_for_backward(uh, w)
        return loss

    @staticmethod
    def backward(ctx, g):
        uh, w = ctx.saved_tensors
        g = g.to(w.dtype).contiguous()
        grad = torch.empty_like(uh)
        check(_lib.load().pfft_weighted_energy_grad(ctx.prec, uh.numel(), _ptr(uh), _ptr(w), _ptr(g), _ptr(grad),
                                                    _stream_handle(uh.device)), "pfft_weighted_energy_grad")
        return grad, None


def weighted_energy(uh: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """sum_k w(k) |uh(k)|^2 for a real weight w (the real type of uh) on the
    same buffer, and its gradient 2 w uh (torch's convention for complex
    inputs), each in one pass of the library's kernels (pfft_weighted_energy,
    pfft_weighted_energy_grad): the loss of the differentiation workload."""
    return _WeightedEnergy.apply(uh, w)


def wavenumber_weight(plan: Plan, layout: int = -1, hermitian: bool = True) -> torch.Tensor:
    """w(k) = |k|^2 on a (spectral) layout: signed integer wavenumbers on the
    full axes, 0..N/2 on the half axis of a real-input plan.  For a real-input
    plan with ``hermitian`` set, a half-axis bin k with 0 < k < N - k stands
    for the two bins k and N - k of the full spectrum (equal magnitudes for a
    real field, equal |k|^2) and carries twice the weight: the weighted energy
    of the stored half spectrum is then the sum over the whole spectrum."""
    if layout < 0:
        layout = plan.num_layouts + layout
    idx = global_indices(plan, layout)
    nd = len(plan.shape)
    real = plan.kind == "r2c"
    w = torch.zeros(idx[0].numel(), dtype=torch.float64, device=idx[0].device)
    for m in range(nd):
        n = plan.shape[m]
        k = idx[m]
        if not (real and m == nd - 1):
            k = torch.where(k >= (n + 1) // 2, k - n, k)
        w += (k * k).to(torch.float64)
    if real and hermitian:
        n, k = plan.shape[-1], idx[-1]
        w = torch.where((k > 0) & (k < n - k), 2.0 * w, w)
    return w
