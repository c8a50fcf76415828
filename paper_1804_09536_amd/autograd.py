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

from .plan import Plan


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


class _WeightedEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, uh, w):
        wu = w * uh
        ctx.save_for_backward(wu)
        return torch.vdot(uh, wu).real

    @staticmethod
    def backward(ctx, g):
        (wu,) = ctx.saved_tensors
        return wu * (2 * g), None


def weighted_energy(uh: torch.Tensor, w: torch.Tensor) -> torch.Tensor:
    """sum_k w(k) |uh(k)|^2 for a real weight w on the same buffer, with its
    gradient 2 w uh (torch's convention for complex inputs) formed in one
    pass: the loss of the differentiation workload without the chain of
    elementwise kernels autograd would record for it."""
    return _WeightedEnergy.apply(uh, w)


def wavenumber_weight(plan: Plan, layout: int = -1) -> torch.Tensor:
    """w(k) = |k|^2 on a (spectral) layout: signed integer wavenumbers on the
    full axes, 0..N/2 on the half axis of a real-input plan."""
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
    return w
