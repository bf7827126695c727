"""Differentiation form of the energy: a torch.autograd.Function whose
backward is the hand-written adjoint kernel of the library, with the HVP as
its double backward.

    E = energy(m, theta, Lx, Ly)          # m [batch][3][N] or [3][N] on the GPU
    dE/dm      = g(m)                      (moto_energy_grad)
    dE/dtheta  = partials                  (moto_energy_grad, FP64 reductions)
    d(g.u)/dm  = A u                       (moto_hessian_apply: the Euclidean HVP)
    d(g.u)/dtheta = mixed partials         (moto_param_mixed)
    d(dE/dtheta . w)/dm = sum_q w_q dg/dtheta_q   (moto_param_grad_apply)

theta = (J_0..J_{ns-1}, D_0..D_{ns-1}, K, Bx, By, Bz) as a float64 tensor.
E is linear in theta, so every second derivative in theta alone vanishes.
Every value comes from the HIP kernels; this module only marshals tensors.
"""
from __future__ import annotations

from collections import OrderedDict

import torch

from . import moto as M


def _split_theta(theta: torch.Tensor, ns: int):
    t = theta.detach().double().cpu().tolist()
    return t[:ns], t[ns:2 * ns], t[2 * ns], tuple(t[2 * ns + 1:2 * ns + 4])


_PLANS: "OrderedDict[tuple, M.Plan]" = OrderedDict()
_PLAN_CACHE = 8


def _plan(Lx: int, Ly: int, theta: torch.Tensor) -> M.Plan:
    """The plan of (Lx, Ly, theta), reused across forward and backward calls
    (a plan holds shell tables and a pinned read-back buffer); the least
    recently used of more than eight is closed."""
    ns = (theta.numel() - 4) // 2
    J, D, K, B = _split_theta(theta, ns)
    key = (Lx, Ly, tuple(J), tuple(D), K, B)
    plan = _PLANS.get(key)
    if plan is None:
        plan = M.Plan(Lx, Ly, J, D, K, B)
        _PLANS[key] = plan
        while len(_PLANS) > _PLAN_CACHE:
            _, old = _PLANS.popitem(last=False)
            torch.cuda.synchronize()  # nothing queued may still use it
            old.close()
    else:
        _PLANS.move_to_end(key)
    return plan


def _batch(m: torch.Tensor, N: int) -> int:
    return m.numel() // (3 * N)


class _GradFn(torch.autograd.Function):
    """(m, theta) -> (g(m) [like m], dE/dtheta [batch][n_params] float64)."""

    @staticmethod
    def forward(ctx, m, theta, Lx, Ly):
        m = m.contiguous()
        plan = _plan(Lx, Ly, theta)
        _, g, _, _, dth = M.moto_energy_grad(plan, m, want_grad=True, want_c=False, want_F=False,
                                             want_dtheta=True)
        ctx.save_for_backward(m, theta)
        ctx.dims = (Lx, Ly)
        return g.view_as(m), dth

    @staticmethod
    def backward(ctx, gg, gdth):
        m, theta = ctx.saved_tensors
        Lx, Ly = ctx.dims
        plan = _plan(Lx, Ly, theta)
        N = Lx * Ly
        B = _batch(m, N)
        gm = None
        gth = None
        if gg is not None:
            gg = gg.contiguous().to(m.dtype)
            gm = M.moto_hessian_apply(plan, gg, batch=B).view_as(m)
            gth = M.moto_param_mixed(plan, m, gg, batch=B).sum(0)
        if gdth is not None:
            w = gdth.contiguous().double().view(B, -1)
            extra = torch.empty_like(m)
            M._check(M.lib().moto_param_grad_apply(plan.handle, M._dt(m), B, M._ptr(m), M._ptr(w), M._ptr(extra),
                                                   M._stream()), "moto_param_grad_apply")
            gm = extra if gm is None else gm + extra
        if gth is not None:
            gth = gth.to(theta.dtype)
        return gm, gth, None, None


class _EnergyFn(torch.autograd.Function):
    """(m, theta) -> E [batch] (float64)."""

    @staticmethod
    def forward(ctx, m, theta, Lx, Ly):
        m = m.contiguous()
        plan = _plan(Lx, Ly, theta)
        E, _, _, _, _ = M.moto_energy_grad(plan, m, want_grad=False, want_c=False, want_F=False)
        ctx.save_for_backward(m, theta)
        ctx.dims = (Lx, Ly)
        return E

    @staticmethod
    def backward(ctx, gE):
        m, theta = ctx.saved_tensors
        Lx, Ly = ctx.dims
        g, dth = _GradFn.apply(m, theta, Lx, Ly)
        B = _batch(m, Lx * Ly)
        gEv = gE.view(B, *([1] * (m.dim() - 1))) if m.dim() == 3 else gE.view(())
        gm = (gEv.to(g.dtype) * g)
        gth = (gE.view(B, 1) * dth).sum(0).to(theta.dtype)
        return gm, gth, None, None


def energy(m: torch.Tensor, theta: torch.Tensor, Lx: int, Ly: int) -> torch.Tensor:
    """Energy of each lattice in m ([3][N] or [batch][3][N]); differentiable
    in m and theta to second order."""
    E = _EnergyFn.apply(m, theta, Lx, Ly)
    return E[0] if m.dim() == 2 else E


def theta_of(p) -> torch.Tensor:
    """Parameter vector of a parameter record (J, D padded to the same shell count)."""
    ns = max(len(p.J), len(p.D), 1)
    J = [float(p.J[s]) if s < len(p.J) else 0.0 for s in range(ns)]
    D = [float(p.D[s]) if s < len(p.D) else 0.0 for s in range(ns)]
    return torch.tensor(J + D + [float(p.K)] + [float(b) for b in p.B], dtype=torch.float64, device="cuda")
