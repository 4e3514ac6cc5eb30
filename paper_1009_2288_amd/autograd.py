"""Differentiable EPTV operators for torch.autograd, on top of the HIP kernels.

P (Sec. 2.1, Eq. 1: exact ray/pixel intersection lengths) and P^T (Sec. 2.2)
are linear, so each one's backward is the other.  The P2 descent direction
g = lambda (f - v) + (A2 variation of the EPTV term) (Eq. 9, App. II) gets
its backward from the hand-written vector-Jacobian product kernel
(``Plan.tv_gradient_vjp``).  Unrolled EPTV iterations (the algorithm of
Sec. 2.2) compose these with torch arithmetic on the CGLS scalars (App. I)
and the descent updates; sigma and the Armijo step sizes are decided by the
forward pass (with the library's own selection and line-search kernels) and
held constant, so the gradient is that of the iteration map for the recorded
schedule.  Every operator call goes through the C ABI; nothing here falls
back to another implementation.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import torch
import torch.utils.checkpoint as tcp

from .eptv import Params, Plan


def _map_images(fn, x: torch.Tensor, out_shape) -> torch.Tensor:
    """Apply a single-slice operator over the leading dimensions of x."""
    lead = x.shape[:-2]
    xs = x.reshape(-1, *x.shape[-2:])
    out = torch.empty((xs.shape[0], *out_shape), dtype=x.dtype, device=x.device)
    for b in range(xs.shape[0]):
        fn(xs[b].contiguous(), out[b])
    return out.reshape(*lead, *out_shape)


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return _map_images(lambda a, o: plan.project(a, o), x, (plan.n_views, plan.n_bins))

    @staticmethod
    def backward(ctx, gq: torch.Tensor):
        plan = ctx.plan
        return _map_images(lambda a, o: plan.backproject(a, o), gq.contiguous(), (plan.ny, plan.nx)), None


class _Backproject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return _map_images(lambda a, o: plan.backproject(a, o), r, (plan.ny, plan.nx))

    @staticmethod
    def backward(ctx, gz: torch.Tensor):
        plan = ctx.plan
        return _map_images(lambda a, o: plan.project(a, o), gz.contiguous(), (plan.n_views, plan.n_bins)), None


def project(plan: Plan, x: torch.Tensor) -> torch.Tensor:
    """P x for x [..., ny, nx] (float32, on the plan's device); differentiable."""
    return _Project.apply(x, plan)


def backproject(plan: Plan, r: torch.Tensor) -> torch.Tensor:
    """P^T r for r [..., n_views, n_bins]; differentiable."""
    return _Backproject.apply(r, plan)


class _TVDirection(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f: torch.Tensor, v: torch.Tensor, plan: Plan, lam: float, sigma: float, eps: float):
        ctx.plan, ctx.lam, ctx.sigma, ctx.eps = plan, lam, sigma, eps
        ctx.save_for_backward(f)
        g, _, _ = plan.tv_gradient(f.contiguous(), v.contiguous(), lam, sigma, eps, with_weights=False)
        return g

    @staticmethod
    def backward(ctx, gg: torch.Tensor):
        (f,) = ctx.saved_tensors
        gg = gg.contiguous()
        df = ctx.plan.tv_gradient_vjp(f.contiguous(), gg, ctx.lam, ctx.sigma, ctx.eps)
        return df, -ctx.lam * gg, None, None, None, None


def tv_direction(plan: Plan, f: torch.Tensor, v: torch.Tensor, lam: float, sigma: float, eps: float):
    """The P2 direction g(f; v) of Eq. 9 (one slice), differentiable in f and v
    with sigma held constant."""
    return _TVDirection.apply(f, v, plan, lam, sigma, eps)


@dataclass
class Schedule:
    """Decisions of the forward pass: sigma per outer iteration and the Armijo
    backtrack index per descent step (-1: no step accepted)."""

    sigma: list = field(default_factory=list)
    armijo_k: list = field(default_factory=list)


def _dot(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    return (a.double() * b.double()).sum()


def eptv_iteration(plan: Plan, f: torch.Tensor, y: torch.Tensor, params: Params, schedule: Schedule, k: int):
    """One outer EPTV iteration, differentiable in f and y.  Uses schedule entry
    k when it exists (recomputation, or a replay) and records it otherwise."""
    M, T = params.cgls_iters, params.tv_iters
    # Step 1: P1 by CGLS from f (App. I), or the gradient form of Eq. 8
    if M > 0:
        u = f
        r = y - project(plan, u)
        s = backproject(plan, r)
        gam = _dot(s, s)
        for m in range(M):
            q = project(plan, s)
            a = (gam / _dot(q, q)).to(s.dtype)
            u = u + a * s
            r = r - a * q
            if m == M - 1:
                break
            z = backproject(plan, r)
            gnew = _dot(z, z)
            s = z + (gnew / gam).to(z.dtype) * s
            gam = gnew
        v = u
    else:
        v = f - (params.mu / params.lam) * backproject(plan, project(plan, f) - y)
    # Step 2: P2 by T descent steps from v (or f), sigma and steps from the schedule
    h = f if params.p2_start else v
    if k >= len(schedule.sigma):
        with torch.no_grad():
            hd = h.detach().contiguous()
            if params.sigma_fixed >= 0:
                sigma = float(params.sigma_fixed)
            else:
                sigma = float(plan.select_sigma(hd, params.edge_quantile, params.tv_eps, params.sigma_floor).item())
            ks, _ = plan.tv_step(hd.clone(), v.detach().contiguous(), params, T, sigma) if T > 0 else ([], sigma)
        schedule.sigma.append(sigma)
        schedule.armijo_k.append([int(x) for x in ks])
    sigma, ks = schedule.sigma[k], schedule.armijo_k[k]
    t0 = params.armijo_t0 if params.armijo_t0 > 0 else 1.0 / params.lam
    for kk in ks:
        if kk >= 0:
            h = h - (t0 * params.armijo_shrink ** kk) * tv_direction(plan, h, v, params.lam, sigma, params.tv_eps)
    # Step 3: positivity
    return torch.relu(h) if params.positivity else h


def unrolled(plan: Plan, f0: torch.Tensor, y: torch.Tensor, params: Params, n_iters: int,
             checkpoint: bool = True, schedule: Optional[Schedule] = None):
    """n_iters EPTV iterations from f0, differentiable in f0 and y.  With
    checkpoint, each iteration's intermediates are recomputed in the backward
    pass instead of being kept (the recomputation replays the recorded
    schedule).  Returns (f, schedule)."""
    sched = schedule if schedule is not None else Schedule()
    f = f0
    for k in range(n_iters):
        if checkpoint and torch.is_grad_enabled():
            f = tcp.checkpoint(lambda a, b, kk=k: eptv_iteration(plan, a, b, params, sched, kk), f, y,
                               use_reentrant=False)
        else:
            f = eptv_iteration(plan, f, y, params, sched, k)
    return f, sched
