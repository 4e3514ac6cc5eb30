"""Differentiable EPTV operators for torch.autograd, on top of the HIP kernels.

P (Sec. 2.1, Eq. 1: exact ray/pixel intersection lengths) and P^T (Sec. 2.2)
are linear, so each one's backward is the other.  With a ``Plan`` they act on
one slice (leading dimensions looped over); with a ``Batch`` on a stack
[S, ny, nx] of its S slices, each operator one launch over all slices
(``eptv_batch_project`` / ``eptv_batch_backproject``).  The P2 descent
direction g = lambda (f - v) + (A2 variation of the EPTV term) (Eq. 9, App. II)
gets its backward from the hand-written vector-Jacobian product kernel
(``Plan.tv_gradient_vjp``).

Unrolled EPTV iterations (the algorithm of Sec. 2.2) compose these with the
CGLS scalars (App. I) and the descent updates written as torch element-wise
arithmetic: sums and scaled sums of a few images per step, whose derivatives
autograd forms exactly (the scalars a_m = gamma_m / delta_m and b_m are
differentiated through their inner products).  The operators and the A2
direction, where the arithmetic of the method lives, are the library's
kernels in both passes.  sigma and the Armijo step sizes are decided by the
forward pass (with the library's own selection and line-search kernels) and
held constant, so the gradient is that of the iteration map for the recorded
schedule.  Nothing here falls back to another implementation.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Union

import torch
import torch.utils.checkpoint as tcp

from .eptv import Batch, Params, Plan

Op = Union[Plan, Batch]


def _map_images(fn, x: torch.Tensor, out_shape) -> torch.Tensor:
    """Apply a single-slice operator over the leading dimensions of x."""
    lead = x.shape[:-2]
    xs = x.reshape(-1, *x.shape[-2:])
    out = torch.empty((xs.shape[0], *out_shape), dtype=x.dtype, device=x.device)
    for b in range(xs.shape[0]):
        fn(xs[b].contiguous(), out[b])
    return out.reshape(*lead, *out_shape)


def _first(op: Op) -> Plan:
    return op.plans[0] if isinstance(op, Batch) else op


def _apply_p(op: Op, x: torch.Tensor) -> torch.Tensor:
    if isinstance(op, Batch):
        return op.project(x.contiguous())
    return _map_images(lambda a, o: op.project(a, o), x, (op.n_views, op.n_bins))


def _apply_pt(op: Op, r: torch.Tensor) -> torch.Tensor:
    if isinstance(op, Batch):
        return op.backproject(r.contiguous())
    return _map_images(lambda a, o: op.backproject(a, o), r, (op.ny, op.nx))


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, op: Op) -> torch.Tensor:
        ctx.op = op
        return _apply_p(op, x)

    @staticmethod
    def backward(ctx, gq: torch.Tensor):
        return _apply_pt(ctx.op, gq.contiguous()), None


class _Backproject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r: torch.Tensor, op: Op) -> torch.Tensor:
        ctx.op = op
        return _apply_pt(op, r)

    @staticmethod
    def backward(ctx, gz: torch.Tensor):
        return _apply_p(ctx.op, gz.contiguous()), None


def _check_batch(op: Op, t: torch.Tensor, last2) -> None:
    if isinstance(op, Batch):
        p = op.plans[0]
        if any((q.ny, q.nx, q.n_views, q.n_bins) != (p.ny, p.nx, p.n_views, p.n_bins) for q in op.plans):
            raise ValueError("stacked batch operators need slices of one shape")
        if tuple(t.shape) != (len(op), *last2):
            raise ValueError(f"expected a [{len(op)}, {last2[0]}, {last2[1]}] stack, got {tuple(t.shape)}")


def project(op: Op, x: torch.Tensor) -> torch.Tensor:
    """P x, differentiable: x [..., ny, nx] for a Plan, [S, ny, nx] for a Batch of S slices."""
    _check_batch(op, x, (_first(op).ny, _first(op).nx))
    return _Project.apply(x, op)


def backproject(op: Op, r: torch.Tensor) -> torch.Tensor:
    """P^T r, differentiable: r [..., n_views, n_bins] for a Plan, [S, n_views, n_bins] for a Batch."""
    _check_batch(op, r, (_first(op).n_views, _first(op).n_bins))
    return _Backproject.apply(r, op)


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
    backtrack index per descent step (-1: no step accepted); for a Batch, per
    iteration one entry per slice."""

    sigma: list = field(default_factory=list)
    armijo_k: list = field(default_factory=list)


def _dot(a: torch.Tensor, b: torch.Tensor, stacked: bool) -> torch.Tensor:
    """<a, b> in float64: per slice ([S, 1, 1]) for a stack, else a scalar."""
    p = a.double() * b.double()
    return p.sum(dim=(-2, -1), keepdim=True) if stacked else p.sum()


def eptv_iteration(op: Op, f: torch.Tensor, y: torch.Tensor, params: Params, schedule: Schedule, k: int):
    """One outer EPTV iteration, differentiable in f and y (for a Batch, f
    [S, ny, nx] and y [S, n_views, n_bins]).  Uses schedule entry k when it
    exists (recomputation, or a replay) and records it otherwise."""
    M, T = params.cgls_iters, params.tv_iters
    stacked = isinstance(op, Batch)
    plans = op.plans if stacked else [op]
    # Step 1: P1 by CGLS from f (App. I), or the gradient form of Eq. 8
    if M > 0:
        u = f
        r = y - project(op, u)
        s = backproject(op, r)
        gam = _dot(s, s, stacked)
        for m in range(M):
            q = project(op, s)
            a = (gam / _dot(q, q, stacked)).to(s.dtype)
            u = u + a * s
            r = r - a * q
            if m == M - 1:
                break
            z = backproject(op, r)
            gnew = _dot(z, z, stacked)
            s = z + (gnew / gam).to(z.dtype) * s
            gam = gnew
        v = u
    else:
        v = f - (params.mu / params.lam) * backproject(op, project(op, f) - y)
    # Step 2: P2 by T descent steps from v (or f), sigma and steps from the schedule
    h = f if params.p2_start else v
    hs = [h] if not stacked else list(h.unbind(0))
    vs = [v] if not stacked else list(v.unbind(0))
    if k >= len(schedule.sigma):
        sig, kss = [], []
        with torch.no_grad():
            for p, hh, vv in zip(plans, hs, vs):
                hd = hh.detach().contiguous()
                if params.sigma_fixed >= 0:
                    sg = float(params.sigma_fixed)
                else:
                    sg = float(p.select_sigma(hd, params.edge_quantile, params.tv_eps, params.sigma_floor).item())
                ks, _ = p.tv_step(hd.clone(), vv.detach().contiguous(), params, T, sg) if T > 0 else ([], sg)
                sig.append(sg)
                kss.append([int(x) for x in ks])
        schedule.sigma.append(sig if stacked else sig[0])
        schedule.armijo_k.append(kss if stacked else kss[0])
    sig = schedule.sigma[k] if stacked else [schedule.sigma[k]]
    kss = schedule.armijo_k[k] if stacked else [schedule.armijo_k[k]]
    t0 = params.armijo_t0 if params.armijo_t0 > 0 else 1.0 / params.lam
    out = []
    for p, hh, vv, sg, ks in zip(plans, hs, vs, sig, kss):
        for kk in ks:
            if kk >= 0:
                hh = hh - (t0 * params.armijo_shrink ** kk) * tv_direction(p, hh, vv, params.lam, sg, params.tv_eps)
        out.append(hh)
    h = torch.stack(out) if stacked else out[0]
    # Step 3: positivity
    return torch.relu(h) if params.positivity else h


def unrolled(op: Op, f0: torch.Tensor, y: torch.Tensor, params: Params, n_iters: int,
             checkpoint: bool = True, schedule: Optional[Schedule] = None):
    """n_iters EPTV iterations from f0, differentiable in f0 and y (one slice
    with a Plan, a stack of slices with a Batch).  With checkpoint, each
    iteration's intermediates are recomputed in the backward pass instead of
    being kept (the recomputation replays the recorded schedule).  Returns
    (f, schedule)."""
    sched = schedule if schedule is not None else Schedule()
    f = f0
    for k in range(n_iters):
        if checkpoint and torch.is_grad_enabled():
            f = tcp.checkpoint(lambda a, b, kk=k: eptv_iteration(op, a, b, params, sched, kk), f, y,
                               use_reentrant=False)
        else:
            f = eptv_iteration(op, f, y, params, sched, k)
    return f, sched
