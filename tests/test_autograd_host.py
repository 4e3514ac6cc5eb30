"""The autograd composition of the differentiable EPTV iteration, checked on
the CPU in float64: the operators are supplied by an object that calls the
FP64 oracle (P, P^T, the P2 direction and its VJP, sigma, the Armijo steps),
so the gradients of the composed iteration can be compared with central
differences free of float32 rounding.  The GPU tests run the same composition
on the HIP kernels."""
import numpy as np
import pytest
import torch

from paper_1009_2288_amd import autograd as A
from paper_1009_2288_amd import eptv as E
from paper_1009_2288_amd import synth


class OraclePlan:
    """The operator calls the autograd module makes, answered by the oracle."""

    def __init__(self, oracle, g):
        self.O, self.M = oracle, oracle.Matrix(g)
        self.nx, self.ny, self.n_views, self.n_bins = g.nx, g.ny, g.n_views, g.n_bins

    def project(self, x, out):
        out.copy_(torch.from_numpy(self.M.project(x.detach().numpy())))
        return out

    def backproject(self, r, out):
        out.copy_(torch.from_numpy(self.M.backproject(r.detach().numpy())))
        return out

    def tv_gradient(self, f, v, lam, sigma, eps, with_weights=True):
        g, _, _ = self.O.tv_gradient(f.detach().numpy(), v.detach().numpy(), lam, sigma, eps)
        return torch.from_numpy(g), None, None

    def tv_gradient_vjp(self, f, u, lam, sigma, eps):
        return torch.from_numpy(self.O.tv_gradient_vjp(f.detach().numpy(), u.detach().numpy(), lam, sigma, eps))

    def select_sigma(self, f, q, eps, floor):
        return torch.tensor([self.O.select_sigma(f.numpy(), eps, q, floor)])

    def tv_step(self, f, v, params, n, sigma):
        op = self.O.Params(**{k: getattr(params, k) for k in (
            "cgls_iters", "tv_iters", "mu", "lam", "edge_quantile", "sigma_fixed", "sigma_floor", "tv_eps",
            "armijo_c", "armijo_shrink", "armijo_t0", "armijo_max_backtracks", "p2_start", "positivity")})
        _, ks, _, s = self.O.tv_step(f.numpy(), v.numpy(), op, n, sigma)
        return ks, s


def geom():
    return synth.Geometry(24, 20, 1.0, 12, 48, synth.fan_dbeta(24, 20, 1.0, 80.0, 48), 80.0, 160.0)


@pytest.mark.parametrize("kw", [dict(), dict(cgls_iters=0, mu=1.0, lam=400.0, p2_start=1), dict(tv_iters=0),
                                dict(sigma_fixed=float("inf"))])
def test_unrolled_gradient_matches_central_differences(oracle, kw):
    g = geom()
    P = OraclePlan(oracle, g)
    rng = np.random.default_rng(3)
    ell = [synth.Ellipse(0.0, 0.0, 9.0, 7.0, 0.2, 0.02), synth.Ellipse(3.0, -2.0, 3.0, 2.0, 0.0, 0.01)]
    ref = torch.from_numpy(synth.raster(ell, g.nx, g.ny, g.pixel_mm))
    y0 = torch.from_numpy(synth.line_integrals(ell, g) + 1e-3 * rng.normal(size=(g.n_views, g.n_bins)))
    prm = E.Params(**{"cgls_iters": 3, "tv_iters": 3, "lam": 1000.0, "tv_eps": 1e-3, "positivity": 0, **kw})
    f0 = torch.zeros_like(ref)

    def loss(y, sched, checkpoint=False):
        f, s = A.unrolled(P, f0, y, prm, 4, checkpoint=checkpoint, schedule=sched)
        return 0.5 * ((f - ref) ** 2).sum(), s

    y = y0.clone().requires_grad_(True)
    L, sched = loss(y, None, checkpoint=True)
    (gy,) = torch.autograd.grad(L, y)
    eps = 1e-6
    for k in range(3):
        d = torch.from_numpy(np.random.default_rng(10 + k).normal(size=y0.shape))
        with torch.no_grad():
            fd = (float(loss(y0 + eps * d, sched)[0]) - float(loss(y0 - eps * d, sched)[0])) / (2 * eps)
        an = float((gy * d).sum())
        assert abs(fd - an) <= 1e-5 * abs(an) + 1e-12, (k, fd, an)
