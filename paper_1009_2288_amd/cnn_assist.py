"""CNN-assisted EPTV: a learned start for the iteration of Sec. 2.2.

A U-Net (``eptv.UNet``, bf16 MFMA kernels) looks at an early EPTV
reconstruction f^(n0) and proposes what the plain iteration only reaches
later: the image f^(k_t), as a change from f^(n0), and the half-edge weights
of Eq. 5 / A3 at that image.  EPTV then continues from the proposed image
with the proposed weights held fixed for the first iterations (P2 of Eq. 8
with given weights) and adaptive afterwards (Sec. 2.1).  Plain EPTV stays in
charge: the result is always an EPTV iterate started from the proposal, and
if the proposal is poor the adaptive iterations simply carry on as plain EPTV
would from any other start.

Training pairs come from plain EPTV on the GPU (no phantom is needed):
input ``IN_SCALE * f^(n0)`` (one channel); target the weight maps at
``f^(k_t)`` (sigma chosen from f^(k_t) by the edge-quantile rule) and
``RES_SCALE * (f^(k_t) - f^(n0))``.  ``k_t`` = 30 is where plain EPTV's error
to the phantom bottoms out on the thorax phantoms at 20-60 views; its
100-iteration image has drifted back up (a network copying it could never
reach the 100-iteration error before plain EPTV does).

Every step runs in the library's kernels; torch provides memory and streams.
"""
from __future__ import annotations

import math
import os
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import eptv as E
from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
IN_SCALE = 50.0      # attenuation (mm^-1) of the input image to unit order
RES_SCALE = 1000.0   # the image change f^(k_t) - f^(n0) to unit order
N0 = 1               # plain iterations before the network
K_T = 30             # plain iterations behind the targets


def weights_path(n0: int = None, k_t: int = K_T) -> str:
    return os.path.join(HERE, "weights", f"eptv_unet_512_n{N0 if n0 is None else n0}_k{k_t}.npz")


WEIGHTS = weights_path()
NET = dict(c_in=1, c_out=3, base=32, levels=4)
SOLVER = dict(cgls_iters=3, tv_iters=5, lam=1000.0, edge_quantile=0.9, tv_eps=1e-4)


# ----------------------------------------------------------------------------- parameters

def layer_shapes(c_in: int, c_out: int, base: int, levels: int):
    """(name, weight shape) in the library's parameter order: encoder levels
    (two 3x3 each), then per decoder level from the bottom up the 2x2
    transposed convolution and two 3x3, then the 1x1 head.  Weight shapes are
    [kh][kw][C_in][C_out]; each is followed by a bias of C_out."""
    out, c = [], c_in
    for l in range(levels):
        out.append((f"e{l}a", (3, 3, c, base << l)))
        out.append((f"e{l}b", (3, 3, base << l, base << l)))
        c = base << l
    for l in range(levels - 2, -1, -1):
        out.append((f"u{l}", (2, 2, c, base << l)))
        out.append((f"d{l}a", (3, 3, 2 * (base << l), base << l)))
        out.append((f"d{l}b", (3, 3, base << l, base << l)))
        c = base << l
    out.append(("head", (1, 1, c, c_out)))
    return out


def init_params(seed: int = 0, head_bias=(0.9, 0.9, 0.0), **net) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the head starts
    near 'no change, weights ~ head_bias'."""
    net = {**NET, **net}
    rng = np.random.default_rng(seed)
    parts = []
    for name, (kh, kw, ci, co) in layer_shapes(**net):
        fan_in = kh * kw * ci if name[0] != "u" else ci
        std = math.sqrt(2.0 / fan_in) if name != "head" else 1e-3
        parts.append((rng.standard_normal(kh * kw * ci * co) * std).astype(np.float32))
        b = np.zeros(co, np.float32)
        if name == "head":
            b[:len(head_bias)] = head_bias[:co]
        parts.append(b)
    return np.concatenate(parts)


def forward_flops(height: int, width: int, **net) -> float:
    """Algorithmic flops (2 per multiply-add, no padding) of one forward pass
    on a height x width image."""
    net = {**NET, **net}
    tot = 0
    for name, (kh, kw, ci, co) in layer_shapes(**net):
        lev = 0 if name == "head" else int(name[1])
        if name[0] == "u":
            lev += 1  # the transposed convolution runs over its coarser input grid
        px = (height >> lev) * (width >> lev)
        tot += 2 * px * kh * kw * ci * co
    return float(tot)


def bias_mask(**net) -> np.ndarray:
    """True where the flat parameter vector holds a bias."""
    net = {**NET, **net}
    m = []
    for _, (kh, kw, ci, co) in layer_shapes(**net):
        m.append(np.zeros(kh * kw * ci * co, bool))
        m.append(np.ones(co, bool))
    return np.concatenate(m)


def _to_bf16_bits(a: np.ndarray) -> np.ndarray:
    u = a.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16          # round to nearest even
    return r.astype(np.uint16)


def save_params(path: str, flat: np.ndarray, meta: dict, **net) -> None:
    """Weights as bf16 (what the kernels compute with), biases as fp32: the
    forward pass of the loaded network equals the trained one bit for bit."""
    m = bias_mask(**net)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez_compressed(path, weights_bf16=_to_bf16_bits(flat[~m]), biases=flat[m].astype(np.float32),
                        meta=np.array(repr(meta)))


def load_params(path: str = WEIGHTS, **net) -> np.ndarray:
    m = bias_mask(**net)
    with np.load(path, allow_pickle=False) as z:
        w = (z["weights_bf16"].astype(np.uint32) << 16).view(np.float32)
        b = z["biases"]
    if w.size + b.size != m.size:
        raise ValueError(f"{path}: {w.size + b.size} parameters, the network has {m.size}")
    flat = np.empty(m.size, np.float32)
    flat[~m] = w
    flat[m] = b
    return flat


def network(max_batch: int = 1, height: int = 512, width: int = 512, params: Optional[np.ndarray] = None,
            **net) -> E.UNet:
    net = {**NET, **net}
    u = E.UNet(net["c_in"], net["c_out"], net["base"], net["levels"], max_batch, height, width)
    u.set_params(params if params is not None else init_params(**net))
    return u


# ----------------------------------------------------------------------------- training data

def training_cases(n: int, seed: int = 10000, side: int = 512, views=(20, 60), i0=5e4):
    """Thorax phantoms (seeds from 10000, none shared with the evaluation
    seeds 0-9) on the paper-scale fan geometry with 20-60 views."""
    bins = 736 if side == 512 else max(64, side * 736 // 512)
    return synth.batch_cases(n, seed, sizes=(side,), views=views, bins=(bins, bins), i0=(i0, i0),
                             with_phantom=False)


class _Plans:
    def __init__(self):
        self.plans = {}

    def get(self, g) -> E.Plan:
        ang = None if g.view_angles_rad is None else np.asarray(g.view_angles_rad, np.float64).tobytes()
        key = (g.nx, g.ny, g.pixel_mm, g.n_views, g.n_bins, g.dbeta_rad, g.bin_offset, g.sad_mm, g.sdd_mm, ang)
        if key not in self.plans:
            self.plans[key] = E.Plan(g)
        return self.plans[key]


def make_pairs(cases, n0: int = N0, k_t: int = K_T, solver: Optional[dict] = None, log=None):
    """(X [n][ny][nx][1], T [n][ny][nx][3]) on the GPU from plain EPTV runs."""
    solver = {**SOLVER, **(solver or {})}
    g0 = cases[0].geom
    n = len(cases)
    X = torch.empty((n, g0.ny, g0.nx, 1), dtype=torch.float32, device="cuda")
    T = torch.empty((n, g0.ny, g0.nx, 3), dtype=torch.float32, device="cuda")
    plans = _Plans()
    t0 = time.time()
    for i, c in enumerate(cases):
        if (c.geom.nx, c.geom.ny) != (g0.nx, g0.ny):
            raise ValueError("all training cases must share the image size")
        P = plans.get(c.geom)
        y = torch.from_numpy(np.ascontiguousarray(c.y, np.float32)).cuda()
        f, _ = P.reconstruct(y, E.Params(outer_iters=n0, zero_init=1, **solver), stats=False)
        f0 = f.clone()
        E.maps_from_eptv(f0, scale=IN_SCALE, out=X[i:i + 1])
        P.reconstruct(y, E.Params(outer_iters=k_t - n0, zero_init=0, **solver), f=f, stats=False)
        sig = float(P.select_sigma(f, solver["edge_quantile"], solver["tv_eps"]).item())
        _, wx, wy = P.tv_gradient(f, f, solver["lam"], sig, solver["tv_eps"])
        E.maps_from_eptv(f, wx, wy, scale=RES_SCALE, f_base=f0, out=T[i:i + 1])
        if log and (i + 1) % 200 == 0:
            log(f"pairs {i + 1}/{n} ({time.time() - t0:.1f} s)")
    return X, T


# ----------------------------------------------------------------------------- training

@dataclass
class TrainConfig:
    epochs: int = 10
    batch: int = 8
    lr: float = 1e-3
    lr_final: float = 2e-5
    warmup_steps: int = 50
    seed: int = 0
    holdout: int = 96


def train(net: E.UNet, X: torch.Tensor, T: torch.Tensor, cfg: TrainConfig = TrainConfig(), log=print):
    """Adam on the mean squared error over all three channels, contiguous
    mini-batches visited in a shuffled order per epoch, cosine learning rate.
    The last ``cfg.holdout`` pairs are held out for the validation loss.
    Returns the loss history."""
    n = X.shape[0] - cfg.holdout
    nb = n // cfg.batch
    if nb < 1:
        raise ValueError("fewer training pairs than one batch")
    rng = np.random.default_rng(cfg.seed)
    total = cfg.epochs * nb
    step = 0
    hist = []
    acc = torch.zeros(1, dtype=torch.float32, device=X.device)
    t0 = time.time()
    for ep in range(cfg.epochs):
        acc.zero_()
        for b in rng.permutation(nb):
            s0 = int(b) * cfg.batch
            x, t = X[s0:s0 + cfg.batch], T[s0:s0 + cfg.batch]
            y = net.forward(x)
            loss, dy = net.mse(y, t)
            net.backward(dy)
            step += 1
            if step <= cfg.warmup_steps:
                lr = cfg.lr * step / cfg.warmup_steps
            else:
                q = (step - cfg.warmup_steps) / max(total - cfg.warmup_steps, 1)
                lr = cfg.lr_final + 0.5 * (cfg.lr - cfg.lr_final) * (1 + math.cos(math.pi * q))
            net.adam(lr, step)
            acc += loss
        train_loss = float(acc.item()) / nb
        val = validate(net, X[n:], T[n:], cfg.batch) if cfg.holdout else float("nan")
        hist.append({"epoch": ep + 1, "train_mse": train_loss, "val_mse": val, "seconds": time.time() - t0})
        log(f"epoch {ep + 1}/{cfg.epochs}: train mse {train_loss:.5f}, held-out mse {val:.5f}, "
            f"{time.time() - t0:.1f} s")
    return hist


def validate(net: E.UNet, X: torch.Tensor, T: torch.Tensor, batch: int) -> float:
    tot, cnt = 0.0, 0
    for s0 in range(0, X.shape[0] - batch + 1, batch):
        y = net.forward(X[s0:s0 + batch])
        loss, _ = net.mse(y, T[s0:s0 + batch], want_grad=False)
        tot += float(loss.item())
        cnt += 1
    return tot / max(cnt, 1)


# ----------------------------------------------------------------------------- inference

def propose(net: E.UNet, f0: torch.Tensor, stream=None):
    """(image, wx, wy) proposed from the early reconstruction f0 [ny][nx]."""
    x = E.maps_from_eptv(f0, scale=IN_SCALE, stream=stream)
    m = net.forward(x, stream=stream)
    f, wx, wy = E.maps_to_eptv(m, scale=RES_SCALE, f_base=f0, stream=stream)
    return f[0], wx[0], wy[0]


def assisted_reconstruct(P: E.Plan, net: E.UNet, y: torch.Tensor, outer_iters: int, frozen_iters: int = 1,
                         n0: int = N0, f_ref: Optional[torch.Tensor] = None, stats: bool = True,
                         solver: Optional[dict] = None, stream=None):
    """n0 plain EPTV iterations, the network's proposal, then ``outer_iters``
    EPTV iterations warm-started from the proposed image, the proposed
    weights frozen for the first ``frozen_iters``.  Returns (f, stats of the
    warm-started iterations or None)."""
    solver = {**SOLVER, **(solver or {})}
    f0, _ = P.reconstruct(y, E.Params(outer_iters=n0, zero_init=1, **solver), stats=False, stream=stream)
    f, wx, wy = propose(net, f0, stream=stream)
    return P.reconstruct(y, E.Params(outer_iters=outer_iters, zero_init=0, **solver), f=f, f_ref=f_ref,
                         stats=stats, weights=(wx, wy), frozen_iters=frozen_iters, stream=stream)


def time_to_rmse(P: E.Plan, y: torch.Tensor, ref: torch.Tensor, target: float, net: Optional[E.UNet] = None,
                 frozen_iters: int = 1, max_iters: int = 100, reps: int = 5, n0: int = N0,
                 solver: Optional[dict] = None):
    """Seconds (median of ``reps`` runs, HIP events on the current stream)
    until the RMSE to ``ref`` is <= target: plain EPTV from zero, or (with
    ``net``) the assisted pipeline.  The runs stop themselves (``stop_rmse``,
    the RMSE record read back after every iteration), so the time includes
    each iteration's check.  ``solver`` overrides entries of SOLVER (e.g.
    ``stored_matrix=1`` once the plan holds the matrix)."""
    import numpy as np
    solver = {**SOLVER, **(solver or {})}
    s = torch.cuda.current_stream()
    secs, st = [], None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        if net is None:
            _, st = P.reconstruct(y, E.Params(outer_iters=max_iters, zero_init=1, stop_rmse=target, **solver),
                                  f_ref=ref)
        else:
            _, st = assisted_reconstruct(P, net, y, max_iters, frozen_iters, n0=n0, f_ref=ref,
                                         solver={**solver, "stop_rmse": target})
        e1.record(s)
        torch.cuda.synchronize()
        secs.append(e0.elapsed_time(e1) / 1e3)
    k = st["iters_run"]
    if st["rmse"][k - 1] > target:
        return {"iterations": None, "seconds": None, "rmse_min": float(st["rmse"].min())}
    return {"iterations": k, "seconds": float(np.median(secs)), "rmse": float(st["rmse"][k - 1]),
            "seconds_runs": [float(v) for v in secs]}
