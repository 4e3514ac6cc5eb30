"""FP64 CPU oracle of the U-Net that proposes EPTV edge weights and a warm start.

TEST INFRASTRUCTURE.  Plain numpy in float64, written for clarity, not speed:
the reference the network's HIP kernels (forward and backward) are checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may use it; the product path never does, and it shares no code with
the HIP library.

The network is not part of the paper (which has no learned component); it
maps an early EPTV reconstruction to the half-edge weight maps of Eq. 5 / A3
and to an image, for warm-starting the EPTV iteration of Sec. 2.2.

Precision: float64 arithmetic.  The network is specified with bf16 weights
and activations and fp32 accumulation; ``bf16`` rounds to that format, and
the forward / backward passes take an optional ``store`` function applied
wherever such an implementation stores a tensor (each layer's output, the
pooled and the upsampled features, each layer's input gradient, the skip
gradient after the pooling path joins it), so the reference can follow the
specified storage precision while computing every sum exactly.

Layout: activations [N][H][W][C] (channels last); 3x3 convolution weights
[3][3][C_in][C_out] (cross-correlation, zero padding 1, stride 1); 2x2
transposed-convolution weights [2][2][C_in][C_out] (stride 2); 1x1 weights
[C_in][C_out]; biases [C_out].
"""
from __future__ import annotations

import numpy as np


def bf16(a):
    """Round to the nearest bfloat16 (8-bit significand), ties to even; float64 out."""
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _same(a):
    return a


# ------------------------------------------------------------------ layers
def conv3x3(x, w, b):
    """y[n,i,j,o] = b[o] + sum_{a,c,k} x[n, i+a-1, j+c-1, k] w[a,c,k,o] (x = 0 outside)."""
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((N, H, W, w.shape[3]))
    for a in range(3):
        for c in range(3):
            y += xp[:, a:a + H, c:c + W, :] @ w[a, c]
    return y + b


def conv3x3_backward(x, w, dy):
    """Gradients (dx, dw, db) of sum(dy * conv3x3(x, w, b))."""
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for a in range(3):
        for c in range(3):
            dxp[:, a:a + H, c:c + W, :] += dy @ w[a, c].T
            dw[a, c] = np.einsum("nhwk,nhwo->ko", xp[:, a:a + H, c:c + W, :], dy)
    return dxp[:, 1:-1, 1:-1, :], dw, dy.sum(axis=(0, 1, 2))


def conv1x1(x, w, b):
    return x @ w + b


def conv1x1_backward(x, w, dy):
    return dy @ w.T, np.einsum("nhwk,nhwo->ko", x, dy), dy.sum(axis=(0, 1, 2))


def tconv2x2(x, w, b):
    """Stride-2 transposed convolution: y[n, 2i+a, 2j+c, o] = b[o] + x[n,i,j,:] . w[a,c,:,o]."""
    N, H, W, _ = x.shape
    y = np.zeros((N, 2 * H, 2 * W, w.shape[3]))
    for a in range(2):
        for c in range(2):
            y[:, a::2, c::2, :] = x @ w[a, c]
    return y + b


def tconv2x2_backward(x, w, dy):
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for a in range(2):
        for c in range(2):
            d = dy[:, a::2, c::2, :]
            dx += d @ w[a, c].T
            dw[a, c] = np.einsum("nhwk,nhwo->ko", x, d)
    return dx, dw, dy.sum(axis=(0, 1, 2))


def avgpool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_backward(dy):
    return 0.25 * np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2)


def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(y, dy):
    """dy masked where the ReLU output y is zero."""
    return np.where(y > 0.0, dy, 0.0)


# ------------------------------------------------------------------ the U-Net
def unet_shapes(c_in: int = 1, c_out: int = 3, base: int = 32, levels: int = 4) -> dict:
    """Parameter shapes: per encoder level two 3x3 convs; average-pool down;
    stride-2 transposed conv up; skip by channel concatenation; two 3x3 convs
    per decoder level; a 1x1 head."""
    s = {}
    c = c_in
    for l in range(levels):
        ch = base << l
        s[f"e{l}a"] = ((3, 3, c, ch), (ch,))
        s[f"e{l}b"] = ((3, 3, ch, ch), (ch,))
        c = ch
    for l in range(levels - 2, -1, -1):
        ch = base << l
        s[f"u{l}"] = ((2, 2, c, ch), (ch,))
        s[f"d{l}a"] = ((3, 3, 2 * ch, ch), (ch,))
        s[f"d{l}b"] = ((3, 3, ch, ch), (ch,))
        c = ch
    s["head"] = ((c, c_out), (c_out,))
    return s


def unet_init(shapes: dict, seed: int) -> dict:
    """He-normal weights, zero biases (PCG64 with the given seed)."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, (ws, bs) in shapes.items():
        fan_in = int(np.prod(ws[:-1]))
        p[k + ".w"] = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=ws)
        p[k + ".b"] = np.zeros(bs)
    return p


def _levels(p: dict) -> int:
    return sum(1 for k in p if k.startswith("e") and k.endswith("a.w"))


def unet_forward(p: dict, x, store=_same):
    """Returns (output, cache).  Every conv but the head is followed by a ReLU."""
    L = _levels(p)
    x = store(x)
    cache = {"x": x}
    h = x
    skips = []
    for l in range(L):
        if l > 0:
            h = store(avgpool2(h))
        cache[f"e{l}a.in"] = h
        h = store(relu(conv3x3(h, p[f"e{l}a.w"], p[f"e{l}a.b"])))
        cache[f"e{l}a.out"] = h
        h = store(relu(conv3x3(h, p[f"e{l}b.w"], p[f"e{l}b.b"])))
        cache[f"e{l}b.in"] = cache[f"e{l}a.out"]
        cache[f"e{l}b.out"] = h
        skips.append(h)
    for l in range(L - 2, -1, -1):
        cache[f"u{l}.in"] = h
        h = store(relu(tconv2x2(h, p[f"u{l}.w"], p[f"u{l}.b"])))
        cache[f"u{l}.out"] = h
        h = np.concatenate([skips[l], h], axis=3)
        cache[f"d{l}a.in"] = h
        h = store(relu(conv3x3(h, p[f"d{l}a.w"], p[f"d{l}a.b"])))
        cache[f"d{l}a.out"] = h
        cache[f"d{l}b.in"] = h
        h = store(relu(conv3x3(h, p[f"d{l}b.w"], p[f"d{l}b.b"])))
        cache[f"d{l}b.out"] = h
    cache["head.in"] = h
    return conv1x1(h, p["head.w"], p["head.b"]), cache


def unet_backward(p: dict, cache: dict, dout, store=_same) -> dict:
    """Gradients of sum(dout * output) with respect to every parameter (and "x")."""
    L = _levels(p)
    g = {}
    dout = store(dout)
    dh, g["head.w"], g["head.b"] = conv1x1_backward(cache["head.in"], p["head.w"], dout)
    dh = store(dh)
    dskip = [None] * L
    for l in range(0, L - 1):
        dh = relu_backward(cache[f"d{l}b.out"], dh)
        dh, g[f"d{l}b.w"], g[f"d{l}b.b"] = conv3x3_backward(cache[f"d{l}b.in"], p[f"d{l}b.w"], dh)
        dh = relu_backward(cache[f"d{l}a.out"], store(dh))
        dh, g[f"d{l}a.w"], g[f"d{l}a.b"] = conv3x3_backward(cache[f"d{l}a.in"], p[f"d{l}a.w"], dh)
        dh = store(dh)
        cs = cache[f"e{l}b.out"].shape[3]
        dskip[l], dh = dh[..., :cs], dh[..., cs:]
        dh = relu_backward(cache[f"u{l}.out"], dh)
        dh, g[f"u{l}.w"], g[f"u{l}.b"] = tconv2x2_backward(cache[f"u{l}.in"], p[f"u{l}.w"], dh)
        dh = store(dh)
    for l in range(L - 1, -1, -1):
        if dskip[l] is not None:
            dh = store(dh + dskip[l])
        dh = relu_backward(cache[f"e{l}b.out"], dh)
        dh, g[f"e{l}b.w"], g[f"e{l}b.b"] = conv3x3_backward(cache[f"e{l}b.in"], p[f"e{l}b.w"], dh)
        dh = relu_backward(cache[f"e{l}a.out"], store(dh))
        dh, g[f"e{l}a.w"], g[f"e{l}a.b"] = conv3x3_backward(cache[f"e{l}a.in"], p[f"e{l}a.w"], dh)
        dh = store(dh)
        if l > 0:
            dh = avgpool2_backward(dh)
    g["x"] = dh
    return g


def mse(y, t):
    """Loss mean((y - t)^2) and its gradient with respect to y."""
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(p: dict, g: dict, m: dict, v: dict, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8) -> None:
    """Adam (Kingma & Ba, Algorithm 1), in place; step counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
