"""Pins of the FP64 U-Net oracle: library routines (scipy's 2-D correlation),
brute-force loops, central finite differences and closed forms.  CPU only."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn_oracle as C


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 7, 9, 3))
    w = rng.normal(size=(3, 3, 3, 4))
    b = rng.normal(size=4)
    y = C.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, :, :, k], w[:, :, k, o], mode="same") for k in range(3))
            np.testing.assert_allclose(y[n, :, :, o], ref, rtol=1e-12, atol=1e-12)


def _fd_check(fn, args, grads, names, h=1e-6, picks=12, seed=0):
    """Central differences of sum(dy * fn(*args)) along single entries."""
    rng = np.random.default_rng(seed)
    for name, g in zip(names, grads):
        arr = args[name]
        for _ in range(picks):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            old = arr[idx]
            arr[idx] = old + h
            fp = fn()
            arr[idx] = old - h
            fm = fn()
            arr[idx] = old
            fd = (fp - fm) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[idx])


def test_conv3x3_backward_finite_differences():
    rng = np.random.default_rng(2)
    a = {"x": rng.normal(size=(2, 5, 6, 3)), "w": rng.normal(size=(3, 3, 3, 4)), "b": rng.normal(size=4)}
    dy = rng.normal(size=(2, 5, 6, 4))
    dx, dw, db = C.conv3x3_backward(a["x"], a["w"], dy)
    _fd_check(lambda: float(np.sum(dy * C.conv3x3(a["x"], a["w"], a["b"]))), a, [dx, dw, db], ["x", "w", "b"])


def test_tconv2x2_bruteforce_and_backward():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(1, 3, 4, 2))
    w = rng.normal(size=(2, 2, 2, 3))
    b = rng.normal(size=3)
    y = C.tconv2x2(x, w, b)
    ref = np.zeros((1, 6, 8, 3))
    for i in range(3):
        for j in range(4):
            for a in range(2):
                for c in range(2):
                    for o in range(3):
                        ref[0, 2 * i + a, 2 * j + c, o] = b[o] + sum(x[0, i, j, k] * w[a, c, k, o] for k in range(2))
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)
    dy = rng.normal(size=y.shape)
    args = {"x": x, "w": w, "b": b}
    dx, dw, db = C.tconv2x2_backward(x, w, dy)
    _fd_check(lambda: float(np.sum(dy * C.tconv2x2(args["x"], args["w"], args["b"]))), args, [dx, dw, db],
              ["x", "w", "b"])


def test_avgpool_and_its_adjoint():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(2, 6, 4, 3))
    y = C.avgpool2(x)
    assert y.shape == (2, 3, 2, 3)
    assert np.isclose(y[1, 2, 1, 2], x[1, 4:6, 2:4, 2].mean())
    d = rng.normal(size=y.shape)
    assert np.isclose(np.vdot(y, d), np.vdot(x, C.avgpool2_backward(d)))


def test_unet_parameter_count_at_the_configured_size():
    """4 levels, 32 base channels, 1 input and 3 output channels: about 2 M."""
    s = C.unet_shapes(1, 3, 32, 4)
    n = sum(int(np.prod(w)) + int(np.prod(b)) for w, b in s.values())
    assert 1.8e6 < n < 2.2e6, n


def test_unet_backward_finite_differences():
    rng = np.random.default_rng(5)
    p = C.unet_init(C.unet_shapes(2, 3, 3, 3), seed=6)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(scale=0.1, size=p[k].shape)
    x = rng.normal(size=(2, 8, 8, 2))
    dout = rng.normal(size=(2, 8, 8, 3))
    y, cache = C.unet_forward(p, x)
    assert y.shape == (2, 8, 8, 3)
    g = C.unet_backward(p, cache, dout)
    args = dict(p)
    args["x"] = x

    def f():
        pp = {k: v for k, v in args.items() if k != "x"}
        return float(np.sum(dout * C.unet_forward(pp, args["x"])[0]))

    names = sorted(p) + ["x"]
    _fd_check(f, args, [g[k] for k in names], names, picks=3, seed=7)


def test_adam_first_step_is_a_signed_step_of_lr():
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.5, -4.0, 1e-3])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    C.adam_step(p, g, m, v, step=1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(p["a"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], rtol=1e-9)


def test_mse_gradient_finite_differences():
    rng = np.random.default_rng(8)
    y, t = rng.normal(size=(2, 3, 4, 3)), rng.normal(size=(2, 3, 4, 3))
    loss, g = C.mse(y, t)
    assert np.isclose(loss, np.mean((y - t) ** 2))
    a = {"y": y}
    _fd_check(lambda: C.mse(a["y"], t)[0], a, [g], ["y"])


def test_bf16_rounding_known_values():
    """bfloat16 keeps 8 significand bits: 1 + 2^-8 is a tie (to even: 1),
    1 + 3 * 2^-8 rounds up to 1 + 2^-6, and exactly representable values stay."""
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.0 * 2.0 ** -130, 1.0 + 2.0 ** -7])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, -2.5, 3.0 * 2.0 ** -130, 1.0 + 2.0 ** -7])
    np.testing.assert_array_equal(C.bf16(vals), want)


def test_unet_store_identity_is_the_exact_network():
    """With the default store the passes are the exact ones pinned above; with
    bf16 storage they stay within bf16 resolution on the forward output."""
    rng = np.random.default_rng(9)
    p = C.unet_init(C.unet_shapes(1, 2, 4, 2), seed=10)
    x = rng.normal(size=(1, 8, 8, 1))
    y, _ = C.unet_forward(p, x)
    y2, _ = C.unet_forward(p, x, store=lambda a: a)
    np.testing.assert_array_equal(y, y2)
    yb, _ = C.unet_forward(p, x, store=C.bf16)
    assert np.linalg.norm(yb - y) <= 2e-2 * np.linalg.norm(y)
