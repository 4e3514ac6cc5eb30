"""The U-Net's HIP kernels (bf16 MFMA, fp32 accumulation) against the FP64
oracle of the same network: forward outputs and every parameter gradient.

The network is specified with bf16 weights and activations, so the oracle is
fed the bf16-rounded parameters and runs with bf16 storage at the points
where the kernels store a tensor (every sum still exact, in float64).  Then
only fp32-vs-float64 accumulation differs, which moves an occasional stored
value by one bf16 step: bars 2e-3 on the output, 1e-2 on each gradient
tensor (relative L2).  Against the oracle without the storage rounding the
output still agrees to 2e-2 (one bf16 rounding per layer); the gradients do
not, by 6-8 % in these small random cases, which a float64 emulation of the
same rounding on the CPU reproduces."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_1009_2288_amd import eptv
    eptv.library()
    return eptv


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def flatten(p, shapes):
    return np.concatenate([np.concatenate([p[k + ".w"].ravel(), p[k + ".b"].ravel()]) for k in shapes])


def unflatten(flat, shapes):
    out, o = {}, 0
    for k, (ws, bs) in shapes.items():
        n = int(np.prod(ws))
        out[k + ".w"] = flat[o:o + n].reshape(ws)
        o += n
        out[k + ".b"] = flat[o:o + bs[0]]
        o += bs[0]
    return out


@pytest.mark.parametrize("c_in,c_out,base,levels,n,h,w", [
    (1, 3, 8, 1, 2, 16, 24),     # one level: 3x3 convs (scalar and vector gathers) and the 1x1 head
    (2, 3, 8, 3, 2, 32, 32),     # pooling, transposed convs, skip concatenation
    (1, 3, 16, 4, 1, 64, 64),    # four levels
    (1, 3, 8, 2, 3, 48, 80),     # several pixel chunks in the gradient sums, a ragged last one
    # 3x3 weight gradients from LDS tiles (C_in a multiple of 32): ragged tile
    # rows and columns at both levels
    (1, 3, 32, 2, 2, 36, 72),
    # ... 48 output channels (a half-empty channel block), three 32-channel
    # chunks, two tiles per pixel chunk, ragged columns
    (1, 3, 48, 2, 2, 96, 136),
    # 8-row x 64-channel conv tiles (the forward's direct epilogue, the
    # backward's LDS-staged one with the ReLU mask), ragged rows and columns
    (1, 3, 64, 1, 4, 124, 250),
])
def test_unet_forward_and_gradients_match_oracle(E, c_in, c_out, base, levels, n, h, w):
    shapes = C.unet_shapes(c_in, c_out, base, levels)
    p = C.unet_init(shapes, seed=11)
    rng = np.random.default_rng(12)
    for k in p:
        if k.endswith(".b"):
            p[k] = rng.normal(scale=0.05, size=p[k].shape)
    net = E.UNet(c_in, c_out, base, levels, n, h, w)
    flat = flatten(p, shapes)
    assert flat.size == net.n_params
    net.set_params(flat)
    pq = {k: C.bf16(v) if k.endswith(".w") else np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}
    x = rng.normal(size=(n, h, w, c_in))
    y = net.forward(torch.from_numpy(x.astype(np.float32)).cuda()).cpu().numpy()
    yo, cache = C.unet_forward(pq, x, store=C.bf16)
    assert rel(y, yo) <= 2e-3
    assert rel(y, C.unet_forward(pq, C.bf16(x))[0]) <= 2e-2
    dy = rng.normal(size=yo.shape)
    dx = net.backward(torch.from_numpy(dy.astype(np.float32)).cuda(), want_dx=True)
    go = C.unet_backward(pq, cache, dy, store=C.bf16)
    gg = unflatten(net.grads().astype(np.float64), shapes)
    errs = {k: rel(gg[k], go[k]) for k in gg}
    errs["x"] = rel(dx.cpu().numpy(), go["x"])
    print("relative errors", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-2, errs


def test_unet_adam_step_matches_oracle(E):
    shapes = C.unet_shapes(1, 3, 8, 2)
    p = C.unet_init(shapes, seed=21)
    net = E.UNet(1, 3, 8, 2, 2, 16, 16)
    net.set_params(flatten(p, shapes))
    rng = np.random.default_rng(22)
    x = torch.from_numpy(rng.normal(size=(2, 16, 16, 1)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.normal(size=(2, 16, 16, 3)).astype(np.float32)).cuda()
    y = net.forward(x)
    loss, dy = net.mse(y, t)
    yn, tn = y.cpu().numpy().astype(np.float64), t.cpu().numpy().astype(np.float64)
    lo, go = C.mse(yn, tn)
    assert abs(float(loss.item()) - lo) <= 1e-5 * lo
    assert rel(dy.cpu().numpy(), go) <= 1e-5
    net.backward(dy)
    g = net.grads().astype(np.float64)
    before = net.params().astype(np.float64)
    net.adam(1e-3, step=1)
    after = net.params().astype(np.float64)
    pd, gd = {"a": before.copy()}, {"a": g}
    C.adam_step(pd, gd, {"a": np.zeros_like(g)}, {"a": np.zeros_like(g)}, step=1, lr=1e-3)
    np.testing.assert_allclose(after, pd["a"], rtol=1e-5, atol=1e-7)


def test_maps_between_eptv_and_network_layout(E):
    """The 3-channel network layout of an image and its half-edge weights and
    back: a pure re-indexing with the image scaled, clamps on the way back,
    the border half-edges copied from their neighbours (bit for bit)."""
    rng = np.random.default_rng(4)
    n, ny, nx, s = 2, 5, 7, 50.0
    f = rng.uniform(0, 0.03, (n, ny, nx)).astype(np.float32)
    wx = rng.uniform(0, 1, (n, ny, nx + 1)).astype(np.float32)
    wy = rng.uniform(0, 1, (n, ny + 1, nx)).astype(np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    m = E.maps_from_eptv(dev(f), dev(wx), dev(wy), scale=s).cpu().numpy()
    assert m.shape == (n, ny, nx, 3)
    assert np.array_equal(m[..., 0], wx[:, :, 1:])
    assert np.array_equal(m[..., 1], wy[:, 1:, :])
    assert np.array_equal(m[..., 2], f * np.float32(s))
    m1 = E.maps_from_eptv(dev(f[0]), scale=s).cpu().numpy()
    assert m1.shape == (1, ny, nx, 1) and np.array_equal(m1[0, ..., 0], f[0] * np.float32(s))
    # back, from maps with out-of-range values
    q = rng.uniform(-0.5, 1.5, (n, ny, nx, 3)).astype(np.float32)
    f2, wx2, wy2 = (t.cpu().numpy() for t in E.maps_to_eptv(dev(q), scale=s))
    inv = np.float32(1) / np.float32(s)
    assert np.array_equal(f2, np.maximum(q[..., 2] * inv, 0))
    assert np.array_equal(wx2[:, :, 1:], np.clip(q[..., 0], 0, 1))
    assert np.array_equal(wx2[:, :, 0], wx2[:, :, 1])
    assert np.array_equal(wy2[:, 1:, :], np.clip(q[..., 1], 0, 1))
    assert np.array_equal(wy2[:, 0, :], wy2[:, 1, :])
    # residual form: the image channel relative to a base image
    b = rng.uniform(0, 0.03, (n, ny, nx)).astype(np.float32)
    mr = E.maps_from_eptv(dev(f), dev(wx), dev(wy), scale=s, f_base=dev(b)).cpu().numpy()
    assert np.array_equal(mr[..., 2], (f - b) * np.float32(s))
    f3, _, _ = (t.cpu().numpy() for t in E.maps_to_eptv(dev(q), scale=s, f_base=dev(b)))
    want = np.maximum(q[..., 2].astype(np.float64) * inv + b, 0)
    assert np.allclose(f3, want, rtol=2 ** -23, atol=1e-12)
    assert E._lib().eptv_maps_to_eptv(1, ny, nx, m.ctypes.data, 0.0, None, None, None, None,
                                      None) == E.EPTV_ERR_ARG
