"""Pins of the FP64 denoiser oracle against definitions it does not share code
with: brute-force loops, scipy's correlation, the adjoint identity of the
transposed convolution, central finite differences of the whole network, and
closed forms of the loss and of Adam's first step."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import denoiser as dn


def brute_conv(x, w, b, stride, pad):
    Z, Y, X, ci = x.shape
    k, co = w.shape[0], w.shape[4]
    Zo = (Z + 2 * pad - k) // stride + 1
    Yo = (Y + 2 * pad - k) // stride + 1
    Xo = (X + 2 * pad - k) // stride + 1
    out = np.zeros((Zo, Yo, Xo, co))
    for oz in range(Zo):
        for oy in range(Yo):
            for ox in range(Xo):
                for o in range(co):
                    s = b[o]
                    for tz in range(k):
                        for ty in range(k):
                            for tx in range(k):
                                z = oz * stride + tz - pad
                                y = oy * stride + ty - pad
                                xx = ox * stride + tx - pad
                                if 0 <= z < Z and 0 <= y < Y and 0 <= xx < X:
                                    for i in range(ci):
                                        s += x[z, y, xx, i] * w[tz, ty, tx, i, o]
                    out[oz, oy, ox, o] = s
    return out


@pytest.mark.parametrize("k,stride,pad,shape", [(3, 1, 1, (3, 4, 5)), (2, 2, 0, (4, 2, 6)),
                                                (1, 1, 0, (2, 3, 2))])
def test_conv3d_brute_force(k, stride, pad, shape):
    rng = np.random.default_rng(1)
    x = rng.normal(size=shape + (2,))
    w = rng.normal(size=(k, k, k, 2, 3))
    b = rng.normal(size=3)
    np.testing.assert_allclose(dn.conv3d(x, w, b, stride, pad), brute_conv(x, w, b, stride, pad),
                               rtol=1e-12, atol=1e-12)


def test_conv3d_single_channel_is_scipy_correlate():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(6, 5, 7))
    w = rng.normal(size=(3, 3, 3))
    ref = ndimage.correlate(x, w, mode="constant", cval=0.0)
    got = dn.conv3d(x[..., None], w[..., None, None])[..., 0]
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def _fd_check(f, arr, grad, idx, h=1e-6):
    for i in idx:
        old = arr.flat[i]
        arr.flat[i] = old + h
        fp = f()
        arr.flat[i] = old - h
        fm = f()
        arr.flat[i] = old
        assert (fp - fm) / (2 * h) == pytest.approx(grad.flat[i], rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("k,stride,pad", [(3, 1, 1), (2, 2, 0)])
def test_conv3d_gradients_finite_differences(k, stride, pad):
    rng = np.random.default_rng(3)
    x = rng.normal(size=(4, 4, 6, 3))
    w = rng.normal(size=(k, k, k, 3, 2))
    y0 = dn.conv3d(x, w, None, stride, pad)
    g = rng.normal(size=y0.shape)

    def f():
        return float((dn.conv3d(x, w, None, stride, pad) * g).sum())

    gx = dn.conv3d_bwd_data(g, w, x.shape, stride, pad)
    gw = dn.conv3d_bwd_weight(x, g, k, stride, pad)
    _fd_check(f, x, gx, rng.choice(x.size, 25, replace=False))
    _fd_check(f, w, gw, rng.choice(w.size, 25, replace=False))


def test_conv_transpose2_definition_and_adjoint():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(2, 3, 2, 3))
    w = rng.normal(size=(2, 2, 2, 3, 4))
    out = dn.conv_transpose2(x, w)
    for z, y, xx in np.ndindex(4, 6, 4):
        v = (z // 2, y // 2, xx // 2)
        t = (z % 2, y % 2, xx % 2)
        np.testing.assert_allclose(out[z, y, xx], x[v] @ w[t], rtol=1e-12)
    # <up(x; w), g> = <x, down(g; w^T)>: the transposed convolution is the
    # adjoint of the 2x2x2 stride-2 convolution with channels swapped
    g = rng.normal(size=out.shape)
    down = dn.conv3d(g, np.swapaxes(w, 3, 4), None, 2, 0)
    assert float((out * g).sum()) == pytest.approx(float((x * down).sum()), rel=1e-12)
    np.testing.assert_allclose(dn.conv_transpose2_bwd_data(g, w), down, rtol=1e-12, atol=1e-12)
    gw = dn.conv_transpose2_bwd_weight(x, g)

    def f():
        return float((dn.conv_transpose2(x, w) * g).sum())

    _fd_check(f, w, gw, rng.choice(w.size, 20, replace=False))


def test_network_shapes_and_identity():
    theta = np.zeros(dn.num_params())
    P = dn.unflatten(theta)
    assert set(P) == {s[0] for s in dn.layer_specs()}
    # zero weights: every hidden activation is 0, delta = head bias
    P["head"][1][:] = 0.25
    x = np.random.default_rng(5).random((8, 8, 16, 3))
    y, a = dn.forward(theta, x)
    np.testing.assert_allclose(y, x[..., 0] + 0.25, rtol=1e-15)
    assert a["enc4b"].shape == (1, 1, 2, 64) and a["cat1"].shape == (8, 8, 16, 32)
    assert 0.7e6 < dn.num_params() < 0.8e6


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(6)
    theta = dn.init_params(seed=7)
    # positive biases keep most ReLUs away from their kink for the difference
    P = dn.unflatten(theta)
    for name, (w, b) in P.items():
        b[:] = 0.05
    x = rng.random((8, 8, 8, 3))
    t = x[..., 0] * 1.1 + 0.05 * rng.random((8, 8, 8))

    def f():
        y, _ = dn.forward(theta, x)
        return dn.loss(y, t)[0]

    y, a = dn.forward(theta, x)
    _, gy = dn.loss(y, t)
    g = dn.backward(theta, a, gy)
    assert g.shape == theta.shape
    # one weight and one bias from every layer
    idx, at = [], 0
    for _, kind, ci, co in dn.layer_specs():
        nw = dn.kernel_size(kind) ** 3 * ci * co
        idx += [at + int(rng.integers(nw)), at + nw + int(rng.integers(co))]
        at += nw + co
    for i in idx:
        old = theta[i]
        theta[i] = old + 1e-6
        fp = f()
        theta[i] = old - 1e-6
        fm = f()
        theta[i] = old
        assert (fp - fm) / 2e-6 == pytest.approx(g[i], rel=1e-4, abs=1e-9), i


def test_loss_closed_form():
    t = np.array([0.0, 0.05, 0.5, 1.0])
    y = np.array([0.1, 0.05, 0.4, 1.2])
    # weights 0.1, 0.1, 1, 1 (threshold 0.1 of max t = 1)
    W = 2.2
    ref = (0.1 * 0.01 + 0 + 0.01 + 0.04) / W
    L, g = dn.loss(y, t)
    assert L == pytest.approx(ref, rel=1e-14)
    np.testing.assert_allclose(g, 2 * np.array([0.1, 0.1, 1, 1]) * (y - t) / W, rtol=1e-14)


def test_adam_first_steps():
    g = np.array([3.0, -0.5, 1e-3])
    th, m, v = dn.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01, eps=0.0)
    # bias-corrected first step: m_hat / sqrt(v_hat) = g / |g|
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-12)
    # constant gradient: every step moves by lr (m_hat = g, v_hat = g^2)
    for s in range(2, 6):
        th, m, v = dn.adam_step(th, g, m, v, s, 0.01, eps=0.0)
    np.testing.assert_allclose(th, -0.05 * np.sign(g), rtol=1e-10)


def test_store_hook_defaults_to_plain_fp64():
    """The optional storage-rounding hook is the identity unless given: a
    rounding that does nothing leaves forward and backward bit-identical."""
    rng = np.random.default_rng(8)
    theta = dn.init_params(seed=2)
    x = rng.random((8, 8, 8, 3))
    y0, a0 = dn.forward(theta, x)
    y1, a1 = dn.forward(theta, x, store=lambda v: v + 0.0)
    assert np.array_equal(y0, y1)
    t = x[..., 0] * 0.9
    g0 = dn.backward(theta, a0, dn.loss(y0, t)[1])
    g1 = dn.backward(theta, a1, dn.loss(y1, t)[1], store=lambda v: v * 1.0)
    assert np.array_equal(g0, g1)
    # a coarse rounding changes both (the hook is applied)
    y2, _ = dn.forward(theta, x, store=lambda v: np.round(v, 1))
    assert not np.array_equal(y0, y2)
