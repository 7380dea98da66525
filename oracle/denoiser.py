"""FP64 reference of the learned dose denoiser (test infrastructure only).

The paper has no denoiser; this network is the batching-plus-learning extension
of the plain method: a 3D U-Net that maps a low-history Monte Carlo dose (with
its batch uncertainty and the density) to the dose of a high-history run. This
module is the plain, slow definition the GPU kernels are checked against:
every operation is written from its mathematical definition with numpy array
slicing and matrix products over the channel axis, in float64. It shares no
code with the HIP path. Only tests, the package smoke check and the
benchmark's CPU leg use it.

Layout: volumes are channels-last arrays [z, y, x, c]. A convolution weight is
[kz, ky, kx, c_in, c_out]; a bias is [c_out].

Network (reading of "4 levels, 16-64 channels"): level channels 16, 32, 48, 64.
  encoder level 1: conv3(3->16), conv3(16->16)
  encoder level l>1: down(c_{l-1}->c_l) = 2x2x2 stride-2 conv, conv3, conv3
  decoder level l<4: up(c_{l+1}->c_l) = 2x2x2 stride-2 transposed conv,
                     concatenate [skip, up], conv3(2 c_l->c_l), conv3(c_l->c_l)
  head: 1x1x1 conv(16->1) = delta; output y = x0 + delta (residual on the
  normalised low-history dose x0 = D_low / Dmax_low).
Every conv3, down and up is followed by ReLU; the head is linear. conv3 is a
3x3x3 convolution with stride 1 and zero padding 1.

Loss (per volume): weighted mean square error between y and the normalised
target t = D_high / Dmax_low, weight 1 where t > 0.1 max(t), else 0.1.
Optimiser: Adam with bias correction (Kingma and Ba, 2015).
"""
import numpy as np

CHANNELS = (16, 32, 48, 64)
IN_CHANNELS = 3


# ------------------------------------------------------------------ layers
def conv3d(x, w, b=None, stride=1, pad=1):
    """out[o, co] = b[co] + sum_{t, ci} xpad[o * stride + t, ci] w[t, ci, co]
    with xpad the input zero-padded by `pad` on every side."""
    k = w.shape[0]
    Z, Y, X, ci = x.shape
    co = w.shape[4]
    xp = np.pad(x, ((pad, pad), (pad, pad), (pad, pad), (0, 0)))
    Zo = (Z + 2 * pad - k) // stride + 1
    Yo = (Y + 2 * pad - k) // stride + 1
    Xo = (X + 2 * pad - k) // stride + 1
    out = np.zeros((Zo, Yo, Xo, co))
    for tz in range(k):
        for ty in range(k):
            for tx in range(k):
                patch = xp[tz:tz + stride * Zo:stride, ty:ty + stride * Yo:stride,
                           tx:tx + stride * Xo:stride]
                out += patch @ w[tz, ty, tx]
    if b is not None:
        out += b
    return out


def conv3d_bwd_data(g, w, in_shape, stride=1, pad=1):
    """Gradient with respect to the input of conv3d: every output gradient is
    sent back through the weight of each tap to the input voxel it read."""
    k = w.shape[0]
    Z, Y, X, _ = in_shape
    Zo, Yo, Xo, _ = g.shape
    gp = np.zeros((Z + 2 * pad, Y + 2 * pad, X + 2 * pad, w.shape[3]))
    for tz in range(k):
        for ty in range(k):
            for tx in range(k):
                gp[tz:tz + stride * Zo:stride, ty:ty + stride * Yo:stride,
                   tx:tx + stride * Xo:stride] += g @ w[tz, ty, tx].T
    return gp[pad:pad + Z, pad:pad + Y, pad:pad + X]


def conv3d_bwd_weight(x, g, k, stride=1, pad=1):
    """Gradient with respect to the weight: gw[t, ci, co] = sum_o xpad[o * stride
    + t, ci] g[o, co]."""
    ci = x.shape[3]
    co = g.shape[3]
    Zo, Yo, Xo, _ = g.shape
    xp = np.pad(x, ((pad, pad), (pad, pad), (pad, pad), (0, 0)))
    gw = np.zeros((k, k, k, ci, co))
    g2 = g.reshape(-1, co)
    for tz in range(k):
        for ty in range(k):
            for tx in range(k):
                patch = xp[tz:tz + stride * Zo:stride, ty:ty + stride * Yo:stride,
                           tx:tx + stride * Xo:stride]
                gw[tz, ty, tx] = patch.reshape(-1, ci).T @ g2
    return gw


def conv_transpose2(x, w, b=None):
    """2x2x2 stride-2 transposed convolution: out[2 v + t, co] = b[co] +
    sum_ci x[v, ci] w[t, ci, co]."""
    Z, Y, X, _ = x.shape
    co = w.shape[4]
    out = np.zeros((2 * Z, 2 * Y, 2 * X, co))
    for tz in range(2):
        for ty in range(2):
            for tx in range(2):
                out[tz::2, ty::2, tx::2] = x @ w[tz, ty, tx]
    if b is not None:
        out += b
    return out


def conv_transpose2_bwd_data(g, w):
    gx = 0.0
    for tz in range(2):
        for ty in range(2):
            for tx in range(2):
                gx = gx + g[tz::2, ty::2, tx::2] @ w[tz, ty, tx].T
    return gx


def conv_transpose2_bwd_weight(x, g):
    ci = x.shape[3]
    co = g.shape[3]
    gw = np.zeros((2, 2, 2, ci, co))
    x2 = x.reshape(-1, ci)
    for tz in range(2):
        for ty in range(2):
            for tx in range(2):
                gw[tz, ty, tx] = x2.T @ g[tz::2, ty::2, tx::2].reshape(-1, co)
    return gw


def relu(x):
    return np.maximum(x, 0.0)


# ------------------------------------------------------------------ network
def layer_specs():
    """(name, kind, c_in, c_out) in parameter order; kind is conv3, down, up or
    head. The flat parameter vector is, layer by layer, the weight
    [kz, ky, kx, c_in, c_out] in C order followed by the bias [c_out]."""
    c1, c2, c3, c4 = CHANNELS
    return [("enc1a", "conv3", IN_CHANNELS, c1), ("enc1b", "conv3", c1, c1),
            ("down2", "down", c1, c2), ("enc2a", "conv3", c2, c2), ("enc2b", "conv3", c2, c2),
            ("down3", "down", c2, c3), ("enc3a", "conv3", c3, c3), ("enc3b", "conv3", c3, c3),
            ("down4", "down", c3, c4), ("enc4a", "conv3", c4, c4), ("enc4b", "conv3", c4, c4),
            ("up3", "up", c4, c3), ("dec3a", "conv3", 2 * c3, c3), ("dec3b", "conv3", c3, c3),
            ("up2", "up", c3, c2), ("dec2a", "conv3", 2 * c2, c2), ("dec2b", "conv3", c2, c2),
            ("up1", "up", c2, c1), ("dec1a", "conv3", 2 * c1, c1), ("dec1b", "conv3", c1, c1),
            ("head", "head", c1, 1)]


def kernel_size(kind):
    return {"conv3": 3, "down": 2, "up": 2, "head": 1}[kind]


def unflatten(theta):
    """Split the flat parameter vector into {name: (w, b)}."""
    out, at = {}, 0
    for name, kind, ci, co in layer_specs():
        k = kernel_size(kind)
        nw = k * k * k * ci * co
        w = theta[at:at + nw].reshape(k, k, k, ci, co)
        at += nw
        b = theta[at:at + co]
        at += co
        out[name] = (w, b)
    assert at == theta.size
    return out


def num_params():
    return sum(kernel_size(k) ** 3 * ci * co + co for _, k, ci, co in layer_specs())


def normalise(dose, sigma, rho, dmax):
    """Network input channels [x0, s0, r0] = [D / Dmax, sigma / Dmax, rho / 2]."""
    return np.stack([dose / dmax, sigma / dmax, rho / 2.0], axis=-1)


def _identity(v):
    return v


def forward(theta, x, store=_identity):
    """x: [Z, Y, X, 3] normalised input (Z, Y, X multiples of 8). Returns y =
    x0 + delta and the activations the backward pass needs. `store` is applied
    to every hidden activation as it is kept (identity: plain FP64; a rounding
    function reproduces an implementation that stores activations in a
    narrower format)."""
    P = unflatten(theta)
    a = {"x": x}

    def c3(name, inp):
        w, b = P[name]
        return store(relu(conv3d(inp, w, b, 1, 1)))

    def down(name, inp):
        w, b = P[name]
        return store(relu(conv3d(inp, w, b, 2, 0)))

    def up(name, inp):
        w, b = P[name]
        return store(relu(conv_transpose2(inp, w, b)))

    a["enc1a"] = c3("enc1a", x)
    a["enc1b"] = c3("enc1b", a["enc1a"])
    for l in (2, 3, 4):
        a[f"down{l}"] = down(f"down{l}", a[f"enc{l - 1}b"])
        a[f"enc{l}a"] = c3(f"enc{l}a", a[f"down{l}"])
        a[f"enc{l}b"] = c3(f"enc{l}b", a[f"enc{l}a"])
    prev = a["enc4b"]
    for l in (3, 2, 1):
        a[f"up{l}"] = up(f"up{l}", prev)
        a[f"cat{l}"] = np.concatenate([a[f"enc{l}b"], a[f"up{l}"]], axis=-1)
        a[f"dec{l}a"] = c3(f"dec{l}a", a[f"cat{l}"])
        a[f"dec{l}b"] = c3(f"dec{l}b", a[f"dec{l}a"])
        prev = a[f"dec{l}b"]
    wh, bh = P["head"]
    delta = prev @ wh[0, 0, 0] + bh
    y = x[..., 0] + delta[..., 0]
    return y, a


def loss_weights(t):
    return np.where(t > 0.1 * t.max(), 1.0, 0.1)


def loss(y, t):
    """Weighted mean square error and its gradient with respect to y."""
    w = loss_weights(t)
    W = w.sum()
    r = y - t
    return float((w * r * r).sum() / W), 2.0 * w * r / W


def backward(theta, a, gy, store=_identity):
    """Gradient of a scalar with respect to theta, given its gradient gy with
    respect to the output y (chain rule through every layer, in reverse).
    `store` is applied to every gradient after its ReLU mask (see forward)."""
    P = unflatten(theta)
    G = {}

    def relu_mask(g, out):
        return store(g * (out > 0))

    wh, bh = P["head"]
    gdelta = gy[..., None]
    G["head"] = (np.einsum("zyxc,zyxo->co", a["dec1b"], gdelta).reshape(1, 1, 1, -1, 1),
                 gdelta.sum(axis=(0, 1, 2)))
    gprev = gdelta @ wh[0, 0, 0].T
    gskip = {}
    for l in (1, 2, 3):
        g = relu_mask(gprev, a[f"dec{l}b"])
        w, _ = P[f"dec{l}b"]
        G[f"dec{l}b"] = (conv3d_bwd_weight(a[f"dec{l}a"], g, 3), g.sum(axis=(0, 1, 2)))
        g = conv3d_bwd_data(g, w, a[f"dec{l}a"].shape)
        g = relu_mask(g, a[f"dec{l}a"])
        w, _ = P[f"dec{l}a"]
        G[f"dec{l}a"] = (conv3d_bwd_weight(a[f"cat{l}"], g, 3), g.sum(axis=(0, 1, 2)))
        gcat = conv3d_bwd_data(g, w, a[f"cat{l}"].shape)
        c = a[f"enc{l}b"].shape[-1]
        gskip[l] = gcat[..., :c]
        g = relu_mask(gcat[..., c:], a[f"up{l}"])
        w, _ = P[f"up{l}"]
        src = a["enc4b"] if l == 3 else a[f"dec{l + 1}b"]
        G[f"up{l}"] = (conv_transpose2_bwd_weight(src, g), g.sum(axis=(0, 1, 2)))
        gprev = conv_transpose2_bwd_data(g, w)
    # gprev is now the gradient at enc4b
    for l in (4, 3, 2, 1):
        g = gprev if l == 4 else gprev + gskip[l]
        g = relu_mask(g, a[f"enc{l}b"])
        w, _ = P[f"enc{l}b"]
        G[f"enc{l}b"] = (conv3d_bwd_weight(a[f"enc{l}a"], g, 3), g.sum(axis=(0, 1, 2)))
        g = conv3d_bwd_data(g, w, a[f"enc{l}a"].shape)
        g = relu_mask(g, a[f"enc{l}a"])
        w, _ = P[f"enc{l}a"]
        inp = a["x"] if l == 1 else a[f"down{l}"]
        G[f"enc{l}a"] = (conv3d_bwd_weight(inp, g, 3), g.sum(axis=(0, 1, 2)))
        if l == 1:
            break
        g = conv3d_bwd_data(g, w, inp.shape)
        g = relu_mask(g, a[f"down{l}"])
        w, _ = P[f"down{l}"]
        G[f"down{l}"] = (conv3d_bwd_weight(a[f"enc{l - 1}b"], g, 2, 2, 0), g.sum(axis=(0, 1, 2)))
        gprev = conv3d_bwd_data(g, w, a[f"enc{l - 1}b"].shape, 2, 0)
    flat = []
    for name, _, _, _ in layer_specs():
        gw, gb = G[name]
        flat += [gw.ravel(), gb.ravel()]
    return np.concatenate(flat)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0, scale=1.0):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, kind, ci, co in layer_specs():
        k = kernel_size(kind)
        fan = k ** 3 * ci
        parts.append(rng.normal(0.0, scale * np.sqrt(2.0 / fan), k ** 3 * ci * co))
        parts.append(np.zeros(co))
    return np.concatenate(parts)
