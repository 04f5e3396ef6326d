"""Plain FP64 CPU reference of the learned initial guess (a 3D U-Net).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` (and nothing on the product
path).  The GPU library computes the same network with BF16 tensors and FP32
accumulation; this module states each operation by its definition, in
float64, with no blocking or fusion.

The paper's method is insensitive to the first guess (Sec. 2, Sec. 6): the
learned guess only replaces the zero start of the V-cycle iteration, whose
FP64 stopping test is unchanged.  The network and its conventions are this
library's own, fixed here:

* tensors are channels-last ``(N, D, H, W, C)``;
* a 3x3x3 convolution with zero padding has weights ``w[tap, co, ci]`` with
  ``tap = 9 (dz + 1) + 3 (dy + 1) + (dx + 1)``; it computes
  ``out[v, co] = b[co] + sum_tap sum_ci w[tap, co, ci] x[v + (dz, dy, dx), ci]``;
* down-sampling is the 2x2x2 mean, up-sampling is nearest (each coarse value
  copied to its 8 children), skips are channel concatenations with the
  up-sampled tensor first;
* every 3x3x3 convolution is followed by ReLU; the head is a 1x1x1 map from 16
  channels to one;
* the input has 16 channels: rho / s on active cells (0 elsewhere), the mask
  (+1 / -1), the Dirichlet field / s, and 13 zero channels, where ``s`` is the
  root mean square of rho over active cells; the guess is
  ``phi0 = s * y / 256`` on active cells and 0 elsewhere.

Parameter vector (float32 on the device, float64 here): for each layer of
``LAYERS`` in order, its weights ``[27, cout, cin]`` then its bias
``[cout]``; last the head weights ``[16]`` and head bias ``[1]``.
"""
from __future__ import annotations

import numpy as np

OUT_SCALE = 1.0 / 256.0
IN_CHANNELS = 16

# (name, channels of the up-sampled input, channels of the full-resolution
# input, output channels, level); level 1 is the input resolution.
LAYERS = [
    ("enc1a", 0, 16, 16, 1), ("enc1b", 0, 16, 16, 1),
    ("enc2a", 0, 16, 32, 2), ("enc2b", 0, 32, 32, 2),
    ("enc3a", 0, 32, 64, 3), ("enc3b", 0, 64, 64, 3),
    ("mid4a", 0, 64, 128, 4), ("mid4b", 0, 128, 128, 4),
    ("dec3a", 128, 64, 64, 3), ("dec3b", 0, 64, 64, 3),
    ("dec2a", 64, 32, 32, 2), ("dec2b", 0, 32, 32, 2),
    ("dec1a", 32, 16, 16, 1), ("dec1b", 0, 16, 16, 1),
]


def param_layout():
    """Offsets ``{name: (w_off, b_off, cin, cout)}`` and the total count."""
    off = 0
    lay = {}
    for name, ca, cb, co, _ in LAYERS:
        cin = ca + cb
        lay[name] = (off, off + 27 * co * cin, cin, co)
        off += 27 * co * cin + co
    lay["head"] = (off, off + 16, 16, 1)
    return lay, off + 17


def unpack(params):
    """Split a flat parameter vector into ``{name: (w, b)}`` views."""
    lay, total = param_layout()
    assert params.size == total
    out = {}
    for name, (wo, bo, cin, co) in lay.items():
        if name == "head":
            out[name] = (params[wo:wo + 16], params[bo:bo + 1])
        else:
            out[name] = (params[wo:bo].reshape(27, co, cin), params[bo:bo + co])
    return out


def taps():
    """The 27 offsets (dz, dy, dx) in tap order."""
    return [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def _shift(x, dz, dy, dx):
    """``y[n, z, y, x] = x[n, z + dz, y + dy, x + dx]`` with zeros outside."""
    N, D, H, W, C = x.shape
    p = np.zeros((N, D + 2, H + 2, W + 2, C), x.dtype)
    p[:, 1:-1, 1:-1, 1:-1] = x
    return p[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W]


# ------------------------------------------------------------ primitives
def conv3d(x, w, b, relu=True):
    """3x3x3 convolution with zero padding (then ReLU) by its definition."""
    out = np.zeros(x.shape[:4] + (w.shape[1],))
    for t, (dz, dy, dx) in enumerate(taps()):
        out += _shift(x, dz, dy, dx) @ w[t].T
    out += b
    return np.maximum(out, 0.0) if relu else out


def conv3d_backward(x, w, dout):
    """Gradients of ``sum(dout * conv3d(x, w, b, relu=False))``.

    dx[v] = sum_tap w[tap]^T dout[v - shift(tap)], dw[tap] = sum_v dout[v]
    x[v + shift(tap)]^T, db = sum_v dout[v].
    """
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    dflat = dout.reshape(-1, dout.shape[-1])
    for t, (dz, dy, dx_) in enumerate(taps()):
        dx += _shift(dout, -dz, -dy, -dx_) @ w[t]
        dw[t] = dflat.T @ _shift(x, dz, dy, dx_).reshape(-1, x.shape[-1])
    db = dflat.sum(axis=0)
    return dx, dw, db


def pool2(x):
    """Mean over each 2x2x2 block."""
    N, D, H, W, C = x.shape
    return x.reshape(N, D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4, 6))


def pool2_backward(dy):
    """Adjoint of ``pool2``: each child receives 1/8 of its parent's gradient."""
    return up2_nearest(dy) / 8.0


def up2_nearest(x):
    """Copy each value to its 8 children."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2_nearest_backward(dy):
    """Adjoint of ``up2_nearest``: sum over the 8 children."""
    N, D, H, W, C = dy.shape
    return dy.reshape(N, D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4, 6))


# ------------------------------------------------------------- network
def _exact(t):
    return t


def forward(params, x, keep=False, store=_exact):
    """U-Net forward; returns the head output ``y`` of shape (N, D, H, W)
    and, if ``keep``, every intermediate activation.

    ``store`` maps each tensor that is kept between layers (convolution and
    pooling outputs) to the values actually kept; the default keeps them
    exactly.  Tests pass a rounding to a storage format to model a device
    that keeps activations in that format."""
    P = unpack(params)
    a = {"x": x}

    def conv(name, inp):
        w, b = P[name]
        return store(conv3d(inp, w, b, relu=True))

    a["enc1a"] = conv("enc1a", x)
    a["enc1b"] = conv("enc1b", a["enc1a"])
    a["pool1"] = store(pool2(a["enc1b"]))
    a["enc2a"] = conv("enc2a", a["pool1"])
    a["enc2b"] = conv("enc2b", a["enc2a"])
    a["pool2"] = store(pool2(a["enc2b"]))
    a["enc3a"] = conv("enc3a", a["pool2"])
    a["enc3b"] = conv("enc3b", a["enc3a"])
    a["pool3"] = store(pool2(a["enc3b"]))
    a["mid4a"] = conv("mid4a", a["pool3"])
    a["mid4b"] = conv("mid4b", a["mid4a"])
    a["cat3"] = np.concatenate([up2_nearest(a["mid4b"]), a["enc3b"]], axis=-1)
    a["dec3a"] = conv("dec3a", a["cat3"])
    a["dec3b"] = conv("dec3b", a["dec3a"])
    a["cat2"] = np.concatenate([up2_nearest(a["dec3b"]), a["enc2b"]], axis=-1)
    a["dec2a"] = conv("dec2a", a["cat2"])
    a["dec2b"] = conv("dec2b", a["dec2a"])
    a["cat1"] = np.concatenate([up2_nearest(a["dec2b"]), a["enc1b"]], axis=-1)
    a["dec1a"] = conv("dec1a", a["cat1"])
    a["dec1b"] = conv("dec1b", a["dec1a"])
    hw, hb = P["head"]
    y = a["dec1b"] @ hw + hb[0]
    return (y, a) if keep else y


def loss(params, x, active, target):
    """Mean over active cells of (y - target)^2."""
    y = forward(params, x)
    d = (y - target)[active]
    return float((d * d).mean())


def loss_and_grad(params, x, active, target, store=_exact):
    """Loss and its gradient with respect to the flat parameter vector, by
    the chain rule through each layer (reverse order of ``forward``).
    ``store`` as in ``forward``, applied also to each activation gradient
    kept between layers."""
    P = unpack(params)
    lay, total = param_layout()
    g = np.zeros(total)
    y, a = forward(params, x, keep=True, store=store)
    cnt = int(active.sum())
    d = np.where(active, y - target, 0.0)
    L = float((d * d).sum() / cnt)
    dy = 2.0 * d / cnt
    hw, hb = P["head"]
    wo, bo, _, _ = lay["head"]
    g[wo:wo + 16] = (a["dec1b"] * dy[..., None]).reshape(-1, 16).sum(axis=0)
    g[bo] = dy.sum()
    grad = {"dec1b": store(dy[..., None] * hw)}

    def conv_back(name, inp_key, out_grad):
        """ReLU then convolution backward; returns the input gradient."""
        w, _ = P[name]
        dpre = np.where(a[name] > 0.0, out_grad, 0.0)
        dx, dw, db = conv3d_backward(a[inp_key], w, dpre)
        wo_, bo_, cin, co = lay[name]
        g[wo_:bo_] = dw.ravel()
        g[bo_:bo_ + co] = db
        return store(dx)

    def split(dcat, c_up):
        return store(up2_nearest_backward(dcat[..., :c_up])), dcat[..., c_up:]

    grad["dec1a"] = conv_back("dec1b", "dec1a", grad["dec1b"])
    d_up, d_skip1 = split(conv_back("dec1a", "cat1", grad["dec1a"]), 32)
    grad["dec2b"] = d_up
    grad["dec2a"] = conv_back("dec2b", "dec2a", grad["dec2b"])
    d_up, d_skip2 = split(conv_back("dec2a", "cat2", grad["dec2a"]), 64)
    grad["dec3b"] = d_up
    grad["dec3a"] = conv_back("dec3b", "dec3a", grad["dec3b"])
    d_up, d_skip3 = split(conv_back("dec3a", "cat3", grad["dec3a"]), 128)
    grad["mid4b"] = d_up
    grad["mid4a"] = conv_back("mid4b", "mid4a", grad["mid4b"])
    d_pool3 = conv_back("mid4a", "pool3", grad["mid4a"])
    grad["enc3b"] = store(d_skip3 + pool2_backward(d_pool3))
    grad["enc3a"] = conv_back("enc3b", "enc3a", grad["enc3b"])
    d_pool2 = conv_back("enc3a", "pool2", grad["enc3a"])
    grad["enc2b"] = store(d_skip2 + pool2_backward(d_pool2))
    grad["enc2a"] = conv_back("enc2b", "enc2a", grad["enc2b"])
    d_pool1 = conv_back("enc2a", "pool1", grad["enc2a"])
    grad["enc1b"] = store(d_skip1 + pool2_backward(d_pool1))
    grad["enc1a"] = conv_back("enc1b", "enc1a", grad["enc1b"])
    conv_back("enc1a", "x", grad["enc1a"])
    return L, g


def adamw(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
    """One AdamW update (decoupled weight decay) with bias-corrected moments;
    returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    p = params * (1.0 - lr * weight_decay) - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


# --------------------------------------------------- input and output maps
def input_scale(rho, mask):
    """Root mean square of rho over active cells (1 if it is zero)."""
    a = mask == 1
    s = float(np.sqrt(np.mean(rho[a] ** 2))) if a.any() else 0.0
    return s if s > 0.0 else 1.0


def pack_input(rho, mask, dirichlet=None, stride=1):
    """Network input (1, D/stride, H/stride, W/stride, 16) and the scale s.

    For stride 1 the channels are rho/s on active cells, the mask and B/s.
    For stride > 1 each coarse cell summarises its stride^3 fine cells: the
    mean of rho over its active children, +1 if more than half of them are
    active (else -1), and the mean of B over all of them.
    """
    s = input_scale(rho, mask)
    act = (mask == 1)
    nz, ny, nx = mask.shape
    S = stride
    cz, cy, cx = nz // S, ny // S, nx // S

    def blocks(a):
        return a.reshape(cz, S, cy, S, cx, S).transpose(0, 2, 4, 1, 3, 5).reshape(cz, cy, cx, S ** 3)

    cnt = blocks(act.astype(np.float64)).sum(axis=-1)
    rsum = blocks(np.where(act, rho, 0.0)).sum(axis=-1)
    x = np.zeros((1, cz, cy, cx, IN_CHANNELS))
    x[0, ..., 0] = np.where(cnt > 0, rsum / np.maximum(cnt, 1), 0.0) / s
    x[0, ..., 1] = np.where(2 * cnt > S ** 3, 1.0, -1.0)
    if dirichlet is not None:
        x[0, ..., 2] = blocks(dirichlet).mean(axis=-1) / s
    return x, s


def up2_linear(c):
    """Cell-centred linear interpolation to the 2x finer grid, per axis
    3/4 of the parent and 1/4 of the next coarse cell on the child's side
    (the edge cell is repeated past the array end)."""
    out = c
    for ax in range(3):
        n = out.shape[ax]
        i = np.arange(2 * n)
        p = i // 2
        q = np.clip(np.where(i % 2 == 0, p - 1, p + 1), 0, n - 1)
        out = 0.75 * np.take(out, p, axis=ax) + 0.25 * np.take(out, q, axis=ax)
    return out


def guess(params, rho, mask, dirichlet=None, stride=1):
    """Learned first guess on the fine grid: network at 1/stride resolution,
    linear up-sampling by 2 per step, zero on inactive cells."""
    x, s = pack_input(rho, mask, dirichlet, stride)
    y = forward(params, x)[0] * (s * OUT_SCALE)
    while y.shape != mask.shape:
        y = up2_linear(y)
    return np.where(mask == 1, y, 0.0)


def init_params(seed=0):
    """He-normal weights (std sqrt(2 / (27 cin))), zero biases, head std
    sqrt(1/16)."""
    rng = np.random.default_rng(seed)
    lay, total = param_layout()
    p = np.zeros(total)
    for name, (wo, bo, cin, co) in lay.items():
        fan = 16 if name == "head" else 27 * cin
        p[wo:bo] = rng.standard_normal(bo - wo) * np.sqrt((1.0 if name == "head" else 2.0) / fan)
    return p
