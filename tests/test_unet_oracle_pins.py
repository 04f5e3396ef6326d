"""Pins of the FP64 U-Net oracle (learned first guess) against things other
than itself: torch's CPU convolution and autograd (an independent library
implementation), central finite differences, adjoint identities, closed
forms of AdamW's first step and exactness of linear interpolation."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet_oracle as U

pytestmark = pytest.mark.filterwarnings("ignore::UserWarning")


def _torch_conv(x, w, b):
    # x (N, D, H, W, C) -> (N, C, D, H, W); w[tap, co, ci] -> (co, ci, 3, 3, 3)
    co, ci = w.shape[1], w.shape[2]
    tw = torch.from_numpy(w.reshape(3, 3, 3, co, ci).transpose(3, 4, 0, 1, 2).copy())
    tx = torch.from_numpy(x.transpose(0, 4, 1, 2, 3).copy())
    out = F.conv3d(tx, tw, torch.from_numpy(b), padding=1)
    return out.numpy().transpose(0, 2, 3, 4, 1)


def test_conv_matches_torch_library():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6, 7, 3))
    w = rng.standard_normal((27, 4, 3))
    b = rng.standard_normal(4)
    np.testing.assert_allclose(U.conv3d(x, w, b, relu=False), _torch_conv(x, w, b), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(U.conv3d(x, w, b, relu=True), np.maximum(_torch_conv(x, w, b), 0), atol=1e-12)


@pytest.mark.parametrize("tap", [0, 4, 13, 17, 26])
def test_conv_single_tap_is_a_shift(tap):
    rng = np.random.default_rng(tap)
    x = rng.standard_normal((1, 4, 5, 6, 2))
    w = np.zeros((27, 2, 2))
    w[tap] = np.eye(2)
    out = U.conv3d(x, w, np.zeros(2), relu=False)
    dz, dy, dx = tap // 9 - 1, (tap // 3) % 3 - 1, tap % 3 - 1
    for z in range(4):
        for y in range(5):
            for xx in range(6):
                zz, yy, x2 = z + dz, y + dy, xx + dx
                inside = 0 <= zz < 4 and 0 <= yy < 5 and 0 <= x2 < 6
                want = x[0, zz, yy, x2] if inside else np.zeros(2)
                assert np.array_equal(out[0, z, y, xx], want)


def test_conv_backward_adjoint_and_exact_weight_gradient():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 4, 4, 5, 3))
    w = rng.standard_normal((27, 2, 3))
    r = rng.standard_normal((1, 4, 4, 5, 2))
    dx, dw, db = U.conv3d_backward(x, w, r)
    lhs = float((U.conv3d(x, w, np.zeros(2), relu=False) * r).sum())
    assert abs(lhs - float((x * dx).sum())) <= 1e-11 * abs(lhs) + 1e-12
    # the output is linear in w: <conv(x, e_k), r> is exactly dw_k
    for k in [(0, 0, 0), (13, 1, 2), (26, 1, 1), (5, 0, 2)]:
        e = np.zeros_like(w)
        e[k] = 1.0
        val = float((U.conv3d(x, e, np.zeros(2), relu=False) * r).sum())
        assert abs(val - dw[k]) <= 1e-12 * (1 + abs(val))
    np.testing.assert_allclose(db, r.reshape(-1, 2).sum(axis=0), rtol=1e-13)


def test_pool_and_upsample_adjoint_and_values():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 6, 8, 3))
    c = rng.standard_normal((2, 2, 3, 4, 3))
    assert abs(float((U.pool2(x) * c).sum()) - float((x * U.pool2_backward(c)).sum())) < 1e-12
    assert abs(float((U.up2_nearest(c) * x).sum()) - float((c * U.up2_nearest_backward(x)).sum())) < 1e-12
    assert np.allclose(U.pool2(np.full((1, 2, 2, 2, 1), 3.5)), 3.5)
    up = U.up2_nearest(c)
    for z, y, xx in [(0, 0, 0), (3, 5, 7), (1, 2, 6)]:
        assert np.array_equal(up[1, z, y, xx], c[1, z // 2, y // 2, xx // 2])
    # pooling by brute force
    p = U.pool2(x)
    assert abs(p[1, 1, 2, 3, 2] - x[1, 2:4, 4:6, 6:8, 2].mean()) < 1e-15


def _torch_unet(params, x):
    """The same network written with torch's library operators."""
    P = {k: (torch.from_numpy(np.ascontiguousarray(w)), torch.from_numpy(np.ascontiguousarray(b)))
         for k, (w, b) in U.unpack(params).items()}
    t = torch.from_numpy(x.transpose(0, 4, 1, 2, 3).copy())

    def conv(name, inp):
        w, b = P[name]
        co, ci = w.shape[1], w.shape[2]
        return F.relu(F.conv3d(inp, w.reshape(3, 3, 3, co, ci).permute(3, 4, 0, 1, 2), b, padding=1))

    def up(a):
        return F.interpolate(a, scale_factor=2, mode="nearest")

    e1 = conv("enc1b", conv("enc1a", t))
    e2 = conv("enc2b", conv("enc2a", F.avg_pool3d(e1, 2)))
    e3 = conv("enc3b", conv("enc3a", F.avg_pool3d(e2, 2)))
    m4 = conv("mid4b", conv("mid4a", F.avg_pool3d(e3, 2)))
    d3 = conv("dec3b", conv("dec3a", torch.cat([up(m4), e3], 1)))
    d2 = conv("dec2b", conv("dec2a", torch.cat([up(d3), e2], 1)))
    d1 = conv("dec1b", conv("dec1a", torch.cat([up(d2), e1], 1)))
    hw, hb = P["head"]
    return torch.einsum("ncdhw,c->ndhw", d1, hw) + hb[0]


def _small_case(seed=3, n=8, batch=1):
    rng = np.random.default_rng(seed)
    params = U.init_params(seed)
    # non-zero biases so that every bias gradient is exercised
    lay, _ = U.param_layout()
    for name, (wo, bo, cin, co) in lay.items():
        params[bo:bo + co] = 0.05 * rng.standard_normal(co)
    x = rng.standard_normal((batch, n, n, n, 16))
    active = rng.random((batch, n, n, n)) < 0.6
    target = rng.standard_normal((batch, n, n, n))
    return params, x, active, target


def test_forward_matches_torch_library():
    params, x, _, _ = _small_case(batch=2, n=16)
    y = U.forward(params, x)
    want = _torch_unet(params, x).numpy()
    np.testing.assert_allclose(y, want, rtol=1e-10, atol=1e-12)


def test_gradient_matches_torch_autograd():
    params, x, active, target = _small_case()
    L, g = U.loss_and_grad(params, x, active, target)
    tp = torch.from_numpy(params.copy()).requires_grad_(True)
    P = tp  # differentiable parameter vector, sliced like the flat layout
    lay, _ = U.param_layout()

    def view(name):
        wo, bo, cin, co = lay[name]
        if name == "head":
            return P[wo:wo + 16], P[bo:bo + 1]
        return P[wo:bo].reshape(27, co, cin), P[bo:bo + co]

    t = torch.from_numpy(x.transpose(0, 4, 1, 2, 3).copy())

    def conv(name, inp):
        w, b = view(name)
        co, ci = w.shape[1], w.shape[2]
        return F.relu(F.conv3d(inp, w.reshape(3, 3, 3, co, ci).permute(3, 4, 0, 1, 2), b, padding=1))

    up = lambda a: F.interpolate(a, scale_factor=2, mode="nearest")
    e1 = conv("enc1b", conv("enc1a", t))
    e2 = conv("enc2b", conv("enc2a", F.avg_pool3d(e1, 2)))
    e3 = conv("enc3b", conv("enc3a", F.avg_pool3d(e2, 2)))
    m4 = conv("mid4b", conv("mid4a", F.avg_pool3d(e3, 2)))
    d3 = conv("dec3b", conv("dec3a", torch.cat([up(m4), e3], 1)))
    d2 = conv("dec2b", conv("dec2a", torch.cat([up(d3), e2], 1)))
    d1 = conv("dec1b", conv("dec1a", torch.cat([up(d2), e1], 1)))
    hw, hb = view("head")
    y = torch.einsum("ncdhw,c->ndhw", d1, hw) + hb[0]
    a = torch.from_numpy(active)
    d = (y - torch.from_numpy(target))[a]
    tl = (d * d).mean()
    tl.backward()
    assert abs(float(tl) - L) <= 1e-12 * L
    np.testing.assert_allclose(g, tp.grad.numpy(), rtol=1e-9, atol=1e-12 * np.abs(g).max())


def test_gradient_matches_finite_differences():
    params, x, active, target = _small_case(seed=5)
    _, g = U.loss_and_grad(params, x, active, target)
    lay, total = U.param_layout()
    rng = np.random.default_rng(9)
    checked = 0
    for name, (wo, bo, cin, co) in lay.items():
        for idx in (rng.integers(wo, bo), rng.integers(bo, bo + co)):
            eps = 1e-6
            p1 = params.copy()
            p1[idx] += eps
            p2 = params.copy()
            p2[idx] -= eps
            fd = (U.loss(p1, x, active, target) - U.loss(p2, x, active, target)) / (2 * eps)
            assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(g[idx])) + 1e-9, (name, idx, fd, g[idx])
            checked += 1
    assert checked == 2 * len(lay)


def test_adamw_first_step_closed_form():
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, wd, eps = 1e-3, 0.01, 1e-8
    p1, m, v = U.adamw(p, g, np.zeros(50), np.zeros(50), 1, lr, weight_decay=wd, eps=eps)
    # bias-corrected moments equal g and g^2 after one step
    np.testing.assert_allclose(p1, p * (1 - lr * wd) - lr * g / (np.abs(g) + eps), rtol=1e-13)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


def test_pack_input_stride_brute_force():
    rng = np.random.default_rng(6)
    mask = np.where(rng.random((8, 8, 8)) < 0.5, 1, -1).astype(np.int8)
    rho = rng.standard_normal((8, 8, 8))
    B = rng.standard_normal((8, 8, 8))
    x1, s = U.pack_input(rho, mask, B, 1)
    act = mask == 1
    assert abs(s - np.sqrt((rho[act] ** 2).mean())) < 1e-15
    assert np.array_equal(x1[0, ..., 0], np.where(act, rho / s, 0))
    assert np.array_equal(x1[0, ..., 1], mask.astype(float))
    assert np.allclose(x1[0, ..., 2], B / s) and not x1[0, ..., 3:].any()
    x2, _ = U.pack_input(rho, mask, B, 2)
    for z, y, xx in [(0, 0, 0), (3, 1, 2), (2, 3, 3)]:
        blk = (slice(2 * z, 2 * z + 2), slice(2 * y, 2 * y + 2), slice(2 * xx, 2 * xx + 2))
        c = act[blk].sum()
        want0 = rho[blk][act[blk]].sum() / c / s if c else 0.0
        assert abs(x2[0, z, y, xx, 0] - want0) < 1e-14
        assert x2[0, z, y, xx, 1] == (1.0 if 2 * c > 8 else -1.0)
        assert abs(x2[0, z, y, xx, 2] - B[blk].mean() / s) < 1e-14


def test_up2_linear_exact_for_linear_fields():
    n = 6
    ic = np.arange(n)
    # coarse cell centres at (ic + 1/2) * 2h, fine at (i + 1/2) * h
    c = (1.5 + 0.25 * ic[:, None, None] - 0.5 * ic[None, :, None] + 2.0 * ic[None, None, :]) * np.ones((n, n, n))
    f = U.up2_linear(c)
    i = np.arange(2 * n)
    xc = (i + 0.5) / 2 - 0.5  # fine centre in coarse index units
    want = 1.5 + 0.25 * xc[:, None, None] - 0.5 * xc[None, :, None] + 2.0 * xc[None, None, :]
    inner = slice(1, 2 * n - 1)
    np.testing.assert_allclose(f[inner, inner, inner], want[inner, inner, inner], rtol=1e-14, atol=1e-13)


def test_guess_shape_and_inactive_zero():
    params = U.init_params(1)
    rng = np.random.default_rng(7)
    mask = np.where(rng.random((16, 16, 16)) < 0.6, 1, -1).astype(np.int8)
    rho = rng.standard_normal((16, 16, 16))
    for stride in (1, 2):
        g = U.guess(params, rho, mask, None, stride)
        assert g.shape == mask.shape and not g[mask != 1].any() and np.isfinite(g).all()


def test_param_count():
    _, total = U.param_layout()
    assert total == 27 * 54272 + 704 + 17
