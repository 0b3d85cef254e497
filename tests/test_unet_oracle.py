"""Pins of the U-Net reference (oracle/unet_ref.py), on the CPU.

Each operation is checked against something other than itself: SciPy's 2-D
correlation, torch's FP64 CPU operators and autograd (library routines
independent of the HIP network), central finite differences, adjoint
identities, and closed forms (Adam's first step, hand-made pooling ties).
"""
import numpy as np
import pytest
import scipy.signal
import torch
import torch.nn.functional as F

from oracle import unet_ref as U

RNG = np.random.default_rng(20240611)


def _t(a, grad=False):
    return torch.tensor(a, dtype=torch.float64, requires_grad=grad)


def _torch_conv(x_nhwc, w, b, ks):
    ci, co = w.shape[1], w.shape[2]
    wt = w.reshape(ks, ks, ci, co).permute(3, 2, 0, 1)
    return F.conv2d(x_nhwc.permute(0, 3, 1, 2), wt, b, padding=ks // 2).permute(0, 2, 3, 1)


@pytest.mark.parametrize("ks", [1, 3])
def test_conv_fwd_against_scipy_correlate(ks):
    x = RNG.standard_normal((2, 5, 7, 3))
    w = RNG.standard_normal((ks * ks, 3, 4))
    b = RNG.standard_normal(4)
    y = U.conv_fwd(x, w, b, ks)
    for bi in range(2):
        for co in range(4):
            ref = np.full((5, 7), b[co])
            for ci in range(3):
                k = w[:, ci, co].reshape(ks, ks)
                ref += scipy.signal.correlate2d(x[bi, :, :, ci], k, mode="same")
            assert np.allclose(y[bi, :, :, co], ref, rtol=0, atol=1e-13)


@pytest.mark.parametrize("ks", [1, 3])
def test_conv_bwd_against_torch_autograd(ks):
    x = RNG.standard_normal((2, 6, 8, 5))
    w = RNG.standard_normal((ks * ks, 5, 3))
    b = RNG.standard_normal(3)
    g = RNG.standard_normal((2, 6, 8, 3))
    xt, wt, bt = _t(x, True), _t(w, True), _t(b, True)
    yt = _torch_conv(xt, wt, bt, ks)
    assert np.allclose(yt.detach().numpy(), U.conv_fwd(x, w, b, ks), atol=1e-13)
    (yt * _t(g)).sum().backward()
    dx, dw, db = U.conv_bwd(x, w, g, ks)
    assert np.allclose(dx, xt.grad.numpy(), atol=1e-12)
    assert np.allclose(dw, wt.grad.numpy(), atol=1e-12)
    assert np.allclose(db, bt.grad.numpy(), atol=1e-12)


def test_conv_bwd_finite_differences():
    x = RNG.standard_normal((1, 4, 5, 2))
    w = RNG.standard_normal((9, 2, 3))
    b = RNG.standard_normal(3)
    g = RNG.standard_normal((1, 4, 5, 3))
    loss = lambda x_, w_, b_: float((U.conv_fwd(x_, w_, b_, 3) * g).sum())
    dx, dw, db = U.conv_bwd(x, w, g, 3)
    h = 1e-6
    for arr, grad in ((x, dx), (w, dw), (b, db)):
        for idx in [tuple(RNG.integers(0, s) for s in arr.shape) for _ in range(6)]:
            p, m = arr.copy(), arr.copy()
            p[idx] += h
            m[idx] -= h
            args_p = [p if a is arr else a for a in (x, w, b)]
            args_m = [m if a is arr else a for a in (x, w, b)]
            fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
            assert abs(fd - grad[idx]) <= 1e-7 * max(1.0, abs(fd))


def test_pool_against_torch_without_ties():
    x = RNG.standard_normal((2, 6, 8, 3))
    g = RNG.standard_normal((2, 3, 4, 3))
    xt = _t(x, True)
    yt = F.max_pool2d(xt.permute(0, 3, 1, 2), 2).permute(0, 2, 3, 1)
    assert np.array_equal(yt.detach().numpy(), U.pool_fwd(x))
    (yt * _t(g)).sum().backward()
    assert np.array_equal(xt.grad.numpy(), U.pool_bwd(x, g))


def test_pool_tie_rule_first_in_row_major_order():
    x = np.zeros((1, 2, 4, 1))
    x[0, :, 2:, 0] = [[1.0, 3.0], [3.0, 3.0]]    # second window: ties at (0,1), (1,0), (1,1)
    g = np.array([[[[5.0], [7.0]]]])
    dx = U.pool_bwd(x, g)
    # first window all zero: (0, 0) takes the gradient; second: (0, 1) of the window
    assert dx[0, 0, 0, 0] == 5.0 and dx[0, :, :2, 0].sum() == 5.0
    assert dx[0, 0, 3, 0] == 7.0 and dx[0, :, 2:, 0].sum() == 7.0


def test_upsample_against_torch_and_adjoint():
    x = RNG.standard_normal((2, 3, 4, 5))
    xt = _t(x)
    ref = F.interpolate(xt.permute(0, 3, 1, 2), scale_factor=2, mode="nearest").permute(0, 2, 3, 1)
    assert np.array_equal(ref.numpy(), U.up_fwd(x))
    y = RNG.standard_normal((2, 6, 8, 5))
    assert np.isclose((U.up_fwd(x) * y).sum(), (x * U.up_bwd(y)).sum(), rtol=1e-13)


def test_relu_bwd_uses_output_sign():
    y = np.array([0.0, 2.0, 0.0, 1e-300])
    assert np.array_equal(U.relu_bwd(y, np.ones(4)), [0.0, 1.0, 0.0, 1.0])


def test_masked_mse_closed_form_and_gradient():
    pred = RNG.standard_normal((2, 3, 4, 3))
    tgt = RNG.standard_normal((2, 3, 4, 3))
    fluid = RNG.integers(0, 2, (2, 3, 4))
    loss, g = U.masked_mse(pred, tgt, fluid)
    sel = fluid.astype(bool)
    assert np.isclose(loss, ((pred - tgt)[sel] ** 2).mean(), rtol=1e-14)
    assert np.all(g[~sel] == 0)
    pt = _t(pred, True)
    m = _t(fluid.astype(float))[..., None]
    l_t = (((pt - _t(tgt)) * m) ** 2).sum() / (m.sum() * 3)
    l_t.backward()
    assert np.allclose(g, pt.grad.numpy(), atol=1e-15)


def test_adam_first_steps_closed_form():
    p = RNG.standard_normal(7)
    g1 = RNG.standard_normal(7)
    lr, eps = 1e-3, 1e-8
    p1, m1, v1 = U.adam(p, g1, np.zeros(7), np.zeros(7), 1, lr, eps=eps)
    # bias correction makes the first moments exactly g and g^2
    assert np.allclose(p1, p - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    g2 = RNG.standard_normal(7)
    p2, _, _ = U.adam(p1, g2, m1, v1, 2, lr, eps=eps)
    mh = (0.9 * 0.1 * g1 + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    assert np.allclose(p2, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=1e-12, atol=0)
    # against torch's Adam
    pt = _t(p, True)
    opt = torch.optim.Adam([pt], lr=lr, eps=eps)
    for g in (g1, g2):
        pt.grad = _t(g)
        opt.step()
    assert np.allclose(pt.detach().numpy(), p2, rtol=1e-12, atol=1e-15)


def _torch_unet(params, x, levels, base, in_ch, out_ch):
    cfg = dict(levels=levels, base=base, in_ch=in_ch, out_ch=out_ch)
    P = U.unpack(params, **cfg)
    T = {k: (_t(w, True), _t(b, True)) for k, (w, b) in P.items()}
    xt = _t(x, True)
    h = xt
    skips = {}
    for l in range(levels):
        if l > 0:
            h = F.max_pool2d(h.permute(0, 3, 1, 2), 2).permute(0, 2, 3, 1)
        h = F.relu(_torch_conv(h, *T[f"enc{l}a"], 3))
        h = F.relu(_torch_conv(h, *T[f"enc{l}b"], 3))
        skips[l] = h
    for l in range(levels - 2, -1, -1):
        u = F.interpolate(h.permute(0, 3, 1, 2), scale_factor=2, mode="nearest").permute(0, 2, 3, 1)
        h = torch.cat([u, skips[l]], dim=-1)
        h = F.relu(_torch_conv(h, *T[f"dec{l}a"], 3))
        h = F.relu(_torch_conv(h, *T[f"dec{l}b"], 3))
    return _torch_conv(h, *T["head"], 1), T, xt


@pytest.mark.parametrize("cfg", [dict(levels=3, base=4, in_ch=2, out_ch=3),
                                 dict(levels=4, base=2, in_ch=2, out_ch=3)])
def test_unet_against_torch_autograd(cfg):
    p = U.init_params(3, **cfg)
    p += 0.01 * RNG.standard_normal(p.size)        # nonzero biases
    x = RNG.standard_normal((2, 16, 24, 2))
    y, cache = U.forward(p, x, **cfg)
    g = RNG.standard_normal(y.shape)
    yt, T, xt = _torch_unet(p, x, **cfg)
    assert np.allclose(yt.detach().numpy(), y, atol=1e-12)
    (yt * _t(g)).sum().backward()
    gt = np.concatenate([np.concatenate([T[n][0].grad.numpy().ravel(), T[n][1].grad.numpy().ravel()])
                         for n, _, _, _ in U.layer_shapes(**cfg)])
    gp, gx = U.backward(p, cache, g, **cfg)
    assert np.allclose(gp, gt, rtol=0, atol=1e-12 * np.abs(gt).max())
    assert np.allclose(gx, xt.grad.numpy(), atol=1e-12)


def test_unet_finite_differences():
    cfg = dict(levels=2, base=2, in_ch=2, out_ch=3)
    p = U.init_params(5, **cfg) + 0.05 * RNG.standard_normal(U.param_count(**cfg))
    x = RNG.standard_normal((1, 4, 8, 2))
    tgt = RNG.standard_normal((1, 4, 8, 3))
    fluid = RNG.integers(0, 2, (1, 4, 8))

    def loss(pp):
        y, _ = U.forward(pp, x, **cfg)
        return U.masked_mse(y, tgt, fluid)[0]

    y, cache = U.forward(p, x, **cfg)
    _, dy = U.masked_mse(y, tgt, fluid)
    gp, _ = U.backward(p, cache, dy, **cfg)
    h = 1e-6
    for i in RNG.choice(p.size, 25, replace=False):
        e = np.zeros_like(p)
        e[i] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - gp[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, gp[i])


def test_layer_table_of_the_warm_start_network():
    shapes = U.layer_shapes()
    assert [s[0] for s in shapes] == ["enc0a", "enc0b", "enc1a", "enc1b", "enc2a", "enc2b",
                                      "enc3a", "enc3b", "dec2a", "dec2b", "dec1a", "dec1b",
                                      "dec0a", "dec0b", "head"]
    assert shapes[8][2:] == (384, 128) and shapes[12][2:] == (96, 32) and shapes[14] == ("head", 1, 32, 3)
    # 9 x 216128 conv weights + 96 head weights + 1411 biases
    assert U.param_count() == 9 * 216128 + 96 + 1411 == 1946659
