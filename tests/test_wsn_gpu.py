"""GPU parity of the warm-start network kernels against the FP64 U-Net reference.

Every layer is called through the C ABI on seeded random inputs and compared
with oracle/unet_ref.py evaluated in FP64 on the same (FP32-rounded) values.
Bar: normalised L2 error ||gpu - ref|| / ||ref|| <= 2e-5 per single layer
output (FP32 accumulation over at most 9 x 384 products) and <= 1e-4 per
gradient tensor of the whole network (whose ReLU masks and pooling choices are
taken from the kernels' FP32 forward values on both sides, after checking that
any choice that differs from the FP64 forward sits within FP32 rounding of its
threshold); pooling, upsampling, concatenation and
the ReLU gradient move values without arithmetic and must match exactly (the
2 x 2 sums of the upsampling gradient to FP32 rounding).
"""
import numpy as np
import pytest
import torch

from oracle import unet_ref as U
from paper_1609_09685_amd import wsn

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(7)
LAYER_TOL = 2e-5
NET_TOL = 1e-4


def dev(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def nl2(gpu, ref):
    g = gpu.detach().double().cpu().numpy() if torch.is_tensor(gpu) else np.asarray(gpu)
    return float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300))


CONV_CASES = [
    # B, H, W, cin, cout, ks
    (2, 8, 64, 2, 32, 3),       # first layer: 2 input channels
    (2, 8, 64, 3, 32, 3),       # first layer with the resistance profile
    (1, 5, 16, 32, 32, 3),      # ragged tile rows (th = 4), narrow width
    (2, 6, 32, 64, 64, 3),      # th = 2 tiles
    (1, 4, 128, 96, 32, 3),     # decoder-level concatenation width
    (1, 2, 32, 384, 128, 3),    # widest K
    (1, 3, 48, 20, 40, 3),      # channels not multiples of the tiles
    (2, 4, 64, 32, 3, 1),       # 1x1 head
    (1, 2, 16, 256, 256, 3),    # bottom level
    (1, 2, 32, 768, 256, 3),    # a fifth level's decoder input (512 + 256 channels)
]


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_forward(case):
    B, H, W, ci, co, ks = case
    x = f32(RNG.standard_normal((B, H, W, ci)))
    w = f32(RNG.standard_normal((ks * ks, ci, co)) / np.sqrt(ks * ks * ci))
    b = f32(RNG.standard_normal(co))
    ref = U.conv_fwd(x, w, b, ks)
    y = wsn.conv_forward(dev(x), dev(w), dev(b), ks, relu=False)
    assert nl2(y, ref) <= LAYER_TOL
    yr = wsn.conv_forward(dev(x), dev(w), dev(b), ks, relu=True)
    assert nl2(yr, U.relu_fwd(ref)) <= LAYER_TOL
    assert (yr.cpu().numpy() >= 0).all()


@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_backward(case):
    B, H, W, ci, co, ks = case
    x = f32(RNG.standard_normal((B, H, W, ci)))
    w = f32(RNG.standard_normal((ks * ks, ci, co)) / np.sqrt(ks * ks * ci))
    g = f32(RNG.standard_normal((B, H, W, co)))
    dx, dw, db = U.conv_bwd(x, w, g, ks)
    assert nl2(wsn.conv_backward_data(dev(g), dev(w), ks), dx) <= LAYER_TOL
    gw, gb = wsn.conv_backward_weight(dev(x), dev(g), ks)
    assert nl2(gw, dw) <= LAYER_TOL
    assert nl2(gb, db) <= LAYER_TOL


def test_conv_weight_grad_many_pixels():
    """Split-K over many pixel ranges (several splits per layer) and ragged end."""
    B, H, W, ci, co = 3, 40, 128, 32, 64
    x = f32(RNG.standard_normal((B, H, W, ci)))
    g = f32(RNG.standard_normal((B, H, W, co)))
    _, dw, db = U.conv_bwd(x, np.zeros((9, ci, co)), g, 3)
    gw, gb = wsn.conv_backward_weight(dev(x), dev(g), 3)
    assert nl2(gw, dw) <= LAYER_TOL and nl2(gb, db) <= LAYER_TOL
    # deterministic: a second call gives the same bits
    gw2, gb2 = wsn.conv_backward_weight(dev(x), dev(g), 3)
    assert torch.equal(gw, gw2) and torch.equal(gb, gb2)


def test_pool_relu_upcat():
    x = RNG.standard_normal((2, 8, 32, 5))
    x = np.maximum(x, 0.0)                       # ReLU outputs: many exact ties at 0
    x[0, 0, 0, 0] = x[0, 0, 1, 0] = 2.5          # a tie between nonzero values
    x = f32(x)
    y = wsn.pool_forward(dev(x))
    assert np.array_equal(y.cpu().numpy(), U.pool_fwd(x).astype(np.float32))
    gy = f32(RNG.standard_normal((2, 4, 16, 5)))
    add = f32(RNG.standard_normal(x.shape))
    ref = U.pool_bwd(x, gy)
    assert np.array_equal(wsn.pool_backward(dev(x), dev(gy)).cpu().numpy(), ref.astype(np.float32))
    assert np.allclose(wsn.pool_backward(dev(x), dev(gy), dev(add)).cpu().numpy(), ref + add,
                       rtol=1e-6, atol=1e-6)
    g = f32(RNG.standard_normal(x.shape))
    gt = dev(g)
    wsn.relu_backward(dev(x), gt)
    assert np.array_equal(gt.cpu().numpy(), U.relu_bwd(x, g).astype(np.float32))
    deep = f32(RNG.standard_normal((2, 4, 16, 6)))
    cat = wsn.upcat_forward(dev(deep), dev(x))
    assert np.array_equal(cat.cpu().numpy(),
                          np.concatenate([U.up_fwd(deep), x], -1).astype(np.float32))
    gc = f32(RNG.standard_normal((2, 8, 32, 11)))
    gd, gs = wsn.upcat_backward(dev(gc), 6)
    assert np.allclose(gd.cpu().numpy(), U.up_bwd(gc[..., :6]), rtol=1e-6, atol=1e-6)
    assert np.array_equal(gs.cpu().numpy(), gc[..., 6:].astype(np.float32))


def test_masked_mse_and_adam():
    pred = f32(RNG.standard_normal((2, 16, 32, 3)))
    tgt = f32(RNG.standard_normal((2, 16, 32, 3)))
    solid = (RNG.random((2, 16, 32)) < 0.3).astype(np.uint8)
    loss_ref, g_ref = U.masked_mse(pred, tgt, 1 - solid)
    loss, g = wsn.masked_mse(dev(pred), dev(tgt), torch.tensor(solid, device="cuda"))
    assert abs(loss.item() - loss_ref) <= 1e-12 * loss_ref
    assert nl2(g, g_ref) <= 1e-6
    assert (g.cpu().numpy()[solid.astype(bool)] == 0).all()
    n = 1000
    p, gg = f32(RNG.standard_normal(n)), f32(RNG.standard_normal(n))
    m, v = np.zeros(n), np.zeros(n)
    pt, mt, vt = dev(p), dev(m), dev(v)
    for t in range(1, 4):
        p, m, v = U.adam(p, gg, m, v, t, 1e-3)
        wsn.adam(pt, dev(gg), mt, vt, t, 1e-3)
        gg = f32(RNG.standard_normal(n))
    assert np.allclose(pt.cpu().numpy(), p, rtol=0, atol=1e-6)
    assert nl2(mt, m) <= 1e-6 and nl2(vt, v) <= 1e-6


NETS = [dict(levels=3, base=8, height=32, width=64, batch=2),
        dict(levels=4, base=32, height=128, width=256, batch=1)]


def _gpu_forward_cache(p, x, cfg):
    """The network's forward pass through the single-layer entry points (the
    same kernels and launches as wsn_forward), as a reference-style cache."""
    P = U.unpack(p, **cfg)

    def conv(h, name, ks, relu):
        w, b = P[name]
        return wsn.conv_forward(h, dev(w), dev(b), ks, relu)

    c = {"x": x}
    h = dev(x)
    for l in range(cfg["levels"]):
        if l > 0:
            c[f"pin{l}"] = h
            h = wsn.pool_forward(h)
        c[f"enc{l}a_in"] = h
        h = conv(h, f"enc{l}a", 3, True)
        c[f"enc{l}a_out"] = h
        h = conv(h, f"enc{l}b", 3, True)
        c[f"enc{l}b_out"] = h
    for l in range(cfg["levels"] - 2, -1, -1):
        cat = wsn.upcat_forward(h, c[f"enc{l}b_out"])
        c[f"dec{l}a_in"] = cat
        h = conv(cat, f"dec{l}a", 3, True)
        c[f"dec{l}a_out"] = h
        h = conv(h, f"dec{l}b", 3, True)
        c[f"dec{l}b_out"] = h
    c["head_in"] = h
    y = conv(h, "head", 1, False)
    return y, {k: (v.double().cpu().numpy() if torch.is_tensor(v) else v) for k, v in c.items()}


def _windows(e):
    B, H, W, C = e.shape
    return e.reshape(B, H // 2, 2, W // 2, 2, C).transpose(0, 1, 3, 5, 2, 4).reshape(-1, 4)


def _check_decisions(cache_gpu, cache_ref, cfg):
    """ReLU and pooling decisions may differ between the FP32 forward and the
    FP64 reference only where the reference value is within FP32 rounding of
    the decision threshold (1e-5 of the layer's RMS)."""
    flips = 0
    for k, r in cache_ref.items():
        if not k.endswith("_out"):
            continue
        g = cache_gpu[k]
        scale = np.sqrt((r ** 2).mean())
        d = (g > 0) != (r > 0)
        assert (np.maximum(np.abs(g), np.abs(r))[d] <= 1e-5 * scale).all(), k
        flips += int(d.sum())
    for l in range(1, cfg["levels"]):
        vr, vg = _windows(cache_ref[f"pin{l}"]), _windows(cache_gpu[f"pin{l}"])
        ar, ag = vr.argmax(1), vg.argmax(1)
        bad = np.nonzero(ar != ag)[0]
        scale = np.sqrt((vr ** 2).mean())
        top = np.sort(vr[bad], axis=1)
        assert (top[:, 3] - top[:, 2] <= 1e-5 * scale).all(), f"pool level {l}"
        flips += len(bad)
    return flips


@pytest.mark.parametrize("net", NETS, ids=["small", "warm_start_size"])
def test_network_forward_backward(net):
    cfg = dict(levels=net["levels"], base=net["base"], in_ch=2, out_ch=3)
    B, H, W = net["batch"], net["height"], net["width"]
    p = U.init_params(11, **cfg) + 0.01 * RNG.standard_normal(U.param_count(**cfg))
    p = f32(p)
    x = np.zeros((B, H, W, 2))
    x[..., 0] = RNG.random((B, H, W)) < 0.3
    x[..., 1] = RNG.uniform(0.1, 1.0, (B, 1, 1))
    tgt = f32(RNG.standard_normal((B, H, W, 3)))
    solid = x[..., 0].astype(np.uint8)
    y_ref, cache_ref = U.forward(p, x, **cfg)
    loss_ref, _ = U.masked_mse(y_ref, tgt, 1 - solid)

    n = wsn.WarmStartNet(p, B, height=H, width=W, **cfg)
    y = n.forward(dev(x))
    assert nl2(y, y_ref) <= NET_TOL
    loss, dy = wsn.masked_mse(y, dev(tgt), torch.tensor(solid, device="cuda"))
    assert abs(loss.item() - loss_ref) <= NET_TOL * loss_ref
    g = n.backward(dy).double().cpu().numpy()

    # the FP64 backward at the kernels' own forward state: same ReLU masks and
    # pooling choices on both sides
    y_layers, cache_gpu = _gpu_forward_cache(p, x, cfg)
    assert torch.equal(y_layers, y)          # the network ran exactly these launches
    flips = _check_decisions(cache_gpu, cache_ref, cfg)
    dy64 = dy.double().cpu().numpy()
    _, dy_ref = U.masked_mse(y.double().cpu().numpy(), tgt, 1 - solid)
    assert nl2(dy, dy_ref) <= 1e-6
    g_ref, _ = U.backward(p, cache_gpu, dy64, **cfg)
    o = 0
    worst = 0.0
    for name, ks, ci, co in U.layer_shapes(**cfg):
        for size in (ks * ks * ci * co, co):
            e = nl2(g[o:o + size], g_ref[o:o + size])
            worst = max(worst, e)
            assert e <= NET_TOL, (name, size, e)
            o += size
    print(f"{net}: worst gradient tensor error {worst:.2e}, decisions within rounding: {flips}")


def test_training_reduces_loss():
    cfg = dict(levels=3, base=8, in_ch=2, out_ch=3)
    B, H, W = 4, 32, 64
    x = np.zeros((B, H, W, 2), np.float32)
    x[..., 0] = RNG.random((B, H, W)) < 0.3
    x[..., 1] = 0.5
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    tgt = np.stack([np.broadcast_to((xx / W - 0.5), (B, H, W)),
                    np.broadcast_to(np.sin(yy / 5.0), (B, H, W)),
                    np.zeros((B, H, W))], -1).astype(np.float32)
    n = wsn.WarmStartNet(U.init_params(0, **cfg), B, height=H, width=W, **cfg)
    xs, ts = dev(x), dev(tgt)
    solid = torch.tensor(x[..., 0].astype(np.uint8), device="cuda")
    losses = [n.train_step(xs, ts, solid, 3e-3).item() for _ in range(60)]
    assert losses[-1] < 0.25 * losses[0], losses[::10]


def test_field_conversions():
    """Solver fields <-> network layout: the affine map with an x slope, the
    velocity mask, the non-finite flag and the input packing."""
    B, H, W = 3, 16, 32
    rho = f32(1.0 + 1e-3 * RNG.standard_normal((B, H, W)))
    u = f32(1e-4 * RNG.standard_normal((B, 2, H, W)))
    shift = f32(RNG.standard_normal((B, 3)))
    slope = f32(1e-3 * RNG.standard_normal((B, 3)))
    scale = f32(RNG.uniform(0.5, 2.0, (B, 3)))
    xp = np.arange(1, W + 1)[None, None, :]
    f = [rho, u[:, 0], u[:, 1]]
    ref = np.stack([(f[k] - shift[:, k, None, None] - slope[:, k, None, None] * xp)
                    * scale[:, k, None, None] for k in range(3)], -1)
    y = wsn.fields_to_nhwc(dev(rho), dev(u), dev(shift), dev(scale), slope=dev(slope))
    assert np.allclose(y.cpu().numpy(), ref, rtol=1e-5, atol=1e-6)
    keep = (RNG.random((B, H, W)) < 0.7).astype(np.uint8)
    yy = y.clone()
    yy[1, 3, 4, 2] = float("nan")
    r2, u2, bad = wsn.nhwc_to_fields(yy, dev(shift), dev(1.0 / scale), slope=dev(slope),
                                     keep_u=torch.tensor(keep, device="cuda"))
    assert bad.cpu().tolist() == [0, 1, 0]
    assert np.allclose(r2.cpu().numpy(), rho, rtol=0, atol=1e-5)
    u2 = u2.cpu().numpy()
    assert (u2[np.broadcast_to(keep[:, None] == 0, u.shape)] == 0).all()
    ok = np.broadcast_to(keep[:, None] == 1, u.shape).copy()
    ok[1, 1, 3, 4] = False                       # the planted NaN
    assert np.allclose(u2[ok], u[ok], rtol=0, atol=1e-6)
    solid = (RNG.random((B, H, W)) < 0.3).astype(np.uint8)
    feat = np.array([0.1, 0.5, 1.7], np.float32)
    x = wsn.pack_input(torch.tensor(solid, device="cuda"), dev(feat)).cpu().numpy()
    assert np.array_equal(x[..., 0], solid.astype(np.float32))
    assert np.array_equal(x[..., 1], np.broadcast_to(feat[:, None, None], (B, H, W)))


@pytest.mark.parametrize("fh,fw", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_mirror(fh, fw):
    """Mirror images of float NHWC images (with per-channel factors, and
    without, and added to an output) and of uint8 masks, against NumPy's flips
    (bitwise where no arithmetic is done), on odd sizes that leave a ragged
    last block."""
    def ref(a, scale=None):
        r = a[:, ::-1] if fh else a
        r = r[:, :, ::-1] if fw else r
        return r * np.asarray(scale, a.dtype) if scale is not None else r
    y = RNG.standard_normal((3, 17, 29, 3)).astype(np.float32)
    scale = (-1.0, 0.25, -0.5)
    out = wsn.mirror(dev(y), fh, fw, scale).cpu().numpy()
    assert np.array_equal(out, ref(y, scale))
    x = RNG.standard_normal((2, 5, 7, 2)).astype(np.float32)
    assert np.array_equal(wsn.mirror(dev(x), fh, fw).cpu().numpy(), ref(x))
    m = (RNG.random((4, 9, 33)) < 0.4).astype(np.uint8)
    got = wsn.mirror(torch.tensor(m, device="cuda"), fh, fw).cpu().numpy()
    assert np.array_equal(got, ref(m))
    pre = torch.full((3, 17, 29, 3), 7.0, device="cuda")
    assert wsn.mirror(dev(y), fh, fw, scale, out=pre) is pre
    assert np.array_equal(pre.cpu().numpy(), ref(y, scale))
    acc = dev(y)
    wsn.mirror(dev(y), fh, fw, scale, out=acc, accumulate=True)
    assert np.array_equal(acc.cpu().numpy(), y + ref(y, scale))
    acc = dev(x)
    wsn.mirror(dev(x), fh, fw, out=acc, accumulate=True)
    assert np.array_equal(acc.cpu().numpy(), x + ref(x))


def _profile_ref(solid):
    """The resistance profile of wsn_column_profile, in float64."""
    B, H, W = solid.shape
    phi = np.maximum((solid == 0).sum(axis=1) / H, 1.0 / H)
    r = (1.0 - phi + 1.0 / H) ** 2 / phi ** 3
    c = np.cumsum(r, axis=1) / r.sum(axis=1, keepdims=True)
    return (np.arange(W) + 1.0) / (W + 1) - c


@pytest.mark.parametrize("H,W", [(5, 37), (3, 300)])
def test_column_profile_and_packing(H, W):
    """The resistance profile against its formula (a fully solid column, a
    fully fluid one, widths below and above one block), and the three-channel
    input packing bitwise."""
    B = 3
    solid = (RNG.random((B, H, W)) < 0.4).astype(np.uint8)
    solid[0, :, 2] = 1
    solid[1, :, 5] = 0
    ts = torch.tensor(solid, device="cuda")
    prof = wsn.column_profile(ts).cpu().numpy()
    assert np.abs(prof - _profile_ref(solid)).max() <= 2e-5   # FP32 running sum
    feat = np.array([0.1, 0.5, 1.7], np.float32)
    x = wsn.pack_input(ts, dev(feat), profile=dev(prof), profile_scale=10.0).cpu().numpy()
    assert x.shape == (B, H, W, 3)
    assert np.array_equal(x[..., 0], solid.astype(np.float32))
    assert np.array_equal(x[..., 1], np.broadcast_to(feat[:, None, None], (B, H, W)))
    assert np.array_equal(x[..., 2], np.broadcast_to((np.float32(10.0) * prof)[:, None, :],
                                                     (B, H, W)))


@pytest.mark.parametrize("in_ch", [2, 3])
def test_augmented_training_views(in_ch):
    """The mirrored training data: the samples, then their three mirror images
    with the target factors of MIRRORS, bitwise against NumPy's flips, and
    inputs formed from the mirrored masks (the profile of an x-mirrored mask
    is its own, not the mirrored profile)."""
    from paper_1609_09685_amd import warmstart as ws
    n, H, W = 3, 8, 16
    y = RNG.standard_normal((n, H, W, 3)).astype(np.float32)
    solid = (RNG.random((n, H, W)) < 0.3).astype(np.uint8)
    taus = [0.6, 0.7, 0.9]
    ts = torch.tensor(solid, device="cuda")
    x = ws.inputs(ts, taus, in_ch)
    data = ws.Dataset(x, None, None, ts, taus, [0] * n, [0.0] * n, [True] * n, list(range(n)))
    xa, ya, sa = (t.cpu().numpy() for t in ws.augmented(data, dev(y)))
    assert xa.shape == (4 * n, H, W, in_ch) and ya.shape == (4 * n, H, W, 3)
    assert sa.shape == (4 * n, H, W)
    x = x.cpu().numpy()
    views = [((0, 0), (1.0, 1.0, 1.0))] + list(ws.MIRRORS)
    for v, ((fh, fw), sign) in enumerate(views):
        def flip(a):
            r = a[:, ::-1] if fh else a
            return r[:, :, ::-1] if fw else r
        blk = slice(v * n, (v + 1) * n)
        assert np.array_equal(sa[blk], flip(solid))
        assert np.array_equal(xa[blk][..., :2], flip(x)[..., :2])
        assert np.array_equal(ya[blk], flip(y) * np.asarray(sign, np.float32))
        if in_ch == 3:
            want = ws.PROFILE_SCALE * _profile_ref(flip(solid))
            assert np.abs(xa[blk][..., 2] - want[:, None, :]).max() <= 2e-4


@pytest.mark.parametrize("in_ch", [2, 3])
@pytest.mark.parametrize("fh,fw", [(1, 0), (0, 1), (1, 1)])
def test_averaged_prediction_is_mirror_equivariant(fh, fw, in_ch):
    """Averaged over the mirror images, the learned start of a mirrored mask is
    the mirrored start of the mask (density deviation from the linear drop and
    u_y with the factors of MIRRORS), for any weights: a flip or factor wrong
    anywhere in the averaging breaks it."""
    from paper_1609_09685_amd import warmstart as ws
    net = ws.new_network(2, seed=3, in_ch=in_ch)
    masks = [ws.sample(s)[0] for s in (20001, 20002)]
    taus = [0.6, 0.85]
    scales = (1.3, 0.2)

    def flip(a):
        r = a[..., ::-1, :] if fh else a
        return r[..., ::-1] if fw else r

    rho, u, bad = (t.cpu().numpy() for t in ws.predict(net, masks, taus, scales, tta=True))
    mm = [np.ascontiguousarray(flip(m)) for m in masks]
    rho2, u2, bad2 = (t.cpu().numpy() for t in ws.predict(net, mm, taus, scales, tta=True))
    assert not bad.any() and not bad2.any()
    lin = ws.RHO_IN + (ws.RHO_OUT - ws.RHO_IN) * (np.arange(ws.NX) + 1.0) / (ws.NX + 1)
    sign = dict(ws.MIRRORS)[(fh, fw)]
    drho = ws.RHO_IN - ws.RHO_OUT
    want_dev = sign[0] * flip(rho.astype(np.float64) - lin)
    assert np.abs((rho2 - lin) - want_dev).max() <= 1e-3 * drho
    for c in range(2):
        want = sign[1 + c] * flip(u[:, c])
        assert np.abs(u2[:, c] - want).max() <= 1e-5 * np.abs(u[:, c]).max()
