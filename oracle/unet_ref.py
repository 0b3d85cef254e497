"""Plain FP64 reference of the warm-start U-Net (forward, backward, loss, Adam).

TEST INFRASTRUCTURE ONLY: imported by the test suite and nothing else.  It
shares no code with the HIP network in ``paper_1609_09685_amd``.

Everything is NumPy float64 written from the definitions, one operation per
function, with the backward pass of each operation derived by hand:

* images are NHWC arrays ``[B, H, W, C]``;
* a convolution has taps t = (dy, dx) in row-major order over a ks x ks window
  centred on the pixel (ks = 3 with zero padding 1, or ks = 1), weights
  ``w[t, ci, co]`` and bias ``b[co]``:
      y[b, h, x, co] = b[co] + sum_t sum_ci  x[b, h + dy, x + dx, ci] w[t, ci, co]
  (dy, dx in {-1, 0, 1} for ks = 3; samples outside the image are zero);
* max pooling over 2 x 2 windows; its gradient goes to the first maximal
  element of the window in row-major order;
* nearest-neighbour upsampling by 2 (each value copied to a 2 x 2 block);
* ReLU after every 3 x 3 convolution, none after the 1 x 1 head;
* masked mean squared error over the fluid pixels and all output channels;
* Adam (Kingma & Ba 2015) with bias-corrected moments.

Network (the warm-start map from the solid mask and Kn to rho', u'): ``levels``
encoder levels with c_l = base * 2^l channels, two 3 x 3 convolutions each; a
2 x 2 max pool between levels; on the way up, upsample, concatenate
(upsampled channels first, then the skip of the same level), two 3 x 3
convolutions; a 1 x 1 head to ``out_ch`` channels.
"""
import numpy as np


# ------------------------------------------------------------------ layers

def conv_taps(ks):
    r = ks // 2
    return [(dy, dx) for dy in range(-r, r + 1) for dx in range(-r, r + 1)]


def shifted(x, dy, dx):
    """s[b, h, x] = x[b, h + dy, x + dx] (zero outside)."""
    B, H, W, C = x.shape
    s = np.zeros_like(x)
    h0, h1 = max(0, -dy), min(H, H - dy)
    w0, w1 = max(0, -dx), min(W, W - dx)
    if h0 < h1 and w0 < w1:
        s[:, h0:h1, w0:w1] = x[:, h0 + dy:h1 + dy, w0 + dx:w1 + dx]
    return s


def conv_fwd(x, w, b, ks):
    y = np.zeros(x.shape[:3] + (w.shape[2],))
    for t, (dy, dx) in enumerate(conv_taps(ks)):
        y += shifted(x, dy, dx) @ w[t]
    return y + b


def conv_bwd(x, w, dy_out, ks):
    """Gradients (dx, dw, db) of conv_fwd for the output gradient dy_out."""
    dw = np.zeros_like(w)
    dx = np.zeros_like(x)
    for t, (dy, dxx) in enumerate(conv_taps(ks)):
        xs = shifted(x, dy, dxx)
        dw[t] = np.einsum("bhwi,bhwo->io", xs, dy_out)
        # y(p) uses x(p + d): the gradient of x(q) collects dy_out(q - d)
        dx += shifted(dy_out @ w[t].T, -dy, -dxx)
    db = dy_out.sum(axis=(0, 1, 2))
    return dx, dw, db


def relu_fwd(x):
    return np.maximum(x, 0.0)


def relu_bwd(y, dy):
    """Gradient through ReLU given its output y (zero where y <= 0)."""
    return np.where(y > 0.0, dy, 0.0)


def pool_fwd(x):
    B, H, W, C = x.shape
    v = x.reshape(B, H // 2, 2, W // 2, 2, C)
    return v.max(axis=(2, 4))


def pool_bwd(x, dy):
    B, H, W, C = x.shape
    dx = np.zeros_like(x)
    taken = np.zeros((B, H // 2, W // 2, C), bool)
    for a in range(2):            # row-major order inside the window
        for c in range(2):
            xv = x[:, a::2, c::2]
            first = (xv == pool_fwd(x)) & ~taken
            dx[:, a::2, c::2] = np.where(first, dy, 0.0)
            taken |= first
    return dx


def up_fwd(x):
    return x.repeat(2, axis=1).repeat(2, axis=2)


def up_bwd(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def masked_mse(pred, target, fluid):
    """Loss and its gradient.  fluid: [B, H, W] (1 = counted)."""
    m = fluid.astype(np.float64)[..., None]
    n = m.sum() * pred.shape[-1]
    d = (pred - target) * m
    return float((d * d).sum() / n), 2.0 * d / n


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t >= 1 is the step number); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ network

def layer_shapes(levels=4, base=32, in_ch=2, out_ch=3):
    """[(name, ks, cin, cout)] in parameter order."""
    ch = [base * 2 ** l for l in range(levels)]
    out = []
    cin = in_ch
    for l in range(levels):
        out += [(f"enc{l}a", 3, cin, ch[l]), (f"enc{l}b", 3, ch[l], ch[l])]
        cin = ch[l]
    for l in range(levels - 2, -1, -1):
        out += [(f"dec{l}a", 3, ch[l + 1] + ch[l], ch[l]), (f"dec{l}b", 3, ch[l], ch[l])]
    out.append(("head", 1, ch[0], out_ch))
    return out


def param_count(**cfg):
    return sum(ks * ks * ci * co + co for _, ks, ci, co in layer_shapes(**cfg))


def unpack(params, **cfg):
    """Flat parameter vector -> {name: (w [taps, cin, cout], b [cout])}, packed
    layer by layer as w then b."""
    out, o = {}, 0
    for name, ks, ci, co in layer_shapes(**cfg):
        n = ks * ks * ci * co
        out[name] = (params[o:o + n].reshape(ks * ks, ci, co), params[o + n:o + n + co])
        o += n + co
    assert o == params.size
    return out


def pack(grads, **cfg):
    return np.concatenate([np.concatenate([grads[name][0].ravel(), grads[name][1].ravel()])
                           for name, _, _, _ in layer_shapes(**cfg)])


def forward(params, x, levels=4, base=32, in_ch=2, out_ch=3):
    """Network output and the activations the backward pass needs."""
    cfg = dict(levels=levels, base=base, in_ch=in_ch, out_ch=out_ch)
    P = unpack(params, **cfg)
    cache = {"x": x}
    h = x
    for l in range(levels):
        if l > 0:
            cache[f"pin{l}"] = h
            h = pool_fwd(h)
        cache[f"enc{l}a_in"] = h
        h = relu_fwd(conv_fwd(h, *P[f"enc{l}a"], 3))
        cache[f"enc{l}a_out"] = h
        h = relu_fwd(conv_fwd(h, *P[f"enc{l}b"], 3))
        cache[f"enc{l}b_out"] = h
    for l in range(levels - 2, -1, -1):
        u = up_fwd(h)
        cat = np.concatenate([u, cache[f"enc{l}b_out"]], axis=-1)
        cache[f"dec{l}a_in"] = cat
        h = relu_fwd(conv_fwd(cat, *P[f"dec{l}a"], 3))
        cache[f"dec{l}a_out"] = h
        h = relu_fwd(conv_fwd(h, *P[f"dec{l}b"], 3))
        cache[f"dec{l}b_out"] = h
    cache["head_in"] = h
    y = conv_fwd(h, *P["head"], 1)
    return y, cache


def backward(params, cache, dy, levels=4, base=32, in_ch=2, out_ch=3):
    """Gradients (flat parameter vector, input) for the output gradient dy,
    taking the forward operations in reverse order."""
    cfg = dict(levels=levels, base=base, in_ch=in_ch, out_ch=out_ch)
    P = unpack(params, **cfg)
    ch = [base * 2 ** l for l in range(levels)]
    return _backward_ordered(P, cache, dy, levels, ch, cfg)


def _backward_ordered(P, cache, dy, levels, ch, cfg):
    G = {}
    g, dw, db = conv_bwd(cache["head_in"], P["head"][0], dy, 1)
    G["head"] = (dw, db)
    skip = {}
    # decoders, top (level 0) to bottom (level levels - 2)
    for l in range(0, levels - 1):
        g = relu_bwd(cache[f"dec{l}b_out"], g)
        g, dw, db = conv_bwd(cache[f"dec{l}a_out"], P[f"dec{l}b"][0], g, 3)
        G[f"dec{l}b"] = (dw, db)
        g = relu_bwd(cache[f"dec{l}a_out"], g)
        g, dw, db = conv_bwd(cache[f"dec{l}a_in"], P[f"dec{l}a"][0], g, 3)
        G[f"dec{l}a"] = (dw, db)
        skip[l] = g[..., ch[l + 1]:]
        g = up_bwd(g[..., :ch[l + 1]])     # gradient of the output of the level below
    # encoders, bottom to top; the output of level l (< levels - 1) also feeds
    # the decoder of level l as its skip
    for l in range(levels - 1, -1, -1):
        if l < levels - 1:
            g = g + skip[l]
        g = relu_bwd(cache[f"enc{l}b_out"], g)
        g, dw, db = conv_bwd(cache[f"enc{l}a_out"], P[f"enc{l}b"][0], g, 3)
        G[f"enc{l}b"] = (dw, db)
        g = relu_bwd(cache[f"enc{l}a_out"], g)
        g, dw, db = conv_bwd(cache[f"enc{l}a_in"], P[f"enc{l}a"][0], g, 3)
        G[f"enc{l}a"] = (dw, db)
        if l > 0:
            g = pool_bwd(cache[f"pin{l}"], g)
    return pack(G, **cfg), g


def init_params(seed, **cfg):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, from a seeded
    NumPy generator: the random numbers that both sides start from."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ks, ci, co in layer_shapes(**cfg):
        parts.append(rng.standard_normal(ks * ks * ci * co) * np.sqrt(2.0 / (ks * ks * ci)))
        parts.append(np.zeros(co))
    return np.concatenate(parts)
