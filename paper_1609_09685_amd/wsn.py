"""Python binding of the warm-start network ABI in ``include/wsn.h``.

Argument marshalling only: every layer, the loss and the optimiser run in the
HIP library; torch allocates the buffers the library asks for and supplies the
stream.  ``WarmStartNet`` holds one network (parameters, Adam moments) and the
activation / work buffers of one batch size.
"""
import ctypes

import numpy as np

from . import lbm
from .lbm import _check, load_library

_c = ctypes
_p = _c.c_void_p
_i = _c.c_int32


class Config(ctypes.Structure):
    _fields_ = [("levels", _i), ("base", _i), ("in_ch", _i), ("out_ch", _i), ("height", _i),
                ("width", _i)]


# name -> (restype, argtypes) for every entry point of include/wsn.h
_SIGS = {
    "wsn_query_sizes": (_c.c_int, [_c.POINTER(Config), _i, _c.POINTER(_c.c_int64),
                                   _c.POINTER(_c.c_size_t), _c.POINTER(_c.c_size_t)]),
    "wsn_forward": (_c.c_int, [_c.POINTER(Config), _i, _p, _p, _p, _p, _p]),
    "wsn_backward": (_c.c_int, [_c.POINTER(Config), _i, _p, _p, _p, _p, _p, _p, _p]),
    "wsn_mse_work": (_c.c_int, [_c.c_int64, _c.POINTER(_c.c_size_t)]),
    "wsn_masked_mse": (_c.c_int, [_p, _p, _p, _c.c_int64, _i, _p, _p, _p, _c.c_size_t, _p]),
    "wsn_adam": (_c.c_int, [_p, _p, _p, _p, _c.c_int64, _c.c_double, _c.c_double, _c.c_double,
                            _c.c_double, _c.c_int64, _p]),
    "wsn_conv_forward": (_c.c_int, [_p, _p, _p, _p, _i, _i, _i, _i, _i, _i, _i, _p]),
    "wsn_conv_backward_data": (_c.c_int, [_p, _p, _p, _p, _i, _i, _i, _i, _i, _i, _p]),
    "wsn_conv_wgrad_work": (_c.c_int, [_i, _i, _i, _i, _i, _i, _c.POINTER(_c.c_size_t)]),
    "wsn_conv_backward_weight": (_c.c_int, [_p, _p, _p, _p, _i, _i, _i, _i, _i, _i, _p,
                                            _c.c_size_t, _p]),
    "wsn_relu_backward": (_c.c_int, [_p, _p, _c.c_int64, _p]),
    "wsn_pool_forward": (_c.c_int, [_p, _p, _i, _i, _i, _i, _p]),
    "wsn_pool_backward": (_c.c_int, [_p, _p, _p, _p, _i, _i, _i, _i, _p]),
    "wsn_upcat_forward": (_c.c_int, [_p, _p, _p, _i, _i, _i, _i, _i, _p]),
    "wsn_upcat_backward": (_c.c_int, [_p, _p, _p, _i, _i, _i, _i, _i, _p]),
    "wsn_pack_input": (_c.c_int, [_p, _p, _i, _i, _i, _p, _p]),
    "wsn_fields_to_nhwc": (_c.c_int, [_p, _p, _p, _p, _p, _i, _i, _i, _p, _p]),
    "wsn_nhwc_to_fields": (_c.c_int, [_p, _p, _p, _p, _p, _i, _i, _i, _p, _p, _p, _p]),
    "wsn_column_profile": (_c.c_int, [_p, _i, _i, _i, _p, _p]),
    "wsn_pack_input_profile": (_c.c_int, [_p, _p, _p, _c.c_float, _i, _i, _i, _p, _p]),
    "wsn_mirror": (_c.c_int, [_p, _i, _i, _i, _i, _i, _i, _i, _c.POINTER(_c.c_float), _i, _p,
                              _p]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = load_library()
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(device=None):
    import torch
    return torch.cuda.current_stream(device).cuda_stream


def _f32(t):
    import torch
    if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("expected a contiguous float32 device tensor")
    return t


# ---------------------------------------------------------------- single layers

def conv_forward(x, w, b, ks, relu=False):
    """x [B,H,W,cin], w [ks*ks, cin, cout], b [cout] or None -> y [B,H,W,cout]."""
    import torch
    B, H, W, ci = x.shape
    co = w.shape[2]
    y = torch.empty((B, H, W, co), dtype=torch.float32, device=x.device)
    _check(lib().wsn_conv_forward(_ptr(_f32(x)), _ptr(_f32(w)), _ptr(b), _ptr(y), B, H, W, ci, co,
                                  ks, 1 if relu else 0, _stream(x.device)))
    return y


def conv_backward_data(dy, w, ks):
    import torch
    B, H, W, co = dy.shape
    ci = w.shape[1]
    dx = torch.empty((B, H, W, ci), dtype=torch.float32, device=dy.device)
    wflip = torch.empty(w.numel(), dtype=torch.float32, device=dy.device)
    _check(lib().wsn_conv_backward_data(_ptr(_f32(dy)), _ptr(_f32(w)), _ptr(dx), _ptr(wflip), B, H,
                                        W, ci, co, ks, _stream(dy.device)))
    return dx


def conv_backward_weight(x, dy, ks, bias=True):
    import torch
    B, H, W, ci = x.shape
    co = dy.shape[3]
    n = ctypes.c_size_t(0)
    _check(lib().wsn_conv_wgrad_work(B, H, W, ci, co, ks, ctypes.byref(n)))
    work = torch.empty(n.value, dtype=torch.uint8, device=x.device)
    dw = torch.empty((ks * ks, ci, co), dtype=torch.float32, device=x.device)
    db = torch.empty(co, dtype=torch.float32, device=x.device) if bias else None
    _check(lib().wsn_conv_backward_weight(_ptr(_f32(x)), _ptr(_f32(dy)), _ptr(dw), _ptr(db), B, H,
                                          W, ci, co, ks, _ptr(work), n.value, _stream(x.device)))
    return dw, db


def relu_backward(y, g):
    """In place: g = (y > 0) ? g : 0."""
    _check(lib().wsn_relu_backward(_ptr(_f32(y)), _ptr(_f32(g)), g.numel(), _stream(g.device)))
    return g


def pool_forward(x):
    import torch
    B, H, W, C = x.shape
    y = torch.empty((B, H // 2, W // 2, C), dtype=torch.float32, device=x.device)
    _check(lib().wsn_pool_forward(_ptr(_f32(x)), _ptr(y), B, H, W, C, _stream(x.device)))
    return y


def pool_backward(x, gy, add=None):
    import torch
    B, H, W, C = x.shape
    gx = torch.empty_like(x)
    _check(lib().wsn_pool_backward(_ptr(_f32(x)), _ptr(_f32(gy)), _ptr(add), _ptr(gx), B, H, W, C,
                                   _stream(x.device)))
    return gx


def upcat_forward(deep, skip):
    import torch
    B, H, W, c2 = skip.shape
    c1 = deep.shape[3]
    cat = torch.empty((B, H, W, c1 + c2), dtype=torch.float32, device=skip.device)
    _check(lib().wsn_upcat_forward(_ptr(_f32(deep)), _ptr(_f32(skip)), _ptr(cat), B, H, W, c1, c2,
                                   _stream(skip.device)))
    return cat


def upcat_backward(gcat, c1):
    import torch
    B, H, W, C = gcat.shape
    c2 = C - c1
    gdeep = torch.empty((B, H // 2, W // 2, c1), dtype=torch.float32, device=gcat.device)
    gskip = torch.empty((B, H, W, c2), dtype=torch.float32, device=gcat.device)
    _check(lib().wsn_upcat_backward(_ptr(_f32(gcat)), _ptr(gdeep), _ptr(gskip), B, H, W, c1, c2,
                                    _stream(gcat.device)))
    return gdeep, gskip


def masked_mse(pred, target, solid):
    """(loss as a 0-d float64 device tensor, gradient) over pixels with solid == 0."""
    import torch
    C = pred.shape[-1]
    npix = pred.numel() // C
    n = ctypes.c_size_t(0)
    _check(lib().wsn_mse_work(npix, ctypes.byref(n)))
    work = torch.empty(n.value, dtype=torch.uint8, device=pred.device)
    loss = torch.empty((), dtype=torch.float64, device=pred.device)
    grad = torch.empty_like(pred)
    if solid.dtype != torch.uint8 or not solid.is_contiguous():
        raise ValueError("solid must be a contiguous uint8 tensor")
    _check(lib().wsn_masked_mse(_ptr(_f32(pred)), _ptr(_f32(target)), _ptr(solid), npix, C,
                                _ptr(loss), _ptr(grad), _ptr(work), n.value, _stream(pred.device)))
    return loss, grad


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    _check(lib().wsn_adam(_ptr(_f32(p)), _ptr(_f32(g)), _ptr(_f32(m)), _ptr(_f32(v)), p.numel(),
                          float(lr), float(b1), float(b2), float(eps), int(t), _stream(p.device)))


def pack_input(solid, feat, out=None, profile=None, profile_scale=1.0):
    """solid uint8 [B,H,W], feat float32 [B] -> x [B,H,W,2], or [B,H,W,3] with
    profile float32 [B,W] (times profile_scale) as the third channel (into
    `out` if given)."""
    import torch
    B, H, W = solid.shape
    C = 2 if profile is None else 3
    x = out if out is not None else torch.empty((B, H, W, C), dtype=torch.float32,
                                                device=solid.device)
    if tuple(x.shape) != (B, H, W, C):
        raise ValueError("out has the wrong shape")
    if profile is None:
        _check(lib().wsn_pack_input(_ptr(solid), _ptr(_f32(feat)), B, H, W, _ptr(x),
                                    _stream(solid.device)))
    else:
        if tuple(profile.shape) != (B, W):
            raise ValueError("profile must be [B,W]")
        _check(lib().wsn_pack_input_profile(_ptr(solid), _ptr(_f32(feat)), _ptr(_f32(profile)),
                                            float(profile_scale), B, H, W, _ptr(x),
                                            _stream(solid.device)))
    return x


def column_profile(solid):
    """solid uint8 [B,H,W] -> float32 [B,W]: the masks' resistance profiles
    along x (wsn_column_profile)."""
    import torch
    if solid.dtype != torch.uint8 or not solid.is_contiguous() or not solid.is_cuda:
        raise ValueError("expected a contiguous uint8 device tensor")
    B, H, W = solid.shape
    prof = torch.empty((B, W), dtype=torch.float32, device=solid.device)
    _check(lib().wsn_column_profile(_ptr(solid), B, H, W, _ptr(prof), _stream(solid.device)))
    return prof


def fields_to_nhwc(rho, u, shift, scale, slope=None):
    """rho [B,H,W], u [B,2,H,W] -> y [B,H,W,3] = (f - shift - slope (x + 1)) * scale
    (per sample and channel; slope optional)."""
    import torch
    B, H, W = rho.shape
    y = torch.empty((B, H, W, 3), dtype=torch.float32, device=rho.device)
    _check(lib().wsn_fields_to_nhwc(_ptr(_f32(rho)), _ptr(_f32(u)), _ptr(_f32(shift)),
                                    _ptr(None if slope is None else _f32(slope)),
                                    _ptr(_f32(scale)), B, H, W, _ptr(y), _stream(rho.device)))
    return y


def nhwc_to_fields(y, shift, scale, slope=None, keep_u=None, out=None):
    """y [B,H,W,3] -> (rho [B,H,W], u [B,2,H,W], bad [B] int32) with
    f = y * scale + shift + slope (x + 1), u = 0 where keep_u (uint8 [B,H,W]) is 0,
    into the tensors of `out` if given."""
    import torch
    B, H, W, _ = y.shape
    if out is not None:
        rho, u, bad = out
        if (tuple(rho.shape) != (B, H, W) or tuple(u.shape) != (B, 2, H, W) or
                tuple(bad.shape) != (B,) or bad.dtype != torch.int32 or not bad.is_contiguous()):
            raise ValueError("out tensors have the wrong shape")
    else:
        rho = torch.empty((B, H, W), dtype=torch.float32, device=y.device)
        u = torch.empty((B, 2, H, W), dtype=torch.float32, device=y.device)
        bad = torch.empty(B, dtype=torch.int32, device=y.device)
    if keep_u is not None and (keep_u.dtype != torch.uint8 or tuple(keep_u.shape) != (B, H, W)
                               or not keep_u.is_contiguous()):
        raise ValueError("keep_u must be a contiguous uint8 [B,H,W] tensor")
    _check(lib().wsn_nhwc_to_fields(_ptr(_f32(y)), _ptr(_f32(shift)),
                                    _ptr(None if slope is None else _f32(slope)),
                                    _ptr(_f32(scale)), _ptr(keep_u), B, H, W, _ptr(rho), _ptr(u),
                                    _ptr(bad), _stream(y.device)))
    return rho, u, bad


def mirror(t, flip_h, flip_w, scale=None, out=None, accumulate=False):
    """Mirror image of t (uint8 [B,H,W] or float32 [B,H,W] / [B,H,W,C]) along H
    (flip_h) and / or W (flip_w), channel k multiplied by scale[k] (float only);
    into `out` if given (same shape and type, not overlapping t), added to it
    with accumulate (float only)."""
    import torch
    if not t.is_cuda or not t.is_contiguous() or t.dtype not in (torch.uint8, torch.float32):
        raise ValueError("expected a contiguous uint8 or float32 device tensor")
    if t.dim() not in (3, 4):
        raise ValueError("expected [B,H,W] or [B,H,W,C]")
    B, H, W = t.shape[:3]
    C = t.shape[3] if t.dim() == 4 else 1
    if accumulate and out is None:
        raise ValueError("accumulate needs out")
    o = out if out is not None else torch.empty_like(t)
    if o.shape != t.shape or o.dtype != t.dtype or not o.is_contiguous():
        raise ValueError("out has the wrong shape or type")
    sc = None
    if scale is not None:
        if len(scale) != C:
            raise ValueError("scale needs one factor per channel")
        sc = (ctypes.c_float * C)(*[float(v) for v in scale])
    _check(lib().wsn_mirror(_ptr(t), t.element_size(), B, H, W, C, int(bool(flip_h)),
                            int(bool(flip_w)), sc, int(bool(accumulate)), _ptr(o),
                            _stream(t.device)))
    return o


# ---------------------------------------------------------------- network

class WarmStartNet:
    """The U-Net with its parameters, Adam state and the buffers of one batch size.

    params: initial parameter vector (NumPy or torch, the layout of wsn.h); the
    random initial values are the caller's.
    """

    def __init__(self, params, batch, levels=4, base=32, in_ch=2, out_ch=3, height=128,
                 width=256, device="cuda"):
        import torch
        self.cfg = Config(levels, base, in_ch, out_ch, height, width)
        self.batch = int(batch)
        self.device = torch.device(device)
        npar, ab, wb = ctypes.c_int64(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(lib().wsn_query_sizes(ctypes.byref(self.cfg), self.batch, ctypes.byref(npar),
                                     ctypes.byref(ab), ctypes.byref(wb)))
        self.n_params = npar.value
        p = torch.as_tensor(np.asarray(params, np.float32) if not torch.is_tensor(params) else params,
                            dtype=torch.float32)
        if p.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.numel()}")
        self.params = p.to(self.device).contiguous().clone()
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.act = torch.empty(ab.value, dtype=torch.uint8, device=self.device)
        self.work = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        self.shape_in = (self.batch, height, width, in_ch)
        self.shape_out = (self.batch, height, width, out_ch)
        self._x = None

    def forward(self, x, y=None):
        import torch
        if tuple(x.shape) != self.shape_in:
            raise ValueError(f"input shape {tuple(x.shape)} != {self.shape_in}")
        if y is None:
            y = torch.empty(self.shape_out, dtype=torch.float32, device=self.device)
        _check(lib().wsn_forward(ctypes.byref(self.cfg), self.batch, _ptr(self.params),
                                 _ptr(_f32(x)), _ptr(y), _ptr(self.act), _stream(self.device)))
        self._x = x
        return y

    def infer(self, x):
        """Forward pass of any batch of at most `batch` inputs; returns y."""
        import torch
        B = x.shape[0]
        if B > self.batch or tuple(x.shape[1:]) != self.shape_in[1:]:
            raise ValueError(f"input shape {tuple(x.shape)} does not fit {self.shape_in}")
        y = torch.empty((B,) + self.shape_out[1:], dtype=torch.float32, device=self.device)
        _check(lib().wsn_forward(ctypes.byref(self.cfg), B, _ptr(self.params), _ptr(_f32(x)),
                                 _ptr(y), _ptr(self.act), _stream(self.device)))
        return y

    def backward(self, dy):
        """Parameter gradient (into self.grad) for the last forward's input."""
        if self._x is None:
            raise RuntimeError("backward before forward")
        _check(lib().wsn_backward(ctypes.byref(self.cfg), self.batch, _ptr(self.params),
                                  _ptr(self._x), _ptr(_f32(dy)), _ptr(self.grad), _ptr(self.act),
                                  _ptr(self.work), _stream(self.device)))
        return self.grad

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        adam(self.params, self.grad, self.m, self.v, self.t, lr, b1, b2, eps)

    def train_step(self, x, target, solid, lr):
        """Forward, masked MSE, backward, Adam.  Returns the loss (device tensor)."""
        y = self.forward(x)
        loss, g = masked_mse(y, target, solid)
        self.backward(g)
        self.adam_step(lr)
        return loss
