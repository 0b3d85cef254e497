"""C ABI checks that need no GPU: the library loads, exports every entry point
that include/*.h declares, and rejects bad arguments before any HIP call."""
import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

from paper_1609_09685_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:lbm|wsn)_[a-z0-9_]+)\s*\(", text)))


def _nm_exports(path):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True,
                         check=True).stdout
    return {ln.split()[-1] for ln in out.splitlines() if ln.strip()}


def _library_of(header):
    from paper_1609_09685_amd import build
    return build.PROBE_LIB if os.path.basename(header) == "lbm_probe.h" else lbm.library_path()


@pytest.mark.parametrize("header", sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))))
def test_every_declared_symbol_is_exported(header):
    names = declared(header)
    assert names
    path = _library_of(header)
    exported = _nm_exports(path)
    missing = [n for n in names if n not in exported]
    assert not missing, f"{os.path.basename(header)}: not exported: {missing}"
    lib = ctypes.CDLL(path)
    for n in names:
        getattr(lib, n)


def test_binding_covers_header():
    from paper_1609_09685_amd import wsn
    names = declared(os.path.join(ROOT, "include", "lbm.h"))
    assert set(names) == set(lbm._SIGS)
    assert set(declared(os.path.join(ROOT, "include", "wsn.h"))) == set(wsn._SIGS)


def _geom(**kw):
    d = dict(lattice=9, nx=100, ny=50, nz=1, precision=lbm.LBM_FP64, check_every=100, rho0=1.0)
    d.update(kw)
    d.setdefault("n_fluid", d["nx"] * d["ny"] * d["nz"])
    return lbm.Geom(**d)


def _status(g):
    fb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    return lbm.load_library().lbm_query_sizes(ctypes.byref(g), ctypes.byref(fb), ctypes.byref(wb)), \
        fb.value, wb.value


@pytest.mark.parametrize("kw", [dict(lattice=7), dict(nz=2), dict(nx=1), dict(ny=0),
                                dict(precision=5), dict(check_every=0), dict(rho0=0.0),
                                dict(rho0=float("nan")), dict(n_fluid=-1),
                                dict(n_fluid=100 * 50 + 1),
                                dict(lattice=19, nx=2048, ny=2048, nz=1025, n_fluid=2**32 + 5),
                                dict(boundary=2), dict(boundary=-1),
                                dict(boundary=1, body_force=float("inf")),
                                dict(body_force=1e-5)])
def test_query_sizes_rejects(kw):
    st, _, _ = _status(_geom(**kw))
    assert st == lbm.LBM_EINVAL
    assert lbm.load_library().lbm_last_error()


@pytest.mark.parametrize("lat,prec,nx,ny,nz,nf,esize", [
    (9, lbm.LBM_FP64, 100, 50, 1, 3700, 8), (9, lbm.LBM_FP32, 100, 50, 1, 3700, 4),
    (19, lbm.LBM_FP32, 512, 512, 512, 80530637, 4), (19, lbm.LBM_FP64, 33, 7, 5, 1, 8),
    (9, lbm.LBM_FP32, 7, 3, 1, 0, 4), (19, lbm.LBM_FP32, 130, 9, 7, 5000, 4)])
def test_query_sizes_layout(lat, prec, nx, ny, nz, nf, esize):
    st, fb, wb = _status(_geom(lattice=lat, precision=prec, nx=nx, ny=ny, nz=nz, n_fluid=nf))
    assert st == lbm.LBM_OK
    nw = (nx + 63) // 64
    S = 4 if nw >= 4 else (2 if nw >= 2 else 1)          # words per row segment
    nsegs = ny * nz * (-(-nw // S))
    align = 128 // esize                                  # segments start on 128 B
    ps = max(64, (nf + (align - 1) * nsegs + 63) // 64 * 64)   # fluid slots + padding room
    assert fb == lat * ps * esize
    assert wb >= ny * nz * (nw + 2) * 8 + ny * nz * nw * 4   # bitmap + prefix counts


def test_init_validates_before_any_hip_call():
    lib = lbm.load_library()
    g = _geom()
    fake = 1 << 20  # never dereferenced: every call below must fail validation first
    bufs = lbm.Buffers()
    bufs.f[0], bufs.f[1], bufs.mask, bufs.work, bufs.stream = fake, fake * 2, fake * 3, fake * 4, 0
    h = ctypes.c_void_p(0)
    cases = [
        (dict(tau=0.5, ri=1.0, ro=1.0), "tau"),
        (dict(tau=0.2, ri=1.0, ro=1.0), "tau"),
        (dict(tau=float("nan"), ri=1.0, ro=1.0), "tau"),
        (dict(tau=0.8, ri=0.0, ro=1.0), "rho"),
        (dict(tau=0.8, ri=1.0, ro=-1.0), "rho"),
    ]
    for kw, word in cases:
        st = lib.lbm_init(ctypes.byref(h), ctypes.byref(g), ctypes.byref(bufs), kw["tau"], kw["ri"], kw["ro"])
        assert st == lbm.LBM_EINVAL
        assert word in lib.lbm_last_error().decode()
        assert not h.value
    nb = lbm.Buffers()
    st = lib.lbm_init(ctypes.byref(h), ctypes.byref(g), ctypes.byref(nb), 0.8, 1.0, 1.0)
    assert st == lbm.LBM_EINVAL
    same = lbm.Buffers()
    same.f[0], same.f[1], same.mask, same.work = fake, fake, fake, fake
    assert lib.lbm_init(ctypes.byref(h), ctypes.byref(g), ctypes.byref(same), 0.8, 1.0, 1.0) == lbm.LBM_EINVAL
    odd = lbm.Buffers()
    odd.f[0], odd.f[1], odd.mask, odd.work = fake + 4, fake * 2, fake, fake * 4
    assert lib.lbm_init(ctypes.byref(h), ctypes.byref(g), ctypes.byref(odd), 0.8, 1.0, 1.0) == lbm.LBM_EINVAL
    # periodic case: one density everywhere (no inlet / outlet)
    gp = _geom(boundary=lbm.LBM_BC_PERIODIC, body_force=1e-5)
    st = lib.lbm_init(ctypes.byref(h), ctypes.byref(gp), ctypes.byref(bufs), 0.8, 1.001, 0.999)
    assert st == lbm.LBM_EINVAL and "periodic" in lib.lbm_last_error().decode()
    assert not h.value
    assert lib.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_set_trt(None, 0.1875) == lbm.LBM_EINVAL
    assert lib.lbm_destroy(None) == lbm.LBM_OK


@pytest.mark.parametrize("Q", [9, 19])
def test_library_lattice_tables(Q):
    """The solver's own direction tables satisfy the lattice identities."""
    c, w = lbm.lattice_table(Q)
    c = c.astype(float)
    d = 2 if Q == 9 else 3
    assert len({tuple(v) for v in c}) == Q
    assert math.isclose(w.sum(), 1.0, rel_tol=1e-15)
    assert np.allclose(w @ c, 0, atol=1e-16)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c)[:d, :d], np.eye(d) / 3, atol=1e-15)
    four = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    e = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", e, e) + np.einsum("ac,bd->abcd", e, e)
           + np.einsum("ad,bc->abcd", e, e)) / 9
    assert np.allclose(four[:d, :d, :d, :d], iso[:d, :d, :d, :d], atol=1e-15)


def test_knudsen():
    for tau, nx in [(0.51, 400), (2.0, 1200), (0.8, 100)]:
        assert lbm.knudsen(tau, nx) == pytest.approx(math.sqrt(math.pi / 6) * (tau - 0.5) / nx,
                                                     rel=1e-15)


def test_solver_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        lbm.Solver(np.zeros((4, 8), np.uint8), 0.8, 1.001, 0.999)


def test_solver_rejects_unknown_names():
    """Bad option strings fail before any GPU or library work."""
    with pytest.raises(ValueError):
        lbm.Solver(np.zeros((4, 8), np.uint8), 0.8, 1.001, 0.999, precision="fp16")
    with pytest.raises(ValueError):
        lbm.Solver(np.zeros((4, 8), np.uint8), 0.8, 1.0, 1.0, boundary="wall")


def test_batch_entry_points_validate():
    """Batch calls reject empty or NULL arguments before touching the device."""
    lib = lbm.load_library()
    wb = ctypes.c_size_t(0)
    assert lib.lbm_batch_query_sizes(0, None, ctypes.byref(wb)) == lbm.LBM_EINVAL
    assert "n >= 1" in lib.lbm_last_error().decode()
    assert lib.lbm_batch_query_sizes(2, None, ctypes.byref(wb)) == lbm.LBM_EINVAL
    nulls = (ctypes.c_void_p * 2)(None, None)
    assert lib.lbm_batch_query_sizes(2, nulls, ctypes.byref(wb)) == lbm.LBM_EINVAL
    assert "NULL" in lib.lbm_last_error().decode()
    h = ctypes.c_void_p(0)
    assert lib.lbm_batch_create(ctypes.byref(h), 2, nulls, 1 << 20, None) == lbm.LBM_EINVAL
    assert not h.value
    assert lib.lbm_batch_create(None, 1, nulls, 1 << 20, None) == lbm.LBM_EINVAL
    for call in (lambda: lib.lbm_batch_step(None, 1),
                 lambda: lib.lbm_batch_run_to_steady(None, 1e-9, 10, None, None, None, None, 0),
                 lambda: lib.lbm_batch_flux(None, None),
                 lambda: lib.lbm_batch_permeability(None, None, None),
                 lambda: lib.lbm_batch_set_option(None, lbm.LBM_BATCH_OPT_GRAPH, 1)):
        assert call() == lbm.LBM_EINVAL
    assert lib.lbm_batch_destroy(None) == lbm.LBM_OK


def test_wsn_sizes_and_validation():
    """Network queries agree with the reference layer table; bad shapes and
    arguments are rejected before any HIP call."""
    from oracle import unet_ref
    from paper_1609_09685_amd import wsn
    L = wsn.lib()
    npar, ab, wb = ctypes.c_int64(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
    cfg = wsn.Config(4, 32, 2, 3, 128, 256)
    assert L.wsn_query_sizes(ctypes.byref(cfg), 8, ctypes.byref(npar), ctypes.byref(ab),
                             ctypes.byref(wb)) == lbm.LBM_OK
    assert npar.value == unet_ref.param_count(levels=4, base=32, in_ch=2, out_ch=3)
    assert ab.value > 8 * 128 * 256 * 4 * 64 and wb.value > ab.value
    for bad in [wsn.Config(0, 32, 2, 3, 128, 256), wsn.Config(4, 32, 2, 3, 100, 256),
                wsn.Config(4, 32, 2, 3, 128, 200), wsn.Config(4, 0, 2, 3, 128, 256),
                wsn.Config(4, 32, 2, 0, 128, 256)]:
        assert L.wsn_query_sizes(ctypes.byref(bad), 8, None, None, None) == lbm.LBM_EINVAL
    assert L.wsn_query_sizes(ctypes.byref(cfg), 0, None, None, None) == lbm.LBM_EINVAL
    fake = 1 << 20
    # width not a multiple of 16, ks not 1/3, NULL buffers
    assert L.wsn_conv_forward(fake, fake, None, fake, 1, 8, 24, 4, 4, 3, 1, None) == lbm.LBM_EINVAL
    assert L.wsn_conv_forward(fake, fake, None, fake, 1, 8, 32, 4, 4, 5, 1, None) == lbm.LBM_EINVAL
    assert L.wsn_conv_forward(None, fake, None, fake, 1, 8, 32, 4, 4, 3, 1, None) == lbm.LBM_EINVAL
    n = ctypes.c_size_t(0)
    assert L.wsn_conv_wgrad_work(2, 16, 32, 8, 8, 3, ctypes.byref(n)) == lbm.LBM_OK and n.value > 0
    assert L.wsn_conv_backward_weight(fake, fake, fake, None, 2, 16, 32, 8, 8, 3, fake, n.value - 1,
                                      None) == lbm.LBM_ENOMEM
    assert L.wsn_pool_forward(fake, fake, 1, 7, 8, 4, None) == lbm.LBM_EINVAL
    assert L.wsn_upcat_forward(fake, fake, fake, 1, 8, 8, 0, 4, None) == lbm.LBM_EINVAL
    assert L.wsn_adam(fake, fake, fake, fake, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == lbm.LBM_EINVAL
    assert L.wsn_adam(fake, fake, fake, fake, 10, 1e-3, 1.0, 0.999, 1e-8, 1, None) == lbm.LBM_EINVAL
    assert L.wsn_mse_work(0, ctypes.byref(n)) == lbm.LBM_EINVAL
    sg = (ctypes.c_float * 9)(*([1.0] * 9))
    other = fake + 4096
    for args in [(fake, 2, 1, 4, 4, 3, 1, 0, None, 0, other),      # element size
                 (fake, 4, 1, 4, 4, 3, 2, 0, None, 0, other),      # flip flag
                 (fake, 4, 1, 4, 4, 3, 1, 0, None, 2, other),      # accumulate flag
                 (fake, 1, 1, 4, 4, 1, 1, 0, sg, 0, other),        # scale on bytes
                 (fake, 1, 1, 4, 4, 1, 1, 0, None, 1, other),      # accumulate on bytes
                 (fake, 4, 1, 4, 4, 9, 1, 0, sg, 0, other),        # scale beyond 8 channels
                 (fake, 4, 1, 4, 4, 3, 1, 1, None, 0, fake),       # in place
                 (None, 4, 1, 4, 4, 3, 1, 1, None, 0, other),
                 (fake, 4, 0, 4, 4, 3, 1, 1, None, 0, other)]:
        assert L.wsn_mirror(*args, None) == lbm.LBM_EINVAL, args
    assert L.wsn_column_profile(None, 1, 4, 16, fake, None) == lbm.LBM_EINVAL
    assert L.wsn_column_profile(fake, 0, 4, 16, fake, None) == lbm.LBM_EINVAL
    assert L.wsn_column_profile(fake, 1, 4, 16385, fake, None) == lbm.LBM_EINVAL
    assert L.wsn_pack_input_profile(fake, fake, None, 1.0, 1, 4, 16, fake, None) == lbm.LBM_EINVAL
    assert L.wsn_pack_input_profile(fake, fake, fake, float("nan"), 1, 4, 16, fake,
                                    None) == lbm.LBM_EINVAL


def test_probe_rejects_bad_arguments():
    """The streaming probes validate before launching (no GPU needed)."""
    from paper_1609_09685_amd import build
    lib = ctypes.CDLL(build.PROBE_LIB)
    f = lib.lbm_probe_stream
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int] * 4 + [ctypes.c_uint64] + [ctypes.c_void_p] * 4
    p = ctypes.c_void_p(256)
    assert f(3, 1, 1, 19, 1024, p, p, p, None) == -1      # mode
    assert f(0, 2, 1, 19, 1024, p, p, p, None) == -1      # vector width
    assert f(0, 1, 1, 7, 1024, p, p, p, None) == -1       # array count
    assert f(0, 4, 1, 19, 1000, p, p, p, None) == -1      # n not a multiple of 1024
    assert f(0, 1, 1, 19, 0, p, p, p, None) == -1         # empty
    assert f(1, 1, 0, 19, 1024, p, None, None, None) == -1  # read mode without a sink
    assert f(0, 1, 1, 19, 1024, ctypes.c_void_p(258), p, p, None) == -1   # misaligned
