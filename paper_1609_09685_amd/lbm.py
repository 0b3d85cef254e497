"""Python binding of the C ABI in ``include/lbm.h`` (argument marshalling only).

Every step of the solver runs in the HIP library ``liblbm.so``; torch only
allocates the device buffers the library asks for and supplies the stream.
There is no CPU fallback: importing this module without the built library, or
constructing a solver without a GPU, raises.
"""
import ctypes
import os

import numpy as np

from . import build as _build

LBM_OK, LBM_EINVAL, LBM_EHIP, LBM_ENOMEM = 0, -1, -2, -3
LBM_ENONFINITE, LBM_ENOTCONV, LBM_ENOFLOW, LBM_ESTATE = -4, -5, -6, -7
LBM_D2Q9, LBM_D3Q19 = 9, 19
LBM_FP64, LBM_FP32 = 0, 1
_PRECISION = {"fp64": LBM_FP64, "fp32": LBM_FP32}
_START = {"uniform": 0, "linear": 1}
LBM_BC_PRESSURE, LBM_BC_PERIODIC = 0, 1
_BOUNDARY = {"pressure": LBM_BC_PRESSURE, "periodic": LBM_BC_PERIODIC}


class LBMError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"[{status}] {message}")
        self.status = status
        self.message = message


class Geom(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("rho0", ctypes.c_double),
                ("n_fluid", ctypes.c_int64), ("boundary", ctypes.c_int32),
                ("body_force", ctypes.c_double)]


class Buffers(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p * 2), ("mask", ctypes.c_void_p), ("work", ctypes.c_void_p),
                ("stream", ctypes.c_void_p)]


_lib = None

# name -> (restype, argtypes) for every entry point of include/lbm.h
_c = ctypes
_SIGS = {
    "lbm_query_sizes": (_c.c_int, [_c.POINTER(Geom), _c.POINTER(_c.c_size_t), _c.POINTER(_c.c_size_t)]),
    "lbm_init": (_c.c_int, [_c.POINTER(_c.c_void_p), _c.POINTER(Geom), _c.POINTER(Buffers),
                            _c.c_double, _c.c_double, _c.c_double]),
    "lbm_reset": (_c.c_int, [_c.c_void_p, _c.c_int32]),
    "lbm_set_macro": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "lbm_step": (_c.c_int, [_c.c_void_p, _c.c_int64]),
    "lbm_smooth": (_c.c_int, [_c.c_void_p, _c.c_int32]),
    "lbm_flux": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_double)]),
    "lbm_flux_noalloc": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_double)]),
    "lbm_permeability": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_double)]),
    "lbm_run_to_steady": (_c.c_int, [_c.c_void_p, _c.c_double, _c.c_int64,
                                     _c.POINTER(_c.c_int64), _c.POINTER(_c.c_double)]),
    "lbm_get_macro": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int32]),
    "lbm_get_populations": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "lbm_set_populations": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "lbm_set_option": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int64]),
    "lbm_set_trt": (_c.c_int, [_c.c_void_p, _c.c_double]),
    "lbm_get_slot_map": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "lbm_lattice": (_c.c_int, [_c.c_int32, _c.c_void_p, _c.c_void_p]),
    "lbm_steps": (_c.c_int, [_c.c_void_p, _c.POINTER(_c.c_int64)]),
    "lbm_knudsen": (_c.c_double, [_c.c_double, _c.c_int32]),
    "lbm_destroy": (_c.c_int, [_c.c_void_p]),
    "lbm_batch_query_sizes": (_c.c_int, [_c.c_int32, _c.c_void_p, _c.POINTER(_c.c_size_t)]),
    "lbm_batch_create": (_c.c_int, [_c.POINTER(_c.c_void_p), _c.c_int32, _c.c_void_p, _c.c_void_p,
                                    _c.c_void_p]),
    "lbm_batch_step": (_c.c_int, [_c.c_void_p, _c.c_int64]),
    "lbm_batch_run_to_steady": (_c.c_int, [_c.c_void_p, _c.c_double, _c.c_int64, _c.c_void_p,
                                           _c.c_void_p, _c.c_void_p, _c.c_void_p, _c.c_int64]),
    "lbm_batch_flux": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "lbm_batch_permeability": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_void_p]),
    "lbm_batch_set_option": (_c.c_int, [_c.c_void_p, _c.c_int32, _c.c_int64]),
    "lbm_batch_destroy": (_c.c_int, [_c.c_void_p]),
    "lbm_last_error": (_c.c_char_p, []),
    "lbm_version": (_c.c_char_p, []),
}


def library_path():
    return _build.LBM_LIB


def load_library():
    """Loads liblbm.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1609_09685_amd.build`"
                          " (the solver has no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, allow=()):
    if status != LBM_OK and status not in allow:
        msg = load_library().lbm_last_error().decode(errors="replace")
        raise LBMError(status, msg)
    return status


LBM_OPT_XCD_REMAP, LBM_OPT_LINEAR_EQ = 1, 2
LBM_OPT_BAND = 6
LBM_OPT_WIDE_OFFSETS = 7
LBM_BATCH_OPT_GRAPH = 1


def query_sizes(lattice, nx, ny, nz, n_fluid, precision="fp32", check_every=100, rho0=1.0):
    g = Geom(lattice, nx, ny, nz, _PRECISION[precision], check_every, rho0, n_fluid)
    fb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _check(load_library().lbm_query_sizes(ctypes.byref(g), ctypes.byref(fb), ctypes.byref(wb)))
    return fb.value, wb.value


def lattice_table(lattice):
    """(c, w) of the library's internal direction order."""
    q = int(lattice)
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q)
    _check(load_library().lbm_lattice(q, c.ctypes.data, w.ctypes.data))
    return c, w


def knudsen(tau, nx):
    return float(load_library().lbm_knudsen(float(tau), int(nx)))


class Solver:
    """One porous domain on one GPU.

    mask: uint8 array, (ny, nx) for D2Q9 or (nz, ny, nx) for D3Q19, 1 = solid.
    precision: "fp64" or "fp32" (populations stored as deviations from rest).
    """

    def __init__(self, mask, tau, rho_in, rho_out, precision="fp32", lattice=None,
                 check_every=100, rho0=1.0, device="cuda", stream=None, boundary="pressure",
                 body_force=0.0):
        """boundary: "pressure" (density at inlet / outlet ghost planes, symmetric
        sides) or "periodic" (six periodic faces driven by the acceleration
        body_force along x; rho_in = rho_out is then the starting density)."""
        import torch

        if precision not in _PRECISION:
            raise ValueError(f"precision must be one of {sorted(_PRECISION)}, got {precision!r}")
        if boundary not in _BOUNDARY:
            raise ValueError(f"boundary must be one of {sorted(_BOUNDARY)}, got {boundary!r}")
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the lattice Boltzmann solver needs a GPU (HIP device)")
        m = np.ascontiguousarray(mask, np.uint8)
        if lattice is None:
            lattice = LBM_D2Q9 if m.ndim == 2 else LBM_D3Q19
        if m.ndim == 2:
            m = m[None]
        if m.ndim != 3:
            raise ValueError("mask must be 2D or 3D")
        self.nz, self.ny, self.nx = (int(s) for s in m.shape)
        self.lattice = int(lattice)
        self.precision = precision
        self.tau, self.rho_in, self.rho_out = float(tau), float(rho_in), float(rho_out)
        self.D = 2 if self.lattice == LBM_D2Q9 else 3
        self.device = torch.device(device)
        self.n_fluid = int((m == 0).sum())
        self.boundary, self.body_force = boundary, float(body_force)
        self.trt_magic = 0.0
        self._geom = Geom(self.lattice, self.nx, self.ny, self.nz, _PRECISION[precision],
                          int(check_every), float(rho0), self.n_fluid, _BOUNDARY[boundary],
                          self.body_force)
        fb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(lib.lbm_query_sizes(ctypes.byref(self._geom), ctypes.byref(fb), ctypes.byref(wb)))
        self.f_bytes, self.work_bytes = fb.value, wb.value
        self._f = [torch.empty(self.f_bytes, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self._work = torch.empty(self.work_bytes, dtype=torch.uint8, device=self.device)
        self._mask = torch.from_numpy(m.reshape(-1).copy()).to(self.device)
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        bufs = Buffers()
        bufs.f[0] = self._f[0].data_ptr()
        bufs.f[1] = self._f[1].data_ptr()
        bufs.mask = self._mask.data_ptr()
        bufs.work = self._work.data_ptr()
        bufs.stream = self._stream.cuda_stream
        self._bufs = bufs
        h = ctypes.c_void_p(0)
        _check(lib.lbm_init(ctypes.byref(h), ctypes.byref(self._geom), ctypes.byref(bufs),
                            self.tau, self.rho_in, self.rho_out))
        self._h = h
        self._lib = lib

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lbm_destroy(h)
            self._h = None

    __del__ = close

    def set_option(self, option, value):
        _check(self._lib.lbm_set_option(self._h, int(option), int(value)))

    def set_linear_equilibrium(self, on=True):
        self.set_option(LBM_OPT_LINEAR_EQ, 1 if on else 0)

    def set_wide_offsets(self, on=True):
        """Address the populations with 64-bit offsets (the form very large domains
        use) even where 32-bit ones fit; results are bitwise the same."""
        self.set_option(LBM_OPT_WIDE_OFFSETS, 1 if on else 0)

    def set_trt(self, magic=3.0 / 16.0):
        """Two-relaxation-time collision with the magic parameter
        (tau - 1/2)(tau_minus - 1/2) = magic; magic = 0 returns to BGK."""
        _check(self._lib.lbm_set_trt(self._h, float(magic)))
        self.trt_magic = float(magic)

    def set_xcd_remap(self, mode=1):
        """Tile order over the XCDs: 0 hardware, 1 contiguous eighths, m >= 2 chunks of
        m - 1 tile rows dealt round-robin."""
        self.set_option(LBM_OPT_XCD_REMAP, int(mode))

    def set_band(self, tile_rows):
        """> 0: banded tile order with bands of `tile_rows` tile rows; 0: off."""
        self.set_option(LBM_OPT_BAND, tile_rows)

    def configure(self, xcd_remap=None, band=None):
        """Launch configuration of the step kernel (results are bitwise identical)."""
        if band is not None:
            self.set_band(band)
        if xcd_remap is not None:
            self.set_xcd_remap(xcd_remap)

    # -- state --------------------------------------------------------------
    def reset(self, start="uniform"):
        _check(self._lib.lbm_reset(self._h, _START[start]))

    def set_macro(self, rho, u):
        """Start from f = f_eq(rho, u); rho (nz,ny,nx) / u (D,nz,ny,nx) float32 device tensors."""
        import torch
        rho = rho.to(self.device, torch.float32).contiguous()
        u = u.to(self.device, torch.float32).contiguous()
        if rho.numel() != self.nx * self.ny * self.nz or u.numel() != self.D * rho.numel():
            raise ValueError("rho / u have the wrong number of elements")
        _check(self._lib.lbm_set_macro(self._h, rho.data_ptr(), u.data_ptr()))
        self._keep = (rho, u)  # kept alive until the stream has consumed them

    def step(self, n=1):
        _check(self._lib.lbm_step(self._h, int(n)))

    def smooth(self, n=1):
        """n passes of: one step, then the mean of the states before and after it
        (removes modes that alternate every step; counts n steps)."""
        _check(self._lib.lbm_smooth(self._h, int(n)))

    @property
    def steps(self):
        s = ctypes.c_int64(0)
        _check(self._lib.lbm_steps(self._h, ctypes.byref(s)))
        return s.value

    def flux(self):
        q = ctypes.c_double(0.0)
        _check(self._lib.lbm_flux(self._h, ctypes.byref(q)))
        return q.value

    def flux_noalloc(self):
        """lbm_flux_noalloc: the same flux with the library's own scratch."""
        q = ctypes.c_double(0.0)
        _check(self._lib.lbm_flux_noalloc(self._h, ctypes.byref(q)))
        return q.value

    def permeability(self):
        k = ctypes.c_double(0.0)
        _check(self._lib.lbm_permeability(self._h, ctypes.byref(k)))
        return k.value

    def run_to_steady(self, tol=1e-9, max_steps=10**6, raise_on_notconv=True):
        """Returns (converged, steps, residual)."""
        s, r = ctypes.c_int64(0), ctypes.c_double(0.0)
        st = self._lib.lbm_run_to_steady(self._h, float(tol), int(max_steps), ctypes.byref(s),
                                         ctypes.byref(r))
        _check(st, allow=() if raise_on_notconv else (LBM_ENOTCONV,))
        return st == LBM_OK, s.value, r.value

    def macro(self, dtype="float64", out=None):
        """(rho (nz,ny,nx), u (D,nz,ny,nx)) as device tensors; solids rho0 and 0.
        out: optional (rho, u) contiguous device tensors of those sizes to fill."""
        import torch
        td = torch.float64 if dtype == "float64" else torch.float32
        if out is not None:
            rho, u = out
            n = self.nx * self.ny * self.nz
            if (rho.dtype != td or u.dtype != td or not rho.is_contiguous() or not u.is_contiguous()
                    or rho.numel() != n or u.numel() != self.D * n):
                raise ValueError("out tensors have the wrong dtype, size or layout")
        else:
            rho = torch.empty((self.nz, self.ny, self.nx), dtype=td, device=self.device)
            u = torch.empty((self.D, self.nz, self.ny, self.nx), dtype=td, device=self.device)
        _check(self._lib.lbm_get_macro(self._h, rho.data_ptr(), u.data_ptr(),
                                       1 if td == torch.float64 else 0))
        return rho, u

    def slot_map(self):
        """Device int32 tensor (nz, ny, nx): slot of every node, -1 for solids."""
        import torch
        m = torch.empty((self.nz, self.ny, self.nx), dtype=torch.int32, device=self.device)
        _check(self._lib.lbm_get_slot_map(self._h, m.data_ptr()))
        return m

    def get_populations(self):
        import torch
        out = torch.empty(self.f_bytes, dtype=torch.uint8, device=self.device)
        _check(self._lib.lbm_get_populations(self._h, out.data_ptr()))
        return out

    def set_populations(self, buf):
        if buf.numel() * buf.element_size() != self.f_bytes:
            raise ValueError("population buffer has the wrong size")
        _check(self._lib.lbm_set_populations(self._h, buf.data_ptr()))
        self._keep = buf

    def knudsen(self):
        return knudsen(self.tau, self.nx)

    def synchronize(self):
        self._stream.synchronize()


class Batch:
    """Many solvers advanced together: one step launch per time step for all.

    Every per-sample result equals, bit for bit, what the same calls on each
    Solver alone would give.  The solvers must share lattice, precision,
    check_every, the linear-equilibrium option and the stream; they stay
    usable on their own.
    """

    def __init__(self, solvers, graph=True):
        import torch

        self.solvers = list(solvers)
        if not self.solvers:
            raise ValueError("a batch needs at least one solver")
        lib = load_library()
        self._lib = lib
        n = len(self.solvers)
        self.n = n
        self._handles = (ctypes.c_void_p * n)(*[s._h.value for s in self.solvers])
        wb = ctypes.c_size_t(0)
        _check(lib.lbm_batch_query_sizes(n, self._handles, ctypes.byref(wb)))
        s0 = self.solvers[0]
        self._stream = s0._stream
        self._work = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=s0.device)
        h = ctypes.c_void_p(0)
        _check(lib.lbm_batch_create(ctypes.byref(h), n, self._handles, self._work.data_ptr(),
                                    self._stream.cuda_stream))
        self._h = h
        self.set_graph(graph)

    @classmethod
    def from_masks(cls, masks, taus, rho_in, rho_out, precision="fp32", check_every=100,
                   graph=True, autotune=False, **kw):
        """Solvers for masks[j] with taus[j] (scalars or per-sample sequences for rho).
        autotune: pick the step kernel's tile order per geometry class (timing only;
        results are bitwise the same)."""
        n = len(masks)
        tau = np.broadcast_to(np.asarray(taus, float), (n,))
        rin = np.broadcast_to(np.asarray(rho_in, float), (n,))
        rout = np.broadcast_to(np.asarray(rho_out, float), (n,))
        solvers = [Solver(m, float(tau[j]), float(rin[j]), float(rout[j]), precision=precision,
                          check_every=check_every, **kw) for j, m in enumerate(masks)]
        if autotune:
            from . import autotune as _at
            for s, m in zip(solvers, masks):
                _at.apply(s, _at.tune(m, precision=precision, lattice=s.lattice))
        return cls(solvers, graph=graph)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.lbm_batch_destroy(h)
            self._h = None

    __del__ = close

    def set_graph(self, on=True):
        """Replay each check window as a HIP graph (on) or launch it kernel by kernel."""
        _check(self._lib.lbm_batch_set_option(self._h, LBM_BATCH_OPT_GRAPH, 1 if on else 0))

    def step(self, n=1):
        _check(self._lib.lbm_batch_step(self._h, int(n)))

    def run_to_steady(self, tol=1e-9, max_steps=10**6, log_windows=0):
        """Returns (status, steps, residual) arrays, one entry per sample (status: LBM_OK,
        LBM_ENOTCONV or LBM_ENONFINITE), plus, when log_windows > 0, the flux after
        each of the first log_windows check windows ([windows, n], NaN after a sample
        retires).  Never raises for a sample that did not converge."""
        steps = np.zeros(self.n, np.int64)
        resid = np.zeros(self.n)
        status = np.zeros(self.n, np.int32)
        log = np.zeros((max(int(log_windows), 0), self.n))
        st = self._lib.lbm_batch_run_to_steady(self._h, float(tol), int(max_steps),
                                               steps.ctypes.data, resid.ctypes.data,
                                               status.ctypes.data,
                                               log.ctypes.data if log.size else None,
                                               int(log.shape[0]))
        _check(st, allow=(LBM_ENOTCONV, LBM_ENONFINITE))
        if log_windows:
            return status, steps, resid, log
        return status, steps, resid

    def flux(self):
        q = np.zeros(self.n)
        _check(self._lib.lbm_batch_flux(self._h, q.ctypes.data))
        return q

    def permeability(self):
        """(k, status) arrays; status LBM_ENOFLOW / LBM_ENONFINITE per sample where k is not a
        permeability."""
        k = np.zeros(self.n)
        status = np.zeros(self.n, np.int32)
        st = self._lib.lbm_batch_permeability(self._h, k.ctypes.data, status.ctypes.data)
        _check(st, allow=(LBM_ENOFLOW, LBM_ENONFINITE))
        return k, status

    def synchronize(self):
        self._stream.synchronize()
