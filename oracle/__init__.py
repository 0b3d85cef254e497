"""Plain FP64 CPU oracle of the lattice Boltzmann permeability computation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU solver in ``paper_1609_09685_amd``: the lattice Boltzmann arithmetic
lives in ``lbm_oracle.c`` (binary64, no floating-point contraction) and the
U-Net reference in ``unet_ref.py`` (NumPy float64).

Populations here are node-major, ``f[node, i]`` with nodes ordered x fastest;
masks are ``uint8`` arrays shaped ``(ny, nx)`` (2D) or ``(nz, ny, nx)`` (3D),
1 = solid.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_ll = ctypes.c_longlong
_p = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_create.restype = _p
    lib.oracle_create.argtypes = [_i, _i, _i, _i, _p, _d, _d, _d, _i]
    lib.oracle_destroy.argtypes = [_p]
    lib.oracle_init_rest.argtypes = [_p, _i]
    lib.oracle_init_fields.argtypes = [_p, _p, _p]
    lib.oracle_set_f.argtypes = [_p, _p]
    lib.oracle_get_f.argtypes = [_p, _p]
    lib.oracle_step.argtypes = [_p, _ll]
    lib.oracle_steps.argtypes = [_p]
    lib.oracle_steps.restype = _ll
    lib.oracle_macro.argtypes = [_p, _p, _p]
    for name in ("oracle_flux", "oracle_mass", "oracle_permeability"):
        getattr(lib, name).argtypes = [_p]
        getattr(lib, name).restype = _d
    lib.oracle_run_to_steady.argtypes = [_p, _d, _i, _ll, ctypes.POINTER(_ll), ctypes.POINTER(_d)]
    lib.oracle_run_to_steady.restype = _i
    lib.oracle_lattice.argtypes = [_i, _p, _p, _p, _p, _p]
    lib.oracle_lattice.restype = _i
    lib.oracle_feq.argtypes = [_i, _d, _p, _i, _p]
    lib.oracle_collide.argtypes = [_i, _p, _d, _i, _p]
    lib.oracle_knudsen.argtypes = [_d, _i]
    lib.oracle_knudsen.restype = _d
    lib.oracle_set_periodic.argtypes = [_p, _i, _d, _d]
    lib.oracle_set_periodic.restype = _i
    lib.oracle_set_trt.argtypes = [_p, _d]
    lib.oracle_set_trt.restype = _i
    lib.oracle_collide_trt.argtypes = [_i, _p, _d, _d, _i, _p]
    lib.oracle_set_threads.argtypes = [_i]
    lib.oracle_threads.restype = _i
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n):
    _load().oracle_set_threads(int(n))


def threads():
    return int(_load().oracle_threads())


def lattice(Q):
    """Lattice tables of D2Q9 (Q=9) or D3Q19 (Q=19): c (Q,3), w, opp, my, mz."""
    lib = _load()
    c = np.zeros((Q, 3), np.int32)
    w = np.zeros(Q)
    opp, my, mz = (np.zeros(Q, np.int32) for _ in range(3))
    if lib.oracle_lattice(Q, _ptr(c), _ptr(w), _ptr(opp), _ptr(my), _ptr(mz)) != Q:
        raise ValueError("unknown lattice")
    return {"c": c, "w": w, "opp": opp, "my": my, "mz": mz}


def feq(Q, rho, u, linear=False):
    out = np.zeros(Q)
    u3 = np.zeros(3)
    u3[: len(u)] = u
    _load().oracle_feq(Q, float(rho), _ptr(u3), int(linear), _ptr(out))
    return out


def collide(Q, fin, tau, linear=False):
    fin = np.ascontiguousarray(fin, np.float64)
    out = np.zeros(Q)
    _load().oracle_collide(Q, _ptr(fin), float(tau), int(linear), _ptr(out))
    return out


def collide_trt(Q, fin, tau, magic, linear=False):
    """One TRT collision of a node's populations fin (length Q), Lambda = magic."""
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    out = np.zeros(Q)
    _load().oracle_collide_trt(Q, _ptr(fin), float(tau), float(magic), int(linear), _ptr(out))
    return out


def knudsen(tau, nx):
    """Kn = sqrt(pi/6) (tau - 1/2) / Nx."""
    return float(_load().oracle_knudsen(float(tau), int(nx)))


def viscosity(tau):
    """Eq. 1 in lattice units: nu = (tau - 1/2)/3."""
    return (tau - 0.5) / 3.0


def intrinsic_permeability(taus, ks):
    """k_int as the tau -> 1/2 limit: least-squares line k = k_int + b (tau - 1/2)^2."""
    lam = (np.asarray(taus, np.float64) - 0.5) ** 2
    A = np.stack([np.ones_like(lam), lam], axis=1)
    sol, *_ = np.linalg.lstsq(A, np.asarray(ks, np.float64), rcond=None)
    return float(sol[0])


class Oracle:
    """One lattice Boltzmann domain on the CPU.

    Q: 9 (D2Q9, mask (ny, nx)) or 19 (D3Q19, mask (nz, ny, nx)).
    """

    def __init__(self, Q, mask, tau, rho_in, rho_out, linear_eq=False, start="uniform",
                 periodic=False, force=0.0, rho0=1.0, trt_magic=0.0):
        """periodic=True: six periodic faces and a body force of density `force`
        (= rho0 g) along x, the paper's 3D case; rho_in = rho_out is then the
        starting density.  trt_magic > 0: two-relaxation-time collision with
        Lambda = (tau - 1/2)(tau_minus - 1/2) = trt_magic (0: BGK)."""
        lib = _load()
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        if m.ndim == 2:
            m = m[None]
        self.Q = Q
        self.nz, self.ny, self.nx = m.shape
        self.mask = m
        self.tau, self.rho_in, self.rho_out = float(tau), float(rho_in), float(rho_out)
        self._h = lib.oracle_create(Q, self.nx, self.ny, self.nz, _ptr(m), self.tau,
                                    self.rho_in, self.rho_out, int(linear_eq))
        if not self._h:
            raise ValueError("oracle_create rejected the arguments")
        self._lib = lib
        self.periodic, self.force, self.rho0 = bool(periodic), float(force), float(rho0)
        if lib.oracle_set_periodic(self._h, int(self.periodic), self.force, self.rho0) != 0:
            raise ValueError("a body force needs the periodic case")
        self.trt_magic = float(trt_magic)
        if lib.oracle_set_trt(self._h, self.trt_magic) != 0:
            raise ValueError("trt_magic must be >= 0")
        self.init_rest(start)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oracle_destroy(h)
            self._h = None

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def init_rest(self, start="uniform"):
        self._lib.oracle_init_rest(self._h, {"uniform": 0, "linear": 1}[start])

    def init_fields(self, rho, u):
        rho = np.ascontiguousarray(rho, np.float64).reshape(-1)
        u = np.asarray(u, np.float64).reshape(self.N, -1)
        u3 = np.zeros((self.N, 3))
        u3[:, : u.shape[1]] = u
        self._lib.oracle_init_fields(self._h, _ptr(rho), _ptr(u3))

    def set_f(self, f):
        f = np.ascontiguousarray(f, np.float64).reshape(self.N, self.Q)
        self._lib.oracle_set_f(self._h, _ptr(f))

    def get_f(self):
        f = np.zeros((self.N, self.Q))
        self._lib.oracle_get_f(self._h, _ptr(f))
        return f

    def step(self, n=1):
        self._lib.oracle_step(self._h, int(n))

    @property
    def steps(self):
        return int(self._lib.oracle_steps(self._h))

    def macro(self):
        """(rho, u): rho shaped (nz, ny, nx), u shaped (nz, ny, nx, 3); NaN on solids."""
        rho = np.zeros(self.N)
        u = np.zeros((self.N, 3))
        self._lib.oracle_macro(self._h, _ptr(rho), _ptr(u))
        return rho.reshape(self.nz, self.ny, self.nx), u.reshape(self.nz, self.ny, self.nx, 3)

    def flux(self):
        return float(self._lib.oracle_flux(self._h))

    def mass(self):
        return float(self._lib.oracle_mass(self._h))

    def permeability(self):
        return float(self._lib.oracle_permeability(self._h))

    def knudsen(self):
        return knudsen(self.tau, self.nx)

    def run_to_steady(self, tol=1e-9, K=100, max_steps=10**6):
        steps = _ll(0)
        resid = _d(0.0)
        rc = self._lib.oracle_run_to_steady(self._h, float(tol), int(K), int(max_steps),
                                            ctypes.byref(steps), ctypes.byref(resid))
        return rc == 0, int(steps.value), float(resid.value)


__all__ = ["Oracle", "lattice", "feq", "collide", "knudsen", "viscosity",
           "intrinsic_permeability", "set_threads", "threads"]
