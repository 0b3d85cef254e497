"""Seeded QSGS porous masks (the paper's "randomly generated quartet structure").

Input generator only: it holds none of the lattice Boltzmann arithmetic, and
both the GPU solver and the CPU checker consume the masks it writes.  The
growth itself runs in ``csrc/qsgs.cpp`` (host C++, OpenMP, counter-based
random numbers, so a mask depends only on its arguments).

Masks are ``uint8`` arrays, 1 = solid: shape ``(ny, nx)`` in 2D and
``(nz, ny, nx)`` in 3D, x fastest.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.QSGS_LIB
        if not os.path.exists(path):
            _build.build_qsgs()
        lib = ctypes.CDLL(path)
        lib.qsgs_generate.restype = ctypes.c_int
        lib.qsgs_generate.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_int)]
        lib.qsgs_percolates.restype = ctypes.c_int
        lib.qsgs_percolates.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p]
        lib.qsgs_open_fluid.restype = ctypes.c_int
        lib.qsgs_open_fluid.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


class QSGSError(RuntimeError):
    pass


def _generate(dim, nx, ny, nz, porosity, probs, seed, percolate, max_attempts):
    lib = _load()
    out = np.zeros((nz, ny, nx), np.uint8)
    p = np.ascontiguousarray(probs, np.float64)
    att = ctypes.c_int(0)
    rc = lib.qsgs_generate(dim, nx, ny, nz, float(porosity), p.ctypes.data, int(seed),
                           int(bool(percolate)), int(max_attempts), out.ctypes.data,
                           ctypes.byref(att))
    if rc != 0:
        raise QSGSError({-1: "invalid arguments", -2: "growth cannot reach the porosity",
                         -3: "no percolating mask within max_attempts"}.get(rc, str(rc)))
    return out, att.value


def qsgs_2d(nx, ny, porosity, seed, p_core=0.01, p_face=0.1, p_diag=0.025,
            percolate=True, max_attempts=64, return_attempts=False):
    """2D QSGS mask of shape (ny, nx): cores with probability p_core, growth to the
    4 face neighbours with p_face and to the 4 diagonal neighbours with p_diag."""
    m, a = _generate(2, nx, ny, 1, porosity, [p_core, p_face, p_diag, 0.0], seed,
                     percolate, max_attempts)
    m = m[0]
    return (m, a) if return_attempts else m


def qsgs_3d(nx, ny, nz, porosity, seed, p_core=0.01, p_face=0.1, p_edge=0.025, p_vertex=0.0,
            percolate=True, max_attempts=64, return_attempts=False):
    """3D QSGS mask of shape (nz, ny, nx): growth to 6 face, 12 edge and 8 vertex
    neighbours with p_face, p_edge and p_vertex."""
    m, a = _generate(3, nx, ny, nz, porosity, [p_core, p_face, p_edge, p_vertex], seed,
                     percolate, max_attempts)
    return (m, a) if return_attempts else m


def percolates(mask):
    """True if the fluid phase connects x = 0 to x = nx-1 along lattice links."""
    m = np.ascontiguousarray(mask, np.uint8)
    dim = 2 if m.ndim == 2 else 3
    m3 = m if m.ndim == 3 else m[None]
    nz, ny, nx = m3.shape
    return bool(_load().qsgs_percolates(dim, nx, ny, nz, m3.ctypes.data))


def open_fluid(mask):
    """uint8 array of the mask's shape: 1 for fluid nodes connected along lattice
    links to a fluid node of the x = 0 or x = nx-1 plane, 0 elsewhere (solids and
    closed pockets, where the steady velocity is exactly zero)."""
    m = np.ascontiguousarray(mask, np.uint8)
    dim = 2 if m.ndim == 2 else 3
    m3 = m if m.ndim == 3 else m[None]
    nz, ny, nx = m3.shape
    out = np.zeros_like(m3)
    if _load().qsgs_open_fluid(dim, nx, ny, nz, m3.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("bad mask")
    return out.reshape(m.shape)
