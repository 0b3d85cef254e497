"""lbm_flux_noalloc against lbm_flux through the C ABI (GPU).

The no-allocation variant runs the same flux pass and the same fixed-order
FP64 reduction as lbm_flux, with its partials in the library's own scratch
array instead of the context's work buffer, so the two must agree bitwise:
on two calls in a row (the second on a smaller domain, so the scratch holds
the first call's larger set of partials), in both precisions, with a body
force (the half-force offset), and a domain beyond the scratch's limit must
be refused with a clear error.
"""
import numpy as np
import pytest

from paper_1609_09685_amd import lbm
from paper_1609_09685_amd.qsgs import qsgs_2d, qsgs_3d

pytestmark = pytest.mark.gpu


def _bits(x):
    return np.float64(x).view(np.uint64)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_flux_equals_flux(precision):
    big = lbm.Solver(qsgs_3d(128, 96, 80, 0.6, 0), 0.6, 1.00005, 0.99995, precision=precision,
                     lattice=19)
    big.step(37)
    q_ref = big.flux()
    q_new = big.flux_noalloc()
    print("D3Q19 128x96x80", precision, q_ref, q_new)
    assert _bits(q_new) == _bits(q_ref)
    small = lbm.Solver(qsgs_2d(100, 50, 0.74, 0), 0.8, 1.0005, 0.9995, precision=precision)
    small.step(11)
    q_ref2 = small.flux()
    q_new2 = small.flux_noalloc()
    print("D2Q9 100x50", precision, q_ref2, q_new2)
    assert _bits(q_new2) == _bits(q_ref2)
    assert q_new2 != q_new
    # and the larger domain again, after the smaller one
    assert _bits(big.flux_noalloc()) == _bits(q_ref)
    big.close()
    small.close()


def test_noalloc_flux_with_body_force():
    m = qsgs_3d(70, 21, 13, 0.6, 1)
    s = lbm.Solver(m, 0.9, 1.0, 1.0, precision="fp64", lattice=19, boundary="periodic",
                   body_force=1e-5)
    s.step(25)
    assert _bits(s.flux_noalloc()) == _bits(s.flux())
    s.close()


def test_noalloc_flux_refuses_beyond_its_scratch():
    # 8192 x 8200 fluid nodes: more than 2^26 slots
    mask = np.zeros((8200, 8192), np.uint8)
    s = lbm.Solver(mask, 0.8, 1.0005, 0.9995, precision="fp32")
    with pytest.raises(lbm.LBMError) as e:
        s.flux_noalloc()
    assert e.value.status == lbm.LBM_EINVAL
    assert "scratch" in str(e.value)
    assert np.isfinite(s.flux())   # the context is untouched
    s.close()
