"""The paper's 2D finding (its Figs. 2 and 3) on a reduced structure: one
100x50 QSGS medium refined 2x and 3x.  k/k_int (k_int: the Lambda -> 0 limit
by TRT) differs strongly between resolutions at equal tau and much less at
equal Kn = sqrt(pi/6)(tau - 1/2)/N_x; on the finest grid it approaches 1 as
tau -> 1/2."""
import pytest

from paper_1609_09685_amd import lbm, tau_sweep

pytestmark = pytest.mark.gpu


def test_collapse_against_kn():
    masks = tau_sweep.media(100, 50, seed=3)
    taus, steps = (0.6, 1.0, 1.5), (0.05, 0.1, 0.25)
    rows = tau_sweep.sweep(masks, tau_sweep.REFINE, taus, steps, tol=1e-9, log=print)
    assert all(r["status"] == lbm.LBM_OK for r in rows), [r for r in rows if r["status"]]
    c = tau_sweep.collapse(rows, taus, steps)
    print(c)
    assert c["spread_equal_tau"][1.5] > 2.0 * c["spread_equal_kn"][0.25]
    assert c["max_spread_equal_tau"] > 2.0 * c["max_spread_equal_kn"]
    fine = sorted((r["tau"], r["k_norm"]) for r in rows if r["refine"] == 3)
    assert abs(fine[0][1] - 1.0) < 0.05, fine
