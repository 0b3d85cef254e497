"""Host logic of the learned warm start (CPU): the step count at which k is
accurate, the gain ratios of an evaluation, the maps between solver fields
and network targets, the mirror factors and the Kn input."""
import math

import numpy as np
import pytest

from paper_1609_09685_amd import lbm, warmstart as ws


def test_steps_to_accuracy():
    """Flux logged after every window of K steps: the count is the end of the
    first window after the last one outside rtol (a late excursion resets it;
    NaN entries past a sample's end are ignored; the sign of the flux does not
    matter)."""
    K = 100
    q_final = np.array([1.0, -2.0, 3.0])
    log = np.full((6, 3), np.nan)
    log[:, 0] = [0.5, 0.9, 1.0002, 1.00005, 0.99999, 1.0]
    log[:4, 1] = [-2.0001, -2.00005, -1.99999, -2.0]
    log[:, 2] = [3.0, 3.0, 3.0, 3.01, 3.0, 3.0]
    got = ws.steps_to_accuracy(log, q_final, np.array([0, 500, 1000]), K)
    assert got.tolist() == [4 * K, 500 + K, 1000 + 5 * K]
    # exactly at the tolerance counts as accurate
    edge = np.array([[1.0 + 1e-4 - 1e-12], [1.0]])
    assert ws.steps_to_accuracy(edge, np.array([1.0]), np.array([0]), K).tolist() == [K]


def test_start_gains():
    """Ratios of sums and of medians and the share of faster samples, over the
    samples every start brought to the residual."""
    ev = {"seeds": [0, 1, 2, 3]}
    ev["zero"] = dict(status=[0, 0, 0, 0], steps=[100, 200, 300, 9],
                      steps_to_k_tol=[10, 20, 30, 1], seconds_to_k_tol=[1.0, 2.0, 3.0, 9.0])
    ev["linear"] = dict(status=[0, 0, 0, 0], steps=[100, 100, 100, 1],
                        steps_to_k_tol=[20, 20, 20, 1], seconds_to_k_tol=[2.0, 2.0, 2.0, 1.0])
    ev["learned"] = dict(status=[0, 0, 0, lbm.LBM_ENOTCONV], steps=[50, 300, 150, 1],
                         steps_to_k_tol=[5, 40, 12, 1], seconds_to_k_tol=[0.5, 4.0, 1.2, 1.0])
    g = ws.start_gains(ev)
    assert g["samples"] == 3
    s = g["steps_to_k_tol"]
    assert s["sum_vs_zero"] == pytest.approx(57 / 60)
    assert s["median_vs_zero"] == pytest.approx(12 / 20)
    assert s["faster_than_zero"] == pytest.approx(2 / 3)
    assert s["sum_vs_linear"] == pytest.approx(57 / 60)
    assert s["median_vs_linear"] == pytest.approx(12 / 20)
    st = g["steps"]
    assert st["sum_vs_zero"] == pytest.approx(500 / 600)
    assert st["median_vs_linear"] == pytest.approx(150 / 100)
    assert st["faster_than_linear"] == pytest.approx(1 / 3)


def test_target_maps():
    """The density target is the deviation from the linear drop between the
    ghost planes (rho_in at x = -1, rho_out at x = nx) in units of drho R; the
    velocity target u nu L / (c_s^2 drho) / U with L = nx + 1; inverse factors
    are reciprocal."""
    taus, nx, U, R = [0.51, 0.8, 1.0], 256, 1.7, 0.13
    shift, slope, fwd, inv = ws.target_maps(taus, nx, (U, R))
    drho = ws.RHO_IN - ws.RHO_OUT
    base = lambda x: shift[:, 0].astype(np.float64) + slope[:, 0] * (x + 1.0)
    assert np.abs(base(-1) - ws.RHO_IN).max() < 1e-7
    assert np.abs(base(nx) - ws.RHO_OUT).max() < 1e-6
    assert (shift[:, 1:] == 0).all() and (slope[:, 1:] == 0).all()
    nu = (np.array(taus) - 0.5) / 3.0
    assert np.allclose(fwd[:, 0], 1.0 / (drho * R), rtol=1e-6)
    assert np.allclose(fwd[:, 1], nu * (nx + 1) / (drho / 3.0) / U, rtol=1e-6)
    assert np.array_equal(fwd[:, 1], fwd[:, 2])
    assert np.allclose(fwd * inv, 1.0, rtol=1e-6)


def test_mirror_factors_compose():
    """The factors of the xy-mirror are those of the x- and the y-mirror
    multiplied (the mirrors commute); every factor is +-1 and the density and
    u_x factors of the y-mirror are +1 (nothing flows across y)."""
    m = dict(ws.MIRRORS)
    assert set(m) == {(1, 0), (0, 1), (1, 1)}
    assert np.array_equal(np.multiply(m[(1, 0)], m[(0, 1)]), m[(1, 1)])
    assert all(abs(v) == 1.0 for f in m.values() for v in f)
    assert m[(1, 0)][:2] == (1.0, 1.0)


def test_kn_input():
    """The second input channel is Kn = sqrt(pi/6)(tau - 1/2)/nx in units of 1e-3."""
    taus = [0.51, 0.75, 1.0]
    want = [math.sqrt(math.pi / 6) * (t - 0.5) / ws.NX / ws.KN_SCALE for t in taus]
    assert np.allclose(ws.features(taus, ws.NX), want, rtol=1e-6)
