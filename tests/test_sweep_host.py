"""Host logic of the experiment sweeps (no GPU): run lists and the collapse
metric of the three-resolution tau sweep, and the refined media."""
import numpy as np

from paper_1609_09685_amd import force_driven, tau_sweep


def test_taus_for_gives_equal_kn_runs():
    for r in tau_sweep.REFINE:
        taus = tau_sweep.taus_for(r)
        assert taus == sorted(set(taus))
        for t in tau_sweep.TAUS:
            assert round(t, 9) in taus
        for d in tau_sweep.KN_STEPS:
            assert round(0.5 + r * d, 9) in taus


def test_collapse_metric():
    """A k/k_int that depends on Kn alone has no spread at equal Kn; one that
    depends on tau alone has none at equal tau."""
    def rows(f):
        return [dict(refine=r, tau=t, k_norm=f(r, t)) for r in tau_sweep.REFINE
                for t in tau_sweep.taus_for(r)]
    c = tau_sweep.collapse(rows(lambda r, t: 1 + 3 * (t - 0.5) / r))
    assert c["max_spread_equal_kn"] < 1e-12 and c["max_spread_equal_tau"] > 0.5
    c = tau_sweep.collapse(rows(lambda r, t: 1 + 3 * (t - 0.5)))
    assert c["max_spread_equal_tau"] < 1e-12 and c["max_spread_equal_kn"] > 0.5
    # runs that did not finish are left out
    rs = rows(lambda r, t: 1.0)
    rs[0]["k_norm"] = None
    c = tau_sweep.collapse(rs)
    assert c["max_spread_equal_kn"] == 0.0


def test_refined_media_are_one_structure():
    m1, m2, m3 = tau_sweep.media(40, 20, seed=2)
    assert m2.shape == (40, 80) and m3.shape == (60, 120)
    assert (m2[::2, ::2] == m1).all() and (m3[1::3, 2::3] == m1).all()
    assert m1.mean() == m2.mean() == m3.mean()


def test_force_driven_medium():
    m = force_driven.medium(24, seed=1)
    assert m.shape == (24, 24, 24)
    assert abs((1 - m.mean()) - force_driven.POROSITY) <= 1.0 / m.size
