"""GPU parity of the two-relaxation-time collision (TRT: even non-equilibrium
halves relax with tau, odd halves with tau- = 1/2 + Lambda/(tau - 1/2)) against
the FP64 oracle and against the channel closed form with the magic parameter
as Lambda, in the pressure-driven and the periodic force-driven case.

Bars: FP64 1e-10 relative (plus the oracle's rounding floor), FP32 1e-4 on k
and fields, 1e-5 of the largest deviation after a few steps from a random
state.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1609_09685_amd import lbm
from paper_1609_09685_amd.qsgs import qsgs_2d, qsgs_3d

from lbm_testutil import (field_floor, fields_match, from_oracle_f, random_state, state_view,
                          to_oracle_f)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}
MAGIC = 3.0 / 16.0


def _pair(Q, mask, precision, tau, magic, periodic=False, g=0.0, linear_eq=False,
          rho=(1.002, 0.998)):
    ri, ro = (1.0, 1.0) if periodic else rho
    kw = dict(boundary="periodic", body_force=g) if periodic else {}
    s = lbm.Solver(mask, tau, ri, ro, precision=precision, lattice=Q, **kw)
    s.set_trt(magic)
    if linear_eq:
        s.set_linear_equilibrium(True)
    o = oracle.Oracle(Q, mask, tau, ri, ro, linear_eq=linear_eq, periodic=periodic,
                      force=g if periodic else 0.0,
                      trt_magic=magic)
    return s, o


@pytest.mark.parametrize("Q,shape", [
    (9, (1, 2)), (9, (5, 65)), (9, (3, 130)), (9, (4, 3)),
    (19, (1, 1, 2)), (19, (3, 9, 67)), (19, (2, 1, 129)), (19, (5, 3, 2)),
])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["pressure", "pressure_linear", "periodic", "periodic_linear"])
def test_edge_shapes_random_state(Q, shape, precision, case):
    rng = np.random.default_rng(hash(shape) % 1000 + 11)
    mask = (rng.random(shape) < 0.25).astype(np.uint8)
    if mask.all():
        mask.reshape(-1)[0] = 0
    periodic = case.startswith("periodic")
    s, o = _pair(Q, mask, precision, 0.7, MAGIC, periodic=periodic,
                 g=2e-4 if periodic else 0.0, linear_eq=case.endswith("linear"))
    g0 = random_state(s, scale=1e-3, seed=5).cpu().numpy()
    o.set_f(to_oracle_f(g0, Q))
    for n in (1, 5):
        s.step(n)
        o.step(n)
        g = state_view(s).cpu().numpy().astype(np.float64)
        go = from_oracle_f(o.get_f(), Q, mask.reshape((1,) * (3 - mask.ndim) + mask.shape).shape)
        fl = ~mask.reshape(go.shape[1:]).astype(bool)
        err = np.abs(g[:, fl] - go[:, fl]).max()
        scale = np.abs(go[:, fl]).max()
        bound = 1e-10 * scale + field_floor(Q, o.steps) if precision == "fp64" else 1e-5 * scale
        assert err <= bound, (n, err, bound)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("periodic", [False, True])
def test_d3q19_qsgs_fixed_steps(precision, periodic):
    m = qsgs_3d(70, 21, 13, 0.6, 0)
    s, o = _pair(19, m, precision, 1.2, MAGIC, periodic=periodic, g=1e-5,
                 rho=(1.00005, 0.99995))
    s.step(400)
    o.step(400)
    kg, ko = s.permeability(), o.permeability()
    assert abs(kg - ko) / ko <= TOL[precision], (kg, ko)
    ok, rel = fields_match(s, o, TOL[precision])
    assert ok, rel


@pytest.mark.parametrize("Q", [9, 19])
@pytest.mark.parametrize("tau", [0.6, 1.0, 2.0])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_channel_closed_form_any_tau(Q, tau, precision):
    """k = phi (H^2 - 1 + 8 Lambda)/12 with the magic parameter as Lambda at
    every tau: force-driven (periodic) and pressure-driven."""
    H = 8
    ny = H + 2
    kcf = (H / ny) * (H * H - 1 + 8 * MAGIC) / 12
    for periodic in (True, False):
        nx = 64
        m = np.zeros((ny, nx), np.uint8) if Q == 9 else np.zeros((3, ny, nx), np.uint8)
        m[..., 0, :] = 1
        m[..., -1, :] = 1
        kw = dict(boundary="periodic", body_force=1e-6) if periodic else {}
        ri, ro = (1.0, 1.0) if periodic else (1.0005, 0.9995)
        s = lbm.Solver(m, tau, ri, ro, precision=precision, lattice=Q, **kw)
        s.set_trt(MAGIC)
        tol = 1e-12 if precision == "fp64" else 1e-7
        ok, _, _ = s.run_to_steady(tol, 400000)
        assert ok
        bar = (1e-9 if periodic else 5e-5) if precision == "fp64" else 1e-4
        assert abs(s.permeability() - kcf) / kcf <= bar, (periodic, s.permeability(), kcf)


def test_porous_medium_tau_independence():
    """Fixed Lambda: k of a porous medium moves by < 2e-3 over tau 0.6-1.5
    (BGK: more than doubles); each value equals the oracle's."""
    m = qsgs_2d(40, 20, 0.7, 5)
    ks = []
    for tau in (0.6, 0.9, 1.5):
        s, o = _pair(9, m, "fp64", tau, MAGIC, periodic=True, g=1e-5, linear_eq=True)
        ok, _, _ = s.run_to_steady(1e-13, 400000)
        ok_o, _, _ = o.run_to_steady(1e-13, 100, 400000)
        assert ok and ok_o
        ks.append(s.permeability())
        assert abs(ks[-1] - o.permeability()) / o.permeability() <= 1e-9
    assert max(ks) - min(ks) <= 2e-3 * ks[0], ks


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_bgk_special_case(precision):
    """magic = 0 is BGK (same kernels, bitwise); magic = (tau - 1/2)^2 gives
    BGK's relaxation through the TRT arithmetic (equal to rounding)."""
    m = qsgs_2d(100, 50, 0.74, 0)
    tau = 0.8
    ref = lbm.Solver(m, tau, 1.0005, 0.9995, precision=precision, lattice=9)
    ref.step(500)
    s = lbm.Solver(m, tau, 1.0005, 0.9995, precision=precision, lattice=9)
    s.set_trt(MAGIC)
    s.set_trt(0.0)
    s.step(500)
    assert s.permeability() == ref.permeability()
    t = lbm.Solver(m, tau, 1.0005, 0.9995, precision=precision, lattice=9)
    t.set_trt((tau - 0.5) ** 2)
    t.step(500)
    assert abs(t.permeability() - ref.permeability()) / ref.permeability() <= (
        1e-12 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("periodic", [False, True])
def test_batch_trt_bitwise(precision, periodic):
    """Samples with different magic parameters in one batch: bitwise equal to
    the samples alone (pressure-driven and force-driven periodic)."""
    masks = [qsgs_2d(100, 50, p, j) for j, p in enumerate((0.7, 0.8, 0.75))]
    taus = (0.7, 0.9, 1.1)
    magics = (3 / 16, 1 / 4, 1 / 12)
    kw = dict(boundary="periodic", body_force=1e-6) if periodic else {}
    ri, ro = (1.0, 1.0) if periodic else (1.0005, 0.9995)

    def solvers():
        out = []
        for mk, t, mg in zip(masks, taus, magics):
            s = lbm.Solver(mk, t, ri, ro, precision=precision, lattice=9, **kw)
            s.set_trt(mg)
            out.append(s)
        return out
    b = lbm.Batch(solvers())
    st, steps, _ = b.run_to_steady(1e-8, 100000)
    kb, kst = b.permeability()
    assert (st == lbm.LBM_OK).all() and (kst == lbm.LBM_OK).all()
    for j, s in enumerate(solvers()):
        ok, n, _ = s.run_to_steady(1e-8, 100000)
        assert ok and n == steps[j]
        assert s.permeability() == kb[j]


def test_batch_rejects_mixed_collision_models():
    a = lbm.Solver(qsgs_2d(64, 20, 0.7, 0), 0.8, 1.0005, 0.9995, lattice=9)
    b = lbm.Solver(qsgs_2d(64, 20, 0.7, 1), 0.8, 1.0005, 0.9995, lattice=9)
    b.set_trt(MAGIC)
    with pytest.raises(lbm.LBMError):
        lbm.Batch([a, b])


def test_batch_refuses_collision_change():
    """Switching a sample between BGK and TRT after the batch was built is an
    error (the batch launches one collision model); changing the magic
    parameter of a TRT sample is not."""
    a = lbm.Solver(qsgs_2d(64, 20, 0.7, 0), 0.8, 1.0005, 0.9995, lattice=9)
    b = lbm.Solver(qsgs_2d(64, 20, 0.7, 1), 0.8, 1.0005, 0.9995, lattice=9)
    a.set_trt(MAGIC)
    b.set_trt(MAGIC)
    batch = lbm.Batch([a, b])
    batch.step(2)
    b.set_trt(0.25)
    batch.step(2)
    b.set_trt(0.0)
    with pytest.raises(lbm.LBMError):
        batch.step(2)


def test_trt_errors():
    s = lbm.Solver(qsgs_2d(64, 20, 0.7, 0), 0.8, 1.0005, 0.9995, lattice=9)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(lbm.LBMError):
            s.set_trt(bad)


# ----------------------------------------- the Lambda -> 0 limit (k_int route)

K_INT_MAGIC = 1e-6   # the magic parameter of the intrinsic-permeability runs


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("Q", [9, 19])
def test_trt_limit_against_oracle(Q, precision):
    """The configuration that gives k_int (the tau -> 1/2 limit of the
    discussion of Figs. 2-3): TRT at tau+ = 1 and Lambda = 1e-6, so that
    tau- = 1/2 + 2e-6 and the odd modes flip sign with a factor -(1 - 8e-6) per
    step, on a QSGS medium in the pressure-driven case, against the oracle at
    equal steps, on k and on the fields."""
    m = qsgs_2d(100, 50, 0.74, 0) if Q == 9 else qsgs_3d(48, 14, 12, 0.6, 3)
    rho = (1.0005, 0.9995) if Q == 9 else (1.00005, 0.99995)
    s, o = _pair(Q, m, precision, 1.0, K_INT_MAGIC, rho=rho)
    steps = 3000 if Q == 9 else 800
    s.step(steps)
    o.step(steps)
    kg, ko = s.permeability(), o.permeability()
    tol = TOL[precision]
    if precision == "fp64":
        # The oracle keeps f ~ w_i (binary64), so every node's momentum carries
        # ~Q ulp(1) of rounding per step; with tau- this close to 1/2 the odd
        # modes hardly decay and these errors add up like a random walk
        # (field_floor).  Relative to the mean momentum per fluid node, averaged
        # over the fluid nodes, that is the oracle's own floor on k.
        n_fluid = int((m == 0).sum())
        j_mean = abs(o.flux()) * o.nx / n_fluid
        tol += field_floor(Q, steps) / (j_mean * math.sqrt(n_fluid))
    assert abs(kg - ko) / ko <= tol, (kg, ko, tol)
    ok, rel = fields_match(s, o, TOL[precision])
    assert ok, rel


def test_trt_limit_independent_of_tau_plus():
    """In the pressure-driven case the steady TRT permeability at Lambda = 1e-6
    hardly moves with tau+ (0.8, 1, 1.5): the bounce-back walls sit where Lambda
    puts them, and what is left is the tau dependence of the pressure boundary
    (non-equilibrium extrapolation), a few 1e-4 on this medium.  So k_int does
    not hinge on the choice tau+ = 1."""
    m = qsgs_2d(100, 50, 0.74, 0)
    ks = []
    for tp in (0.8, 1.0, 1.5):
        s = lbm.Solver(m, tp, 1.0005, 0.9995, precision="fp64", lattice=9)
        s.set_trt(K_INT_MAGIC)
        ok, steps, _ = s.run_to_steady(1e-9, 3_000_000, raise_on_notconv=False)
        assert ok, (tp, steps)
        ks.append(s.permeability())
        s.close()
    spread = (max(ks) - min(ks)) / np.mean(ks)
    print("k(Lambda = 1e-6) for tau+ = 0.8, 1, 1.5:", ks, "spread", spread)
    assert spread <= 5e-4, ks
