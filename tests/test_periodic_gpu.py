"""GPU parity of the force-driven, fully periodic case (the paper's 3D
experiment: body force g along x, six periodic faces, permeability by Eq. 2;
forcing of Guo et al. 2002, about which the paper is silent) against the FP64
oracle and against closed forms.

Bars as in the pressure-driven parity tests: FP64 1e-10 relative (plus the
oracle's rounding floor), FP32 1e-4 on k and fields (1e-5 of the largest
deviation after one or a few steps from a random state).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1609_09685_amd import force_driven, lbm
from paper_1609_09685_amd.qsgs import qsgs_2d, qsgs_3d

from lbm_testutil import (field_floor, fields_match, from_oracle_f, random_state, state_view,
                          to_oracle_f)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}


def _pair(Q, mask, precision, tau, g, linear_eq=False, check_every=100):
    s = lbm.Solver(mask, tau, 1.0, 1.0, precision=precision, lattice=Q,
                   check_every=check_every, boundary="periodic", body_force=g)
    if linear_eq:
        s.set_linear_equilibrium(True)
    o = oracle.Oracle(Q, mask, tau, 1.0, 1.0, linear_eq=linear_eq, periodic=True, force=g)
    return s, o


@pytest.mark.parametrize("Q,shape", [
    (9, (1, 2)), (9, (5, 65)), (9, (3, 130)), (9, (4, 3)), (9, (2, 64)),
    (19, (1, 1, 2)), (19, (3, 9, 67)), (19, (2, 1, 129)), (19, (1, 4, 64)), (19, (5, 3, 2)),
])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("linear_eq", [False, True])
def test_edge_shapes_random_state(Q, shape, precision, linear_eq):
    """Tiny, ragged and degenerate periodic domains (one-node-wide faces wrap
    onto themselves) from a seeded random state: wrap in x, y and z, bounce-back
    and the forcing term, one step and five steps."""
    rng = np.random.default_rng(hash(shape) % 1000 + 7)
    mask = (rng.random(shape) < 0.25).astype(np.uint8)
    if mask.all():
        mask.reshape(-1)[0] = 0
    s, o = _pair(Q, mask, precision, 0.7, 2e-4, linear_eq)
    g0 = random_state(s, scale=1e-3, seed=3).cpu().numpy()
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
    # flux (Eq. 2's mean velocity) of the same state: a sum of Q values per
    # fluid node over nx, each within the bound above
    nf, nx = int(fl.sum()), mask.shape[-1]
    assert abs(s.flux() - o.flux()) <= nf * Q * bound / nx


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("linear_eq", [False, True])
def test_d3q19_qsgs_fixed_steps(precision, linear_eq):
    """A porous QSGS medium, ragged in x (64 + 6) and y: k by Eq. 2 and the
    fields (the forcing scheme's velocity) after 400 steps."""
    m = qsgs_3d(70, 21, 13, 0.6, 0)
    s, o = _pair(19, m, precision, 0.6, 1e-5, linear_eq)
    s.step(400)
    o.step(400)
    kg, ko = s.permeability(), o.permeability()
    assert abs(kg - ko) / ko <= TOL[precision], (kg, ko)
    ok, rel = fields_match(s, o, TOL[precision])
    assert ok, rel


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_inertial_regime_vs_oracle(precision):
    """Small viscosity and a large force (tau = 0.51, g = 1e-4, pore Reynolds
    number ~ 8 at steady state): the nonlinear equilibrium and forcing terms
    carry weight; k and fields after 1500 steps."""
    m = force_driven.medium(24, seed=2)
    s, o = _pair(19, m, precision, 0.51, 1e-4)
    s.step(1500)
    o.step(1500)
    kg, ko = s.permeability(), o.permeability()
    assert abs(kg - ko) / ko <= TOL[precision], (kg, ko)
    ok, rel = fields_match(s, o, TOL[precision])
    assert ok, rel


def test_fig5_inertia_and_linear_equilibrium():
    """The paper's 3D finding (its Fig. 5) on a 48^3 medium of the paper's
    porosity: with the full equilibrium, k for the large force falls below k
    for the small one at small Kn (tau = 0.51) and not at tau = 1; with the
    linear equilibrium both forces give the same k at both tau."""
    m = force_driven.medium(48, seed=1)
    rows, info = force_driven.sweep(m, taus=(0.51, 1.0), forces=(1e-6, 1e-4), tol=1e-8)
    assert abs(info["porosity"] - force_driven.POROSITY) <= 1.0 / m.size   # one voxel
    assert all(r["status"] == lbm.LBM_OK for r in rows), rows
    k = {(r["linear"], r["tau"], r["g"]): r["k"] for r in rows}
    ratio = {(lin, tau): k[(lin, tau, 1e-4)] / k[(lin, tau, 1e-6)]
             for lin in (False, True) for tau in (0.51, 1.0)}
    print(ratio)
    assert ratio[(False, 0.51)] < 0.95
    assert abs(ratio[(False, 1.0)] - 1) < 1e-5
    assert abs(ratio[(True, 0.51)] - 1) < 1e-4
    assert abs(ratio[(True, 1.0)] - 1) < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_d2q9_qsgs_run_to_steady(precision):
    m = qsgs_2d(100, 50, 0.74, 0)
    s, o = _pair(9, m, precision, 0.8, 1e-6)
    ok_o, steps_o, _ = o.run_to_steady(1e-9, 100, 200000)
    ok_g, steps_g, _ = s.run_to_steady(1e-9, 200000)
    assert ok_o and ok_g
    if precision == "fp64":
        assert abs(steps_g - steps_o) <= 100
    kg, ko = s.permeability(), o.permeability()
    assert abs(kg - ko) / ko <= max(TOL[precision], 1e-7)


@pytest.mark.parametrize("Q", [9, 19])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("linear_eq", [False, True])
def test_force_driven_channel_closed_form(Q, precision, linear_eq):
    """Channel of H fluid rows between solid rows, periodic elsewhere: Eq. 2
    gives kappa = phi (H^2 - 1 + 8 Lambda)/12, Lambda = (tau - 1/2)^2."""
    H, tau = 8, 0.5 + math.sqrt(3) / 4
    ny = H + 2
    m = np.zeros((ny, 64), np.uint8) if Q == 9 else np.zeros((3, ny, 64), np.uint8)
    m[..., 0, :] = 1
    m[..., -1, :] = 1
    s = lbm.Solver(m, tau, 1.0, 1.0, precision=precision, lattice=Q, boundary="periodic",
                   body_force=1e-6)
    if linear_eq:
        s.set_linear_equilibrium(True)
    ok, _, _ = s.run_to_steady(1e-12 if precision == "fp64" else 1e-7, 400000)
    assert ok
    lam = (tau - 0.5) ** 2
    kcf = (H / ny) * (H * H - 1 + 8 * lam) / 12
    assert abs(s.permeability() - kcf) / kcf <= (1e-9 if precision == "fp64" else 1e-4)


def test_similarity_scaling():
    """The similarity argument of the paper (Eq. 3): in the Stokes regime the
    lattice permeability of a geometry depends only on its shape in lattice
    cells, so resolving the same channel with 10x finer cells multiplies it by
    100 (kappa_2 = 0.01 kappa_1 at the same physical size).  With
    Lambda = 1/8 the bounce-back slip term 8 Lambda - 1 vanishes, so the
    scaling is exact at any H (linear equilibrium, two forces)."""
    tau = 0.5 + math.sqrt(2) / 4
    k = {}
    for H, g in ((6, 1e-5), (60, 1e-7)):
        m = np.zeros((H + 1, 16), np.uint8)
        m[0, :] = 1
        s = lbm.Solver(m, tau, 1.0, 1.0, precision="fp64", lattice=9, boundary="periodic",
                       body_force=g)
        s.set_linear_equilibrium(True)
        ok, _, _ = s.run_to_steady(1e-13, 2000000)
        assert ok
        k[H] = s.permeability() / (H / (H + 1))      # per unit porosity
    assert abs(k[60] / k[6] - 100.0) <= 1e-8, k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_linear_equilibrium_removes_force_dependence(precision):
    """With the linear equilibrium the state is linear in the force (the
    deviation storage scales with it), so k by Eq. 2 does not depend on g; the
    full equilibrium shows the inertia the paper reports at large g.  Both
    agree with the oracle.  The two forces differ by 2^7, so the linear case
    scales every stored value exactly and k agrees to the last bit."""
    m = qsgs_2d(40, 20, 0.7, 5)
    res = {}
    for lin in (True, False):
        ks = []
        for g in (2.0 ** -20, 2.0 ** -13):
            s, o = _pair(9, m, precision, 0.7, g, lin)
            s.step(3000)
            o.step(3000)
            ks.append(s.permeability())
            assert abs(ks[-1] - o.permeability()) / o.permeability() <= TOL[precision]
        res[lin] = abs(ks[1] - ks[0]) / ks[0]
    assert res[True] <= 1e-15, res
    assert res[False] > 1e-6, res


def test_momentum_budget_and_mass():
    """No solids: each step adds exactly F per node, so after t steps from rest
    the flux is (t - 1/2) F ny nz and every node has u_x = (t - 1/2) F; mass
    stays put with solids and force (sum_i F_i = 0)."""
    F = 2e-5
    m = np.zeros((3, 5, 70), np.uint8)
    s = lbm.Solver(m, 0.8, 1.0, 1.0, precision="fp64", lattice=19, boundary="periodic",
                   body_force=F)
    for t in (1, 7, 40):
        s.step(t - s.steps)
        assert abs(s.flux() - (t - 0.5) * F * 15) <= 1e-14
        rho, u = s.macro("float64")
        assert (rho.cpu().numpy() - 1.0).__abs__().max() <= 1e-15
        u = u.cpu().numpy()
        assert np.abs(u[0] - (t - 0.5) * F).max() <= 1e-15
        assert np.abs(u[1:]).max() <= 1e-15
    mq = qsgs_3d(70, 10, 8, 0.7, 4)
    s = lbm.Solver(mq, 0.7, 1.0, 1.0, precision="fp64", lattice=19, boundary="periodic",
                   body_force=1e-4)
    rho0, _ = s.macro("float64")
    mass0 = float(rho0.sum())
    s.step(1500)
    rho, _ = s.macro("float64")
    assert abs(float(rho.sum()) - mass0) / mass0 <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_set_macro_round_trip(precision):
    """lbm_set_macro takes the velocity lbm_get_macro reports (the forcing
    scheme's u), so a state written from fields reads back as those fields."""
    import torch
    m = qsgs_2d(70, 20, 0.7, 2)
    s = lbm.Solver(m, 0.8, 1.0, 1.0, precision=precision, lattice=9, boundary="periodic",
                   body_force=3e-4)
    s.step(200)
    rho, u = s.macro("float32")
    s.set_macro(rho, u)
    rho2, u2 = s.macro("float32")
    fl = torch.from_numpy(~m.astype(bool)).to(rho.device).view(rho.shape)
    tol = 1e-12 if precision == "fp64" else 1e-6
    assert float((rho2 - rho)[fl].abs().max()) <= tol
    assert float((u2 - u)[:, fl].abs().max()) <= tol * 10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_periodic_bitwise(precision):
    """A batch of periodic samples runs to the same steps, flux and k as the
    samples alone (same kernels, same reduction order)."""
    masks = [qsgs_2d(100, 50, p, j) for j, p in enumerate((0.7, 0.8, 0.75))]
    taus = (0.7, 0.9, 1.1)

    def solvers():
        return [lbm.Solver(mk, t, 1.0, 1.0, precision=precision, lattice=9,
                           boundary="periodic", body_force=1e-6) for mk, t in zip(masks, taus)]
    b = lbm.Batch(solvers())
    st, steps, _ = b.run_to_steady(1e-8, 100000)
    kb, kst = b.permeability()
    assert (st == lbm.LBM_OK).all() and (kst == lbm.LBM_OK).all()
    for j, s in enumerate(solvers()):
        ok, n, _ = s.run_to_steady(1e-8, 100000)
        assert ok and n == steps[j]
        assert s.permeability() == kb[j]


def test_batch_rejects_mixed_boundaries():
    a = lbm.Solver(qsgs_2d(64, 20, 0.7, 0), 0.8, 1.0, 1.0, lattice=9, boundary="periodic",
                   body_force=1e-6)
    b = lbm.Solver(qsgs_2d(64, 20, 0.7, 1), 0.8, 1.001, 0.999, lattice=9)
    with pytest.raises(lbm.LBMError):
        lbm.Batch([a, b])


def test_periodic_errors():
    m = qsgs_2d(64, 20, 0.7, 0)
    with pytest.raises(lbm.LBMError):
        lbm.Solver(m, 0.8, 1.001, 0.999, lattice=9, boundary="periodic", body_force=1e-6)
    with pytest.raises(lbm.LBMError):
        lbm.Solver(m, 0.8, 1.001, 0.999, lattice=9, body_force=1e-6)
    s = lbm.Solver(m, 0.8, 1.0, 1.0, lattice=9, boundary="periodic", body_force=1e-6)
    with pytest.raises(lbm.LBMError):
        s.reset("linear")
    z = lbm.Solver(m, 0.8, 1.0, 1.0, lattice=9, boundary="periodic", body_force=0.0)
    z.step(10)
    with pytest.raises(lbm.LBMError):
        z.permeability()
