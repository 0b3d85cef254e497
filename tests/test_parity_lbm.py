"""GPU parity: the HIP solver against the FP64 CPU oracle, through the C ABI.

Bars (per result): FP64 storage 1e-10 relative, FP32 deviation storage 1e-4
relative, on the permeability and on the velocity field (max norm relative to
max |u|), at equal step counts; converged step counts within one check window.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1609_09685_amd import lbm
from paper_1609_09685_amd.qsgs import qsgs_2d, qsgs_3d

from lbm_testutil import (compact_view, field_floor, fields_match, from_oracle_f, random_state,
                          state_view, to_oracle_f)

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}
# One step from a random state: relative to the largest population deviation
# in the window (FP32: a few ulps of the stored values).
TOL1 = {"fp64": 1e-10, "fp32": 2e-6}
C1 = dict(tau=0.8, rho_in=1.0005, rho_out=0.9995)


def _pair(Q, mask, precision, tau, rho_in, rho_out, start="uniform", check_every=100):
    s = lbm.Solver(mask, tau, rho_in, rho_out, precision=precision,
                   lattice=Q, check_every=check_every)
    o = oracle.Oracle(Q, mask, tau, rho_in, rho_out, start=start)
    if start != "uniform":
        s.reset(start)
    return s, o


@pytest.fixture(scope="module")
def c1_mask():
    return qsgs_2d(100, 50, 0.74, 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_fixed_steps(c1_mask, precision):
    s, o = _pair(9, c1_mask, precision, **C1)
    s.step(3000)
    o.step(3000)
    assert s.steps == o.steps == 3000
    kg, ko = s.permeability(), o.permeability()
    assert abs(kg - ko) / ko <= TOL[precision]
    ok, rel = fields_match(s, o, TOL[precision])
    assert ok, rel


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_run_to_steady(c1_mask, precision):
    s, o = _pair(9, c1_mask, precision, **C1)
    ok_o, steps_o, _ = o.run_to_steady(1e-9, 100, 200000)
    ok_g, steps_g, res_g = s.run_to_steady(1e-9, 200000)
    assert ok_o and ok_g and res_g < 1e-9
    if precision == "fp64":
        assert abs(steps_g - steps_o) <= 100
    # FP32 storage: the flux moves by ~1e-7/sqrt(fluid nodes) per step from
    # rounding, the size of a 1e-9 residual here, and the rounded map settles on
    # its own fixed point; the stopping step is reported, and the converged k is
    # held to the FP32 bar below.
    kg, ko = s.permeability(), o.permeability()
    if steps_g == steps_o:
        assert abs(kg - ko) / ko <= TOL[precision]
    # at equal step counts
    s2, o2 = _pair(9, c1_mask, precision, **C1)
    s2.step(steps_o)
    assert abs(s2.permeability() - ko) / ko <= TOL[precision]
    # converged k of both runs
    assert abs(kg - ko) / ko <= max(TOL[precision], 1e-7)
    print(f"C1 {precision}: steps gpu {steps_g} oracle {steps_o}, k gpu {kg:.10e} "
          f"oracle {ko:.10e} rel {abs(kg - ko) / ko:.2e}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_d3q19_qsgs(precision):
    m = qsgs_3d(70, 21, 13, 0.6, 0)    # ragged in x (64 + 6) and y (5 tiles of 4 + 1)
    s, o = _pair(19, m, precision, 0.6, 1.00005, 0.99995)
    s.step(400)
    o.step(400)
    kg, ko = s.permeability(), o.permeability()
    assert abs(kg - ko) / ko <= TOL[precision]
    ok, rel = fields_match(s, o, TOL[precision])
    assert ok, rel


@pytest.mark.parametrize("Q,shape", [
    (9, (1, 2)), (9, (5, 65)), (9, (3, 130)), (9, (7, 64)), (9, (4, 3)),
    (19, (1, 1, 2)), (19, (3, 9, 67)), (19, (70, 5, 5)), (19, (2, 1, 129)), (19, (1, 4, 64)),
])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_edge_shapes_random_state(Q, shape, precision):
    """Tiny, ragged and degenerate domains from a seeded random state: every
    boundary rule (mirror, bounce-back, ghost, corners) is exercised."""
    rng = np.random.default_rng(hash(shape) % 1000)
    mask = (rng.random(shape) < 0.25).astype(np.uint8)
    if mask.ndim == 3 and Q == 9:
        mask = mask[0]
    if mask.all():
        mask.reshape(-1)[0] = 0
    s, o = _pair(Q, mask, precision, 0.7, 1.002, 0.998)
    g0 = random_state(s, scale=1e-3, seed=1).cpu().numpy()
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


@pytest.mark.parametrize("Q", [9, 19])
def test_rest_state_bitwise(Q):
    m = qsgs_2d(100, 50, 0.74, 1) if Q == 9 else qsgs_3d(40, 24, 20, 0.6, 1)
    s = lbm.Solver(m, 0.8, 1.0, 1.0, precision="fp32")
    s.step(1000)
    v = compact_view(s)
    assert int((v != 0).sum()) == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_closed_box_mass(precision):
    m = qsgs_2d(96, 40, 0.7, 3, percolate=False).copy()
    m[:, 0] = m[:, -1] = 1
    s = lbm.Solver(m, 0.7, 1.01, 0.99, precision=precision)
    g0 = random_state(s, scale=1e-2, seed=2)
    m0 = float(g0.double().sum())
    steps = 2000
    s.step(steps)
    m1 = float(state_view(s).double().sum())
    n_fluid = int((m == 0).sum())
    eps = 2.2e-16 if precision == "fp64" else 1.2e-7
    # The deviations sum to the mass change.  Each stored value is rounded once
    # per step; those errors walk like sqrt(Q * steps * nodes) times eps times
    # the population scale.  A leaking boundary would lose ~1e-3 per step.
    scale = float(g0.abs().max())
    assert abs(m1 - m0) <= 10 * eps * scale * math.sqrt(9 * steps * n_fluid)


@pytest.mark.parametrize("Q,shape", [(9, (50, 100)), (19, (9, 13, 300)), (19, (5, 7, 40))])
def test_padding_slots_stay_zero(Q, shape):
    """Slots that belong to no fluid node (segment padding) are written as zero."""
    import torch
    rng = np.random.default_rng(4)
    m = (rng.random(shape) < 0.35).astype(np.uint8)
    s = lbm.Solver(m, 0.7, 1.002, 0.998, precision="fp32", lattice=Q)
    random_state(s, scale=1e-3, seed=3)
    s.step(7)
    c = compact_view(s)
    used = torch.zeros(c.shape[1], dtype=torch.bool, device=c.device)
    sm = s.slot_map().view(-1)
    used[sm[sm >= 0].long()] = True
    assert int(used.sum()) == int((m == 0).sum())
    assert bool((c[:, ~used] == 0).all())
    slots = sm[sm >= 0]
    assert int(slots.unique().numel()) == int(slots.numel())   # one slot per fluid node


def test_checkpoint_restore_bitwise(c1_mask):
    s = lbm.Solver(c1_mask, **C1, precision="fp32")
    s.step(500)
    ck = s.get_populations().clone()
    s.step(500)
    a = s.get_populations().clone()
    s.set_populations(ck)
    s.step(500)
    b = s.get_populations()
    assert bool((a == b).all())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("linear_eq", [False, True])
def test_linear_start_and_set_macro(c1_mask, precision, linear_eq):
    """Linear-density start, then a start from fields (the equilibrium of the
    oracle's fields, in the model's own equilibrium: full or linear)."""
    import torch
    s, o = _pair(9, c1_mask, precision, **C1, start="linear")
    if linear_eq:
        s.set_linear_equilibrium(True)
        o = oracle.Oracle(9, c1_mask, **C1, start="linear", linear_eq=True)
    s.step(700)
    o.step(700)
    assert abs(s.permeability() - o.permeability()) / abs(o.permeability()) <= TOL[precision]
    # warm start from fields: equilibrium of the oracle's fields at step 700
    rho, u = o.macro()
    rho_f = np.nan_to_num(rho, nan=1.0).astype(np.float32)
    u_f = np.nan_to_num(np.moveaxis(u[..., :2], -1, 0), nan=0.0).astype(np.float32)
    s.set_macro(torch.from_numpy(rho_f), torch.from_numpy(u_f))
    o2 = oracle.Oracle(9, c1_mask, **C1, linear_eq=linear_eq)
    o2.init_fields(rho_f.astype(np.float64), np.moveaxis(u_f, 0, -1).astype(np.float64))
    s.step(300)
    o2.step(300)
    assert abs(s.permeability() - o2.permeability()) / abs(o2.permeability()) <= TOL[precision]


@pytest.mark.parametrize("Q", [9, 19])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_poiseuille_closed_form_gpu(Q, precision):
    H, tau = 8, 0.8
    prof = np.zeros(H + 2, np.uint8)
    prof[0] = prof[-1] = 1
    mask = np.repeat(prof[:, None], 64, axis=1) if Q == 9 else \
        np.repeat(prof[None, :, None], 48, axis=2)
    s = lbm.Solver(mask, tau, 1.0005, 0.9995, precision=precision, lattice=Q)
    ok, _, _ = s.run_to_steady(1e-10 if precision == "fp64" else 1e-7, 400000)
    assert ok
    k = s.permeability()
    kcf = (H / (H + 2)) * (H * H - 1 + 8 * (tau - 0.5) ** 2) / 12
    assert abs(k - kcf) / kcf <= (5e-5 if precision == "fp64" else 1e-4)


def test_no_flow_and_nonfinite():
    import torch
    solid = np.ones((8, 70), np.uint8)
    s2 = lbm.Solver(solid, 0.8, 1.001, 0.999, precision="fp64")
    s2.step(10)
    with pytest.raises(lbm.LBMError) as e:
        s2.permeability()
    assert e.value.status == lbm.LBM_ENOFLOW
    s = lbm.Solver(np.zeros((8, 70), np.uint8), 0.8, 1.001, 0.999, precision="fp64")
    s.step(10)
    buf = s.get_populations()
    buf.view(torch.float64)[5] = float("nan")   # direction 0 of fluid node (0, 0, 5)
    s.set_populations(buf)
    with pytest.raises(lbm.LBMError) as e:
        s.run_to_steady(1e-9, 1000)
    assert e.value.status == lbm.LBM_ENONFINITE


def test_fluid_count_checked_at_init(c1_mask):
    import ctypes
    import torch
    lib = lbm.load_library()
    nf = int((c1_mask == 0).sum())
    g = lbm.Geom(9, 100, 50, 1, lbm.LBM_FP32, 100, 1.0, nf + 1)
    fb, wb = lbm.query_sizes(9, 100, 50, 1, nf + 1)
    f0 = torch.empty(fb, dtype=torch.uint8, device="cuda")
    f1 = torch.empty(fb, dtype=torch.uint8, device="cuda")
    wk = torch.empty(wb, dtype=torch.uint8, device="cuda")
    mk = torch.from_numpy(c1_mask.reshape(-1).copy()).cuda()
    b = lbm.Buffers()
    b.f[0], b.f[1], b.mask, b.work = f0.data_ptr(), f1.data_ptr(), mk.data_ptr(), wk.data_ptr()
    b.stream = torch.cuda.current_stream().cuda_stream
    h = ctypes.c_void_p(0)
    st = lib.lbm_init(ctypes.byref(h), ctypes.byref(g), ctypes.byref(b), 0.8, 1.0005, 0.9995)
    assert st == lbm.LBM_EINVAL and b"fluid" in lib.lbm_last_error()
    assert not h.value


LAUNCH_CONFIGS = [dict(band=0, xcd_remap=0), dict(band=0, xcd_remap=1), dict(band=0, xcd_remap=2),
                  dict(band=0, xcd_remap=3), dict(band=1), dict(band=3), dict(band=64)]


@pytest.mark.parametrize("cfg", LAUNCH_CONFIGS, ids=lambda c: "-".join(f"{k}{v}" for k, v in c.items()))
def test_launch_options_are_bitwise_neutral(c1_mask, cfg):
    """Tile order, shape, runs and cache hints change which wave runs a node,
    not its arithmetic: populations, flux and convergence are bit-identical."""
    for prec in ("fp32", "fp64"):
        a = lbm.Solver(c1_mask, **C1, precision=prec)
        b = lbm.Solver(c1_mask, **C1, precision=prec)
        b.configure(**cfg)
        a.step(300)
        b.step(300)
        assert bool((a.get_populations() == b.get_populations()).all())
        assert a.flux() == b.flux()
        assert a.run_to_steady(1e-9, 50000)[1:] == b.run_to_steady(1e-9, 50000)[1:]


@pytest.mark.parametrize("cfg", [dict(band=0, xcd_remap=0), dict(band=0, xcd_remap=2),
                                 dict(band=0, xcd_remap=4), dict(band=2), dict(band=1), dict(band=7)])
def test_launch_options_3d(cfg):
    m = qsgs_3d(130, 9, 7, 0.6, 3)
    a = lbm.Solver(m, 0.6, 1.00005, 0.99995, precision="fp32")
    b = lbm.Solver(m, 0.6, 1.00005, 0.99995, precision="fp32")
    b.configure(**cfg)
    a.step(50)
    b.step(50)
    assert bool((a.get_populations() == b.get_populations()).all())


def test_not_converged_status(c1_mask):
    s = lbm.Solver(c1_mask, **C1, precision="fp32")
    ok, steps, r = s.run_to_steady(1e-9, 300, raise_on_notconv=False)
    assert not ok and steps == 300 and r > 1e-9


# ----------------------------------------------------------- full-size checks


def _sampled_one_step(s, Q, mask, precision, n_samples, seed):
    """One step from a seeded random state; compare sampled nodes (and their
    neighbourhoods' boundary cases) against the oracle run on the 3x3(x3)
    window around each node, which holds every value the node pulls."""
    rng = np.random.default_rng(seed)
    random_state(s, scale=1e-4, seed=seed)
    before = state_view(s).clone()
    s.step(1)
    after = state_view(s)
    m3 = mask.reshape((1,) * (3 - mask.ndim) + mask.shape)
    nz, ny, nx = m3.shape
    pts = [(z, y, x) for z, y, x in zip(rng.integers(0, nz, n_samples), rng.integers(0, ny, n_samples),
                                        rng.integers(0, nx, n_samples))]
    # boundary nodes: corners and face centres
    for z in {0, nz - 1}:
        for y in {0, ny - 1}:
            for x in {0, nx - 1}:
                pts.append((z, y, x))
    pts += [(nz // 2, ny // 2, 0), (nz // 2, ny // 2, nx - 1), (0, ny // 2, nx // 2),
            (nz // 2, 0, nx // 2)]
    checked = 0
    worst = 0.0
    for z, y, x in pts:
        if m3[z, y, x]:
            continue
        zs, ys, xs = (slice(max(0, a - 1), min(n, a + 2)) for a, n in ((z, nz), (y, ny), (x, nx)))
        win_mask = m3[zs, ys, xs]
        gw = before[:, zs, ys, xs].double().cpu().numpy()
        o = oracle.Oracle(Q, win_mask if Q == 19 else win_mask[0], s.tau, s.rho_in, s.rho_out)
        o.set_f(to_oracle_f(gw, Q))
        o.step(1)
        go = from_oracle_f(o.get_f(), Q, win_mask.shape)
        cz, cy, cx = z - zs.start, y - ys.start, x - xs.start
        ref = go[:, cz, cy, cx]
        got = after[:, z, y, x].double().cpu().numpy()
        scale = np.abs(gw).max()
        err = np.abs(got - ref).max()
        worst = max(worst, err / (TOL1[precision] * scale + (field_floor(Q, 1) if precision == "fp64" else 0.0)))
        checked += 1
    assert checked >= n_samples // 3
    return worst


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_full_size_2d_400x200_sampled(precision):
    m = qsgs_2d(400, 200, 0.74, 0)
    s = lbm.Solver(m, 0.6, 1.0005, 0.9995, precision=precision)
    worst = _sampled_one_step(s, 9, m, precision, 300, 4)
    assert worst <= 1.0


def test_full_size_3d_512_sampled():
    """The benchmark's workload (512^3 D3Q19, FP32 deviations, tau 0.6) in the
    launch configuration the benchmark times."""
    m = qsgs_3d(512, 512, 512, 0.6, 0)
    s = lbm.Solver(m, 0.6, 1.00005, 0.99995, precision="fp32")
    worst = _sampled_one_step(s, 19, m, "fp32", 300, 5)
    assert worst <= 1.0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_smooth_is_mean_of_consecutive_states(precision):
    """lbm_smooth(1) from a random state equals the mean of the oracle's state
    and its state one step later (populations of every fluid node)."""
    mask = qsgs_2d(130, 37, 0.7, 4)
    s, o = _pair(9, mask, precision, 0.7, 1.002, 0.998)
    g0 = random_state(s, scale=1e-3, seed=5).cpu().numpy()
    o.set_f(to_oracle_f(g0, 9))
    f0 = o.get_f()
    o.step(1)
    ref = from_oracle_f(0.5 * (f0 + o.get_f()), 9, (1,) + mask.shape)
    s.smooth(1)
    assert s.steps == 1
    g = state_view(s).cpu().numpy().astype(np.float64)
    fl = ~mask.astype(bool)
    err = np.abs(g[:, 0][:, fl] - ref[:, 0][:, fl]).max()
    scale = np.abs(ref[:, 0][:, fl]).max()
    bound = 1e-10 * scale + field_floor(9, 1) if precision == "fp64" else 1e-5 * scale
    assert err <= bound, (err, bound)


def test_smooth_removes_trapped_oscillation():
    """Velocity noise excites modes that alternate every step and never decay
    (momentum trapped in dead-end pores); from such a start the run converges
    to a shifted flux.  Two smoothing passes remove them."""
    import torch
    mask = qsgs_2d(128, 64, 0.65, 20012)
    ref = lbm.Solver(mask, 0.68, 1.0005, 0.9995, precision="fp64")
    ref.run_to_steady(1e-9, 400000)
    k0 = ref.permeability()
    rho, u = ref.macro("float32")
    gen = torch.Generator(device="cuda").manual_seed(0)
    noisy = (u + 1e-4 * torch.randn(u.shape, device="cuda", generator=gen)).contiguous()
    shifted = []
    for passes in (0, 2):
        s = lbm.Solver(mask, 0.68, 1.0005, 0.9995, precision="fp64")
        s.set_macro(rho.contiguous(), noisy)
        s.smooth(passes)
        s.run_to_steady(1e-9, 400000)
        q0 = s.flux()
        s.step(1)
        one_step = abs(s.flux() - q0) / abs(q0)
        shifted.append((abs(s.permeability() - k0) / k0, one_step))
    assert shifted[0][0] > 1e-4 and shifted[0][1] > 1e-5, shifted   # the trap is real
    assert shifted[1][0] < 1e-6 and shifted[1][1] < 1e-8, shifted   # and removed


@pytest.mark.parametrize("Q,shape", [
    (9, (1, 2)), (9, (5, 65)), (9, (3, 130)),
    (19, (1, 1, 2)), (19, (3, 9, 67)), (19, (70, 5, 5)),
])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_linear_equilibrium_pressure_random_state(Q, shape, precision):
    """The linear ("Stokes") equilibrium in the pressure-driven case (ghost
    planes, mirrors, bounce-back) from a seeded random state, element by
    element after one and five steps."""
    rng = np.random.default_rng(hash(shape) % 1000 + 3)
    mask = (rng.random(shape) < 0.25).astype(np.uint8)
    if mask.ndim == 3 and Q == 9:
        mask = mask[0]
    if mask.all():
        mask.reshape(-1)[0] = 0
    s = lbm.Solver(mask, 0.7, 1.002, 0.998, precision=precision, lattice=Q)
    s.set_linear_equilibrium(True)
    o = oracle.Oracle(Q, mask, 0.7, 1.002, 0.998, linear_eq=True)
    g0 = random_state(s, scale=1e-3, seed=2).cpu().numpy()
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
def test_linear_equilibrium_pressure_qsgs(c1_mask, precision):
    """C1 medium with the linear equilibrium: k and fields after 3000 steps."""
    s = lbm.Solver(c1_mask, 0.8, 1.0005, 0.9995, precision=precision, lattice=9)
    s.set_linear_equilibrium(True)
    o = oracle.Oracle(9, c1_mask, 0.8, 1.0005, 0.9995, linear_eq=True)
    s.step(3000)
    o.step(3000)
    kg, ko = s.permeability(), o.permeability()
    assert abs(kg - ko) / ko <= TOL[precision], (kg, ko)
    ok, rel = fields_match(s, o, TOL[precision])
    assert ok, rel


@pytest.mark.parametrize("Q", [9, 19])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["pressure", "periodic"])
def test_wide_offsets_bitwise(Q, precision, case):
    """The 64-bit-offset step kernels (used when a direction group passes
    4 GiB) give the same bits as the 32-bit ones, single and batched."""
    import torch
    mask = qsgs_2d(130, 37, 0.7, 4) if Q == 9 else qsgs_3d(70, 21, 13, 0.6, 1)
    kw = dict(boundary="periodic", body_force=1e-5) if case == "periodic" else {}
    ri, ro = (1.0, 1.0) if case == "periodic" else (1.0005, 0.9995)

    def solver(wide):
        s = lbm.Solver(mask, 0.7, ri, ro, precision=precision, lattice=Q, **kw)
        if wide:
            s.set_wide_offsets(True)
        return s
    a, b = solver(False), solver(True)
    for s in (a, b):
        s.step(150)
    assert torch.equal(a.get_populations(), b.get_populations())
    assert a.flux() == b.flux()
    oka, na, _ = a.run_to_steady(1e-6, 20000)
    okb, nb, _ = b.run_to_steady(1e-6, 20000)
    assert oka and okb and na == nb and a.permeability() == b.permeability()
    # batched: both forms, same bits; mixing them in one batch is refused
    ba = lbm.Batch([solver(False), solver(False)])
    bb = lbm.Batch([solver(True), solver(True)])
    ba.step(40)
    bb.step(40)
    assert (ba.flux() == bb.flux()).all()
    with pytest.raises(lbm.LBMError):
        lbm.Batch([solver(False), solver(True)])


# FP32 deviation storage against FP64 at steady state on C2's 400x200 medium
# (seed 0): within the 1e-4 bar from tau = 0.55 up; at tau = 0.51 the FP32 map
# settles on its own fixed point about 1.5e-4 away (not a stopping effect:
# 2e5 more steps or a 1e-11 residual do not move it; the same for density
# drops 1e-4 .. 1e-2 and any deviation reference rho0), the FP32 limit near
# tau = 1/2 that the design notes record.
@pytest.mark.parametrize("tau,bar", [(0.51, 2e-4), (0.55, 1e-4), (0.6, 1e-4)])
def test_fp32_tracks_fp64_near_tau_half(tau, bar):
    m = qsgs_2d(400, 200, 0.74, 0)
    ks = {}
    for precision in ("fp64", "fp32"):
        s = lbm.Solver(m, tau, 1.0005, 0.9995, precision=precision)
        ok, steps, _ = s.run_to_steady(1e-9, 2_000_000)
        assert ok
        ks[precision] = s.permeability()
        s.close()
    rel = abs(ks["fp32"] - ks["fp64"]) / ks["fp64"]
    print(f"tau {tau}: k fp64 {ks['fp64']:.10f} fp32 {ks['fp32']:.10f} rel {rel:.2e}")
    assert rel <= bar, ks
