"""Batched solver: per-sample results bitwise equal to single-domain runs.

The batch advances every sample with one launch per step (and, by default,
replays each check window as a HIP graph); each sample's populations, step
count, residual and permeability must be exactly those of the same sample run
alone through Solver, which the parity tests hold to the oracle.  One batch
sample is also checked against the oracle directly.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1609_09685_amd import lbm
from paper_1609_09685_amd.qsgs import qsgs_2d, qsgs_3d

pytestmark = pytest.mark.gpu

RHO = dict(rho_in=1.0005, rho_out=0.9995)


def _masks_2d():
    # uneven sizes: one bitmap word, a ragged segment tail, several segments
    shapes = [(100, 50), (64, 9), (130, 37), (300, 21), (257, 80)]
    return [qsgs_2d(nx, ny, 0.74, 11 + j) for j, (nx, ny) in enumerate(shapes)]


def _singles(masks, taus, precision, **kw):
    return [lbm.Solver(m, t, precision=precision, **RHO, **kw) for m, t in zip(masks, taus)]


def _bytes(s):
    return s.get_populations().cpu().numpy()


@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_run_to_steady_bitwise(precision, graph):
    masks = _masks_2d()
    taus = [0.8, 0.6, 1.0, 0.7, 0.9]   # different convergence times: samples retire apart
    alone = _singles(masks, taus, precision)
    ref = [s.run_to_steady(1e-9, 60000, raise_on_notconv=False) for s in alone]
    b = lbm.Batch.from_masks(masks, taus, RHO["rho_in"], RHO["rho_out"], precision=precision,
                             graph=graph)
    status, steps, resid = b.run_to_steady(1e-9, 60000)
    k, kst = b.permeability()
    for j, s in enumerate(alone):
        ok, st, r = ref[j]
        assert status[j] == (lbm.LBM_OK if ok else lbm.LBM_ENOTCONV)
        assert steps[j] == st == b.solvers[j].steps
        assert resid[j] == r                      # same residual bit for bit
        assert kst[j] == lbm.LBM_OK
        assert k[j] == s.permeability() == b.solvers[j].permeability()
        assert np.array_equal(_bytes(s), _bytes(b.solvers[j]))
    assert len(set(steps.tolist())) > 1, "samples should retire at different windows"
    print(f"{precision} graph={graph}: steps {steps.tolist()} k {k.tolist()}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_step_mixed_parity(precision):
    """Samples at different ping-pong parities and step counts step together."""
    masks = _masks_2d()[:3]
    taus = [0.8, 0.6, 1.0]
    alone = _singles(masks, taus, precision)
    b = lbm.Batch.from_masks(masks, taus, RHO["rho_in"], RHO["rho_out"], precision=precision)
    for j, n in enumerate([0, 1, 6]):   # desynchronise the parities first
        alone[j].step(n)
        b.solvers[j].step(n)
    b.step(7)
    for s in alone:
        s.step(7)
    status, steps, _ = b.run_to_steady(1e-6, 5000)
    ref = [s.run_to_steady(1e-6, 5000, raise_on_notconv=False) for s in alone]
    for j, s in enumerate(alone):
        assert steps[j] == ref[j][1] == s.steps
        assert np.array_equal(_bytes(s), _bytes(b.solvers[j]))
    q = b.flux()
    assert q.tolist() == [s.flux() for s in alone]


def test_batch_sample_vs_oracle():
    """A batch sample against the oracle at equal steps (FP64 bar 1e-10)."""
    masks = _masks_2d()[:2]
    b = lbm.Batch.from_masks(masks, [0.8, 0.6], RHO["rho_in"], RHO["rho_out"], precision="fp64")
    b.step(1500)
    k, _ = b.permeability()
    for j, m in enumerate(masks):
        o = oracle.Oracle(9, m, [0.8, 0.6][j], RHO["rho_in"], RHO["rho_out"])
        o.step(1500)
        ko = o.permeability()
        assert abs(k[j] - ko) / ko <= 1e-10


def test_batch_d3q19_bitwise():
    masks = [qsgs_3d(40, 20, 12, 0.7, 3), qsgs_3d(70, 9, 7, 0.7, 4), qsgs_3d(33, 16, 16, 0.7, 5)]
    taus = [0.6, 0.8, 1.0]
    alone = _singles(masks, taus, "fp32")
    ref = [s.run_to_steady(1e-7, 20000, raise_on_notconv=False) for s in alone]
    b = lbm.Batch.from_masks(masks, taus, RHO["rho_in"], RHO["rho_out"], precision="fp32")
    status, steps, resid = b.run_to_steady(1e-7, 20000)
    for j, s in enumerate(alone):
        assert steps[j] == ref[j][1]
        assert resid[j] == ref[j][2]
        assert np.array_equal(_bytes(s), _bytes(b.solvers[j]))


def test_batch_launch_options_per_sample():
    """Samples with different tile orders share a launch; results stay bitwise."""
    masks = _masks_2d()[:4]
    taus = [0.8] * 4
    opts = [dict(band=16), dict(band=0, xcd_remap=0), dict(band=0, xcd_remap=1),
            dict(band=3)]
    alone = _singles(masks, taus, "fp32")
    for s in alone:
        s.step(333)
    solvers = _singles(masks, taus, "fp32")
    for s, o in zip(solvers, opts):
        s.configure(**o)
    b = lbm.Batch(solvers)
    b.step(333)
    for j, s in enumerate(alone):
        assert np.array_equal(_bytes(s), _bytes(solvers[j]))


def test_batch_retires_nonfinite_and_notconv():
    masks = _masks_2d()[:3]
    taus = [0.8, 0.8, 0.8]
    b = lbm.Batch.from_masks(masks, taus, RHO["rho_in"], RHO["rho_out"], precision="fp32")
    # poison one population of sample 1 (a fluid slot)
    s1 = b.solvers[1]
    buf = s1.get_populations()
    v = buf.view(torch.float32)
    slot = int(s1.slot_map().view(-1).max().item())
    v[slot] = float("nan")
    s1.set_populations(buf)
    status, steps, resid = b.run_to_steady(1e-9, 700)
    assert status[1] == lbm.LBM_ENONFINITE and steps[1] == 100 and np.isnan(resid[1])
    assert status[0] == status[2] == lbm.LBM_ENOTCONV
    assert steps[0] == steps[2] == 700
    # the healthy samples are unaffected by the poisoned one
    alone = lbm.Solver(masks[0], 0.8, precision="fp32", **RHO)
    alone.step(700)
    assert np.array_equal(_bytes(alone), _bytes(b.solvers[0]))


def test_batch_rejects_mismatch():
    m = _masks_2d()[:2]
    a = lbm.Solver(m[0], 0.8, precision="fp32", **RHO)
    c = lbm.Solver(m[1], 0.8, precision="fp64", **RHO)
    with pytest.raises(lbm.LBMError):
        lbm.Batch([a, c])
    with pytest.raises(lbm.LBMError):
        lbm.Batch([a, a])


def test_autotune_picks_a_candidate_and_stays_bitwise(tmp_path, monkeypatch):
    from paper_1609_09685_amd import autotune
    monkeypatch.setenv("LBM_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    masks = _masks_2d()[:3]
    res = autotune.tune(masks[0], precision="fp32", steps=5)
    assert (res["band"], res["xcd_remap"]) in autotune.CANDIDATES
    assert len(res["timings"]) == len(autotune.CANDIDATES)
    assert autotune.tune(masks[0], precision="fp32") == res      # cached
    b = lbm.Batch.from_masks(masks, [0.8] * 3, RHO["rho_in"], RHO["rho_out"], precision="fp32",
                             autotune=True)
    b.step(250)
    for j, m in enumerate(masks):
        s = lbm.Solver(m, 0.8, precision="fp32", **RHO)
        s.step(250)
        assert np.array_equal(_bytes(s), _bytes(b.solvers[j]))


def test_batch_flux_log():
    """The per-window flux log ends at each sample's retirement and its last two
    entries give the reported residual."""
    masks = _masks_2d()[:3]
    b = lbm.Batch.from_masks(masks, [0.8, 0.6, 1.0], RHO["rho_in"], RHO["rho_out"],
                             precision="fp64")
    status, steps, resid, log = b.run_to_steady(1e-7, 30000, log_windows=400)
    for d in range(3):
        q = log[:, d]
        n = int(np.isfinite(q).sum())
        assert n == steps[d] // 100 and np.isfinite(q[:n]).all() and np.isnan(q[n:]).all()
        assert abs(q[n - 1] - q[n - 2]) / abs(q[n - 1]) == resid[d]
