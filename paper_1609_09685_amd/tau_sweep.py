"""The paper's 2D experiment (its Figs. 2 and 3): permeability of one porous
structure at three resolutions, 400x200, 800x400 and 1200x600 (D2Q9,
pressure-driven along x, symmetric top and bottom), against tau, normalised
by the intrinsic permeability, and the same data against the Knudsen number
Kn = sqrt(pi/6)(tau - 1/2)/N_x.

The paper finds that k/k_int differs strongly between resolutions at equal
tau, approaches 1 only as tau -> 1/2, and collapses onto one curve against
Kn, especially below Kn = 10^-3.  Its structure and its curves are not
published; here one seeded QSGS structure (400x200, porosity 0.7394) is
refined 2x and 3x by splitting every voxel, so the three lattices resolve the
same geometry (the paper re-drew its image, whose porosity moved to
0.7532 / 0.7578).

k_int: the paper only says that k approaches it as tau - 1/2 -> 0.  A steady
BGK state depends on tau only through Lambda = (tau - 1/2)^2 (BGK is the
two-relaxation-time scheme with that magic parameter), so the limit is the
steady state at Lambda -> 0.  BGK itself cannot reach it: with tau <= 0.52
the runs on the refined grids lose stability at the outlet's pressure
boundary (the CPU oracle does the same).  The TRT collision reaches the same
limit at a comfortable tau+ = 1, so k_int is its permeability at
Lambda = K_INT_MAGIC (1e-6).

    python -m paper_1609_09685_amd.tau_sweep [--out results.json]

Each resolution is one batch (one sample per tau) run to the flux residual.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import lbm
from .qsgs import qsgs_2d

TAUS = (0.505, 0.51, 0.52, 0.55, 0.6, 0.7, 0.8, 1.0, 1.2, 1.5, 2.0)
# tau - 1/2 = r d at refinement r: equal Kn at every resolution
KN_STEPS = (0.025, 0.05, 0.1, 0.2, 0.5)
REFINE = (1, 2, 3)
POROSITY = 0.7394
K_INT_MAGIC = 1e-6
K_INT_TAU = 1.0


def media(nx=400, ny=200, porosity=POROSITY, seed=0, refine=REFINE):
    """One QSGS structure at several resolutions (every voxel split r x r)."""
    base = qsgs_2d(nx, ny, porosity, seed)
    return [np.kron(base, np.ones((r, r), np.uint8)) for r in refine]


def intrinsic_permeability(mask, rho=(1.0005, 0.9995), precision="fp32", tol=1e-9,
                           max_steps=2_000_000, magic=K_INT_MAGIC, tau=K_INT_TAU):
    """The Lambda -> 0 limit of the steady permeability, by the TRT collision
    at tau+ = tau with the magic parameter `magic`; (k, steps)."""
    s = lbm.Solver(mask, tau, rho[0], rho[1], precision=precision, lattice=9)
    s.set_trt(magic)
    ok, steps, _ = s.run_to_steady(tol, max_steps, raise_on_notconv=False)
    k = s.permeability() if ok else float("nan")
    s.close()
    return k, steps


def taus_for(refine, taus=TAUS, kn_steps=KN_STEPS):
    """The common taus plus 1/2 + refine d for every d of kn_steps (rounded to
    1e-9), so that every resolution has runs at the same Kn values."""
    return sorted({round(t, 9) for t in taus} |
                  {round(0.5 + refine * d, 9) for d in kn_steps})


def collapse(rows, taus=TAUS, kn_steps=KN_STEPS):
    """Relative spread of k/k_int between the resolutions at equal tau (the
    common taus) and at equal Kn (tau - 1/2 = r d at refinement r, one value
    per d), over the runs that finished."""
    rows = [r for r in rows if r["k_norm"] is not None]
    res = sorted({r["refine"] for r in rows})
    at = {(r["refine"], round(r["tau"], 9)): r["k_norm"] for r in rows}

    def spread(keys):
        v = [at[k] for k in keys if k in at]
        return (max(v) - min(v)) / min(v) if len(v) == len(keys) and v else None
    eq_tau = {t: spread([(r, round(t, 9)) for r in res]) for t in taus}
    eq_kn = {d: spread([(r, round(0.5 + r * d, 9)) for r in res]) for d in kn_steps}
    eq_tau = {t: v for t, v in eq_tau.items() if v is not None}
    eq_kn = {d: v for d, v in eq_kn.items() if v is not None}
    return dict(spread_equal_tau=eq_tau, spread_equal_kn=eq_kn,
                max_spread_equal_tau=max(eq_tau.values()) if eq_tau else None,
                max_spread_equal_kn=max(eq_kn.values()) if eq_kn else None)


def sweep(masks, refine=REFINE, taus=TAUS, kn_steps=KN_STEPS, precision="fp32", tol=1e-9,
          max_steps=2_000_000, rho=(1.0005, 0.9995), log=None):
    """k for every (resolution, tau), k_int per resolution and k/k_int;
    masks[i] is the structure at refinement refine[i]."""
    rows = []
    for r, m in zip(refine, masks):
        t0 = time.time()
        ny, nx = m.shape
        rtaus = taus_for(r, taus, kn_steps)
        b = lbm.Batch.from_masks([m] * len(rtaus), rtaus, rho[0], rho[1],
                                 precision=precision)
        status, steps, _ = b.run_to_steady(tol, max_steps)
        k, kst = b.permeability()
        b.close()
        for s in b.solvers:
            s.close()
        k_int, int_steps = intrinsic_permeability(m, rho, precision, tol, max_steps)
        phi = 1.0 - float(m.mean())
        for j, tau in enumerate(rtaus):
            st = int(status[j]) if status[j] != lbm.LBM_OK else int(kst[j])
            ok = st == lbm.LBM_OK
            rows.append(dict(refine=r, nx=nx, ny=ny, porosity=phi, tau=tau,
                             kn=lbm.knudsen(tau, nx),
                             k=float(k[j]) if ok else None, k_int=k_int,
                             k_norm=float(k[j] / k_int) if ok else None,
                             steps=int(steps[j]), status=st, k_int_steps=int(int_steps)))
        if log:
            log(f"{nx}x{ny} phi {phi:.4f}: k_int {k_int:.6g} ({int_steps} steps), k/k_int "
                + " ".join(f"{x / k_int:.4f}" if st == 0 else "--"
                           for x, st in zip(k, status))
                + f", steps {int(steps.min())}..{int(steps.max())}, {time.time() - t0:.1f} s")
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--nx", type=int, default=400)
    ap.add_argument("--ny", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64"))
    ap.add_argument("--tol", type=float, default=1e-9)
    ap.add_argument("--taus", type=float, nargs="*", default=list(TAUS))
    ap.add_argument("--kn-steps", type=float, nargs="*", default=list(KN_STEPS),
                    help="extra taus 1/2 + r d at refinement r (equal-Kn runs); none: only --taus")
    ap.add_argument("--refine", type=int, nargs="*", default=list(REFINE))
    ap.add_argument("--seeds", type=int, nargs="*", default=None,
                    help="several structures (default: --seed)")
    ap.add_argument("--porosity", type=float, default=POROSITY)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    seeds = a.seeds if a.seeds else [a.seed]
    rows = []
    for seed in seeds:
        masks = media(a.nx, a.ny, porosity=a.porosity, seed=seed, refine=a.refine)
        log(f"structure seed {seed}, porosity {1 - masks[0].mean():.4f}, {a.precision}")
        part = sweep(masks, a.refine, a.taus, a.kn_steps, a.precision, a.tol, log=log)
        for r in part:
            r["seed"] = seed
        rows += part
    c = None
    if len(a.refine) > 1 and len(seeds) == 1:
        c = collapse(rows, a.taus, a.kn_steps)
        log("k/k_int spread between resolutions at equal tau: "
            + ", ".join(f"{t}: {v:.3g}" for t, v in sorted(c["spread_equal_tau"].items())))
        log("at equal Kn (tau - 1/2 = r d): "
            + ", ".join(f"d={d}: {v:.3g}" for d, v in sorted(c["spread_equal_kn"].items())))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(dict(seeds=seeds, precision=a.precision, tol=a.tol, rows=rows,
                           collapse=c), f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
