"""The paper's 3D experiment: intrinsic permeability of a force-driven, fully
periodic porous medium (D3Q19, 100^3 voxels, porosity 0.748587), by Eq. 2,
against the Knudsen number for three body forces, with the full second-order
equilibrium and with the linear ("Stokes") one.

The paper reports the qualitative result (its Fig. 5): k is the same for every
g except at small Kn for the largest g, where inertia lowers it (small tau
means small viscosity, so the Reynolds number grows at a fixed lattice
velocity); with the linear equilibrium the g dependence disappears.  Neither
its g values nor its k values are printed, and its geometry is an image that
is not published, so the medium here is a seeded QSGS structure of the same
size and porosity, and the forces are chosen to span the Stokes and the
inertial regime.

    python -m paper_1609_09685_amd.force_driven [--n 100] [--out results.json]

Each (tau, equilibrium) pair is one batch of the three forces, run to the
flux residual; a line is printed as each batch finishes.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import lbm
from .qsgs import qsgs_3d

TAUS = (0.51, 0.52, 0.55, 0.6, 0.7, 0.8, 1.0, 1.5, 2.0, 3.0)
FORCES = (1e-6, 1e-5, 1e-4)
POROSITY = 0.748587


def medium(n=100, porosity=POROSITY, seed=0):
    """Seeded QSGS medium of n^3 voxels (uint8, 1 = solid)."""
    return qsgs_3d(n, n, n, porosity, seed)


def sweep(mask, taus=TAUS, forces=FORCES, precision="fp32", tol=1e-8, max_steps=400000,
          check_every=100, log=None):
    """k by Eq. 2 for every (linear, tau, g): a list of dicts with tau, Kn, g,
    linear, k, steps, status (lbm status of the run) and reynolds (pore-scale
    Re = <u>_fluid d / nu with d = 4 phi / specific surface, a size estimate)."""
    nx = mask.shape[-1]
    solid = mask.astype(bool)
    phi = 1.0 - solid.mean()
    # specific surface: solid-fluid faces per voxel
    faces = sum(np.count_nonzero(solid != np.roll(solid, 1, axis=a)) for a in range(3))
    d_pore = 4.0 * phi * solid.size / max(faces, 1)
    rows = []
    for linear in (False, True):
        for tau in taus:
            t0 = time.time()
            solvers = [lbm.Solver(mask, tau, 1.0, 1.0, precision=precision, lattice=19,
                                  check_every=check_every, boundary="periodic", body_force=g)
                       for g in forces]
            for s in solvers:
                s.set_linear_equilibrium(linear)
            b = lbm.Batch(solvers)
            status, steps, _ = b.run_to_steady(tol, max_steps)
            k, kst = b.permeability()
            nu = (tau - 0.5) / 3.0
            for j, g in enumerate(forces):
                st = int(status[j]) if status[j] != lbm.LBM_OK else int(kst[j])
                u_mean = k[j] * g / nu / phi           # Eq. 2: <u>_fluid = k g / (nu phi)
                rows.append(dict(tau=tau, kn=lbm.knudsen(tau, nx), g=g, linear=linear,
                                 k=float(k[j]), steps=int(steps[j]), status=st,
                                 reynolds=float(u_mean * d_pore / nu)))
            b.close()
            for s in solvers:
                s.close()
            if log:
                ks = " ".join(f"{k[j]:.6e}" for j in range(len(forces)))
                log(f"{'linear' if linear else 'full  '} tau {tau:<5} Kn {lbm.knudsen(tau, nx):.2e}"
                    f"  k {ks}  steps {list(map(int, steps))}  {time.time() - t0:.1f} s")
    return rows, dict(porosity=float(phi), pore_diameter=float(d_pore))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64"))
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-steps", type=int, default=400000)
    ap.add_argument("--taus", type=float, nargs="*", default=list(TAUS))
    ap.add_argument("--forces", type=float, nargs="*", default=list(FORCES))
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    mask = medium(a.n, seed=a.seed)

    def log(msg):
        print(msg, flush=True)

    log(f"medium {a.n}^3 QSGS seed {a.seed}, porosity {1 - mask.mean():.6f}, "
        f"{a.precision}, tol {a.tol}")
    rows, info = sweep(mask, a.taus, a.forces, a.precision, a.tol, a.max_steps, log=log)
    res = dict(n=a.n, seed=a.seed, precision=a.precision, tol=a.tol, **info, rows=rows)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
