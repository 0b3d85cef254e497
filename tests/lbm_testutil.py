"""Helpers shared by the GPU parity tests: layout conversion between the
solver's internal state (deviation SoA, padded x pitch, its own direction
order) and the oracle's (node-major f, oracle direction order).

Only marshalling lives here: no lattice Boltzmann arithmetic.
"""
import numpy as np

import oracle
from paper_1609_09685_amd import lbm


def direction_map(Q):
    """perm[j] = the solver's direction index with the oracle's c_j."""
    c_gpu, _ = lbm.lattice_table(Q)
    c_or = oracle.lattice(Q)["c"]
    lookup = {tuple(v): i for i, v in enumerate(c_gpu)}
    return np.array([lookup[tuple(v)] for v in c_or])


def _dtype(solver):
    import torch
    return torch.float64 if solver.precision == "fp64" else torch.float32


def compact_view(solver, buf=None):
    """The solver's populations as a device tensor (Q, ps): direction-major,
    one column per slot (fluid nodes and zero padding)."""
    if buf is None:
        buf = solver.get_populations()
    Q = solver.lattice
    return buf.view(_dtype(solver)).view(Q, -1)


def fluid_slots(solver):
    """(dense flat indices of the fluid nodes, their slots), as device tensors."""
    import torch
    sm = solver.slot_map().view(-1)
    idx = torch.nonzero(sm >= 0, as_tuple=False).view(-1)
    return idx, sm[idx].long()


def dense_state(solver, buf=None):
    """(Q, nz, ny, nx) device tensor of the deviations, 0 on solids."""
    import torch
    c = compact_view(solver, buf)
    Q = solver.lattice
    n = solver.nx * solver.ny * solver.nz
    out = torch.zeros((Q, n), dtype=c.dtype, device=c.device)
    idx, slots = fluid_slots(solver)
    out[:, idx] = c[:, slots]
    return out.view(Q, solver.nz, solver.ny, solver.nx)


state_view = dense_state


def to_oracle_f(g_window, Q, rho0=1.0):
    """(Q, z, y, x) deviations in solver order -> node-major f in oracle order."""
    perm = direction_map(Q)
    w = oracle.lattice(Q)["w"]
    g = np.asarray(g_window, np.float64)[perm]          # oracle order
    f = g + (w * rho0)[:, None, None, None]
    return np.moveaxis(f, 0, -1).reshape(-1, Q)


def from_oracle_f(f, Q, shape, rho0=1.0):
    """node-major f (oracle order) -> (Q, nz, ny, nx) deviations in solver order."""
    perm = direction_map(Q)
    w = oracle.lattice(Q)["w"]
    g = (np.asarray(f).reshape(*shape, Q) - w * rho0)
    g = np.moveaxis(g, -1, 0)
    out = np.empty_like(g)
    out[perm] = g
    return out


def random_state(solver, scale=1e-4, seed=0):
    """Seeded random deviations g_i = w_i * scale * N(0,1) on every fluid node
    (padding stays zero), written into the solver's current state; returns the
    dense (Q, nz, ny, nx) view of what was written (0 on solids)."""
    import torch
    Q = solver.lattice
    buf = torch.zeros(solver.f_bytes, dtype=torch.uint8, device=solver.device)
    c = compact_view(solver, buf)
    idx, slots = fluid_slots(solver)
    gen = torch.Generator(device=c.device)
    gen.manual_seed(seed)
    _, w = lbm.lattice_table(Q)
    vals = torch.randn((Q, slots.numel()), generator=gen, dtype=torch.float64,
                       device=c.device).to(c.dtype)
    vals.mul_(torch.tensor(w, dtype=c.dtype, device=c.device).view(Q, 1) * scale)
    c[:, slots] = vals
    solver.set_populations(buf)
    return dense_state(solver, buf)


def solver_mask(solver):
    return solver._mask.view(solver.nz, solver.ny, solver.nx).cpu().numpy()


def fields_gpu(solver):
    """(rho (nz,ny,nx), u (nz,ny,nx,3)) float64 numpy, NaN on solids."""
    rho, u = solver.macro("float64")
    rho = rho.cpu().numpy()
    u = np.moveaxis(u.cpu().numpy(), 0, -1)
    if u.shape[-1] == 2:
        u = np.concatenate([u, np.zeros(u.shape[:-1] + (1,))], axis=-1)
    solid = solver_mask(solver).astype(bool)
    rho[solid] = np.nan
    u[solid] = np.nan
    return rho, u


# The oracle stores f ~ w_i in binary64 (f-form): a node's density and
# momentum are sums of Q values whose partial sums are ~1, so every step adds
# rounding of about Q * ulp(1)/2 = Q * 2**-53 to what it reports.  These
# errors are independent from step to step and add like a random walk; with a
# safety factor of 10 that gives the absolute floor below.  The solver stores
# deviations (values ~1e-4 w_i) whose rounding is negligible next to it, so
# comparisons allow this floor on top of the relative bar.
def field_floor(Q, steps):
    return 10.0 * Q * max(steps, 1) ** 0.5 * 2.0 ** -53


def max_rel_field_error(solver, orc):
    """Max-norm field errors and scales: (u_abs_err, max|u|, rho_abs_err, max|rho - 1|)."""
    rg, ug = fields_gpu(solver)
    ro, uo = orc.macro()
    fl = ~np.isnan(ro)
    return (np.abs(ug[fl] - uo[fl]).max(), np.abs(uo[fl]).max(),
            np.abs(rg[fl] - ro[fl]).max(), np.abs(ro[fl] - 1.0).max())


def fields_match(solver, orc, tol):
    """err <= tol * scale + field_floor for u and rho; also returns the ratios."""
    du, us, dr, rs = max_rel_field_error(solver, orc)
    fl = field_floor(solver.lattice, orc.steps)
    ok = du <= tol * us + fl and dr <= tol * rs + fl
    return ok, (du / us, dr / rs, du, dr, fl)
