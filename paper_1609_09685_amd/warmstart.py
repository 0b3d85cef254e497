"""Learned warm start for the permeability solver.

A small U-Net (the HIP network of ``wsn``) maps a 2D solid mask and the
Knudsen number Kn = sqrt(pi/6)(tau - 1/2)/Nx (the paper's discussion of Fig.
2) to the steady density and velocity fields; the solver then starts from the
equilibrium populations of that prediction and runs, as always, to the same
flux residual.  The network only changes how many steps that takes: the
converged answer is the solver's.

Steps, all on the GPU through the library's entry points:

1. data: batched solver runs (``lbm.Batch``) of random QSGS masks to the
   steady state, fields read back with ``lbm_get_macro`` and normalised by
   Stokes linearity (``wsn_fields_to_nhwc``):
       rho' = (rho - rho_lin(x)) / (drho R),   u' = u nu L / (c_s^2 drho) / U,
   where rho_lin is the linear drop between the ghost planes, L = Nx + 1 and
   drho = rho_in - rho_out: in the Stokes regime both are independent of
   drho, u' is a local permeability (Darcy's law), and rho' holds only the
   local departures from the mean pressure gradient, which a convolutional
   map can see (absolute position it cannot).  The scales U and R are the
   RMS of the two quantities over the training data (``scales_of``), so that
   every channel weighs alike in the loss (with R = 1 the density channel,
   RMS ~0.13, carried ~1 % of the loss and was barely learned);
2. training: masked MSE over fluid nodes, Adam (``wsn_*`` kernels);
3. start: prediction -> fields (``wsn_nhwc_to_fields``, velocity zero in
   closed pockets) -> ``lbm_set_macro`` -> ``lbm_smooth`` (removes the modes
   that alternate every step and never decay, which an imperfect field
   excites at dead-end pores); a sample whose prediction is not finite starts
   from rest instead, and one whose converged state still alternates from
   step to step is rerun from rest (``run_checked``).
"""
import time

import numpy as np

from . import lbm, wsn
from .qsgs import qsgs_2d

NX, NY = 256, 128
RHO_IN, RHO_OUT = 1.0005, 0.9995
KN_SCALE = 1e-3          # network input: Kn / KN_SCALE
CS2 = 1.0 / 3.0
SMOOTH_PASSES = 4        # lbm_smooth passes (period-2 modes) before using a field


def sample(seed, nx=NX, ny=NY):
    """(mask, tau, porosity) of one sample: porosity U[0.6, 0.9], tau U[0.51, 1.0]
    from a generator seeded with `seed`, QSGS mask with the same seed."""
    rng = np.random.default_rng(seed)
    phi = float(rng.uniform(0.6, 0.9))
    tau = float(rng.uniform(0.51, 1.0))
    return qsgs_2d(nx, ny, phi, seed), tau, phi


PROFILE_SCALE = 10.0     # network input: resistance profile (wsn_column_profile) x 10


def features(taus, nx):
    return np.array([lbm.knudsen(t, nx) / KN_SCALE for t in taus], np.float32)


def inputs(solid, taus, in_ch=2, out=None):
    """Network input of the masks solid (device uint8 [B,H,W]) and their taus:
    mask and scaled Kn, and with in_ch = 3 the masks' resistance profile
    along x (``wsn.column_profile``), which carries what lies upstream and
    downstream of a pixel beyond the network's reach."""
    feat = _dev(features(taus, solid.shape[2]))
    if in_ch == 2:
        return wsn.pack_input(solid, feat, out=out)
    if in_ch != 3:
        raise ValueError("in_ch must be 2 or 3")
    return wsn.pack_input(solid, feat, out=out, profile=wsn.column_profile(solid),
                          profile_scale=PROFILE_SCALE)


def target_maps(taus, nx, scales, rho_in=RHO_IN, rho_out=RHO_OUT):
    """Per-sample (shift, slope, scale, inverse scale) [B, 3] between solver fields
    and normalised targets: y = (f - shift - slope (x + 1)) * scale.  The density
    target is the deviation from the linear drop between the ghost planes,
    rho_in + (rho_out - rho_in)(x + 1)/(nx + 1), in units of drho R;
    scales = (U, R), the velocity and density scales."""
    u_scale, rho_scale = scales
    taus = np.asarray(taus, float)
    drho = rho_in - rho_out
    nu = (taus - 0.5) / 3.0
    uf = nu * (nx + 1) / (CS2 * drho) / u_scale          # u -> u'
    shift = np.zeros((len(taus), 3))
    shift[:, 0] = rho_in
    slope = np.zeros((len(taus), 3))
    slope[:, 0] = (rho_out - rho_in) / (nx + 1)
    fwd = np.stack([np.full_like(uf, 1.0 / (drho * rho_scale)), uf, uf], 1)
    inv = 1.0 / fwd
    f32 = lambda a: a.astype(np.float32)
    return f32(shift), f32(slope), f32(fwd), f32(inv)


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


class Dataset:
    """Device tensors of n samples: x [n,H,W,2], fields rho [n,H,W], u [n,2,H,W],
    solid [n,H,W] uint8, and per-sample tau, steps, k, converged."""

    def __init__(self, x, rho, u, solid, taus, steps, k, converged, seeds):
        self.x, self.rho, self.u, self.solid = x, rho, u, solid
        self.taus, self.steps, self.k = np.asarray(taus), np.asarray(steps), np.asarray(k)
        self.converged, self.seeds = np.asarray(converged), np.asarray(seeds)

    def __len__(self):
        return len(self.taus)

    def targets(self, scales):
        shift, slope, fwd, _ = target_maps(self.taus, self.x.shape[2], scales)
        return wsn.fields_to_nhwc(self.rho, self.u, _dev(shift), _dev(fwd), slope=_dev(slope))


def solve(masks, taus, precision="fp32", tol=1e-9, max_steps=400000, starts=None, graph=True):
    """Runs the samples to the steady state in one batch.  starts[j]: None (rest,
    uniform density) or (rho, u) device tensors for lbm_set_macro.  Returns
    (batch, status, steps, resid, seconds)."""
    import torch
    b = lbm.Batch.from_masks(masks, taus, RHO_IN, RHO_OUT, precision=precision, graph=graph)
    if starts is not None:
        for s, st in zip(b.solvers, starts):
            if st is not None:
                s.set_macro(*st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, steps, resid = b.run_to_steady(tol, max_steps)
    torch.cuda.synchronize()
    return b, status, steps, resid, time.perf_counter() - t0


def generate(seeds, chunk=1024, precision="fp32", tol=1e-9, max_steps=400000, log=None, in_ch=2):
    """Steady states of the samples `seeds` (zero-velocity start), in batches of
    `chunk` samples, with network inputs of in_ch channels (``inputs``).  Only
    samples that reach the residual are kept (packed in seed order); the
    others are counted in `dropped`."""
    import torch
    seeds = list(seeds)
    n = len(seeds)
    x = torch.empty((n, NY, NX, in_ch), dtype=torch.float32, device="cuda")
    rho = torch.empty((n, NY, NX), dtype=torch.float32, device="cuda")
    u = torch.empty((n, 2, NY, NX), dtype=torch.float32, device="cuda")
    solid = torch.empty((n, NY, NX), dtype=torch.uint8, device="cuda")
    taus, steps, ks, kept = [], [], [], []
    dropped = {"not_converged": 0, "non_finite": 0}
    for c0 in range(0, n, chunk):
        part = seeds[c0:c0 + chunk]
        smp = [sample(s) for s in part]
        b, status, st, _, sec = solve([m for m, _, _ in smp], [t for _, t, _ in smp], precision,
                                      tol, max_steps)
        k, kst = b.permeability()
        for j, s in enumerate(b.solvers):
            if status[j] != lbm.LBM_OK or kst[j] != lbm.LBM_OK:
                dropped["non_finite" if status[j] == lbm.LBM_ENONFINITE else "not_converged"] += 1
                continue
            i = len(kept)
            # the converged state may still carry modes that alternate every
            # step (mostly in u_y, invisible to the x flux); the fields are
            # read after removing them
            s.smooth(SMOOTH_PASSES)
            s.macro("float32", out=(rho[i], u[i]))
            solid[i] = torch.as_tensor(smp[j][0]).cuda()
            kept.append(part[j])
            taus.append(smp[j][1])
            steps.append(int(st[j]))
            ks.append(float(k[j]))
        torch.cuda.synchronize()
        b.close()
        del b
        if log:
            log(f"samples {c0}..{c0 + len(part) - 1}: {int((status == lbm.LBM_OK).sum())}/"
                f"{len(part)} converged, steps median {int(np.median(st))} max {int(st.max())}, "
                f"{sec:.1f} s")
    m = len(kept)
    inputs(solid[:m], taus, in_ch, out=x[:m])
    d = Dataset(x[:m], rho[:m], u[:m], solid[:m], taus, steps, ks, np.ones(m, bool), kept)
    d.dropped = dropped
    return d


def scales_of(data, sample_count=64):
    """(U, R): the RMS of u nu L / (c_s^2 drho) and of (rho - rho_lin)/drho over
    the fluid nodes of the first samples."""
    shift, slope, fwd, _ = target_maps(data.taus[:sample_count], NX, (1.0, 1.0))
    y = wsn.fields_to_nhwc(data.rho[:sample_count].contiguous(), data.u[:sample_count].contiguous(),
                           _dev(shift), _dev(fwd), slope=_dev(slope)).cpu().numpy()
    fluid = data.solid[:sample_count].cpu().numpy() == 0
    return (float(np.sqrt((y[..., 1:][fluid] ** 2).mean())),
            float(np.sqrt((y[..., 0][fluid] ** 2).mean())))


def new_network(batch, seed=0, levels=4, base=32, in_ch=2):
    """A U-Net with He-normal initial weights drawn from a seeded NumPy generator
    (in_ch input channels: 2, or 3 with the resistance profile)."""
    shapes = []
    ch = [base * 2 ** l for l in range(levels)]
    cin = in_ch
    for l in range(levels):
        shapes += [(3, cin, ch[l]), (3, ch[l], ch[l])]
        cin = ch[l]
    for l in range(levels - 2, -1, -1):
        shapes += [(3, ch[l + 1] + ch[l], ch[l]), (3, ch[l], ch[l])]
    shapes.append((1, ch[0], 3))
    rng = np.random.default_rng(seed)
    parts = []
    for ks, ci, co in shapes:
        parts.append(rng.standard_normal(ks * ks * ci * co) * np.sqrt(2.0 / (ks * ks * ci)))
        parts.append(np.zeros(co))
    return wsn.WarmStartNet(np.concatenate(parts).astype(np.float32), batch, levels=levels,
                            base=base, in_ch=in_ch, height=NY, width=NX)


# Symmetries of the setup (Fig. 1) as (flip_h, flip_w) and the factors of the
# targets (rho', u'_x, u'_y): the symmetric top and bottom planes make the
# y-mirror of a steady state the steady state of the y-mirrored mask (u_y
# changes sign); Stokes linearity makes the x-mirror with the pressure drop
# reversed that of the x-mirrored mask (rho' and u_y change sign: the linear
# drop between the ghost planes is odd about the middle, and mirror and
# reversal each turn u_x round).
MIRRORS = (((1, 0), (1.0, 1.0, -1.0)),
           ((0, 1), (-1.0, 1.0, -1.0)),
           ((1, 1), (-1.0, 1.0, 1.0)))


def augmented(data, y):
    """Inputs, targets and masks of the data followed by those of its three
    mirror images (MIRRORS): 4 n training samples from n solved ones.  The
    inputs of a mirror image are formed from its mirrored masks."""
    import torch
    xs, ys, ss = [data.x], [y], [data.solid]
    for (fh, fw), sign in MIRRORS:
        m = wsn.mirror(data.solid, fh, fw)
        xs.append(inputs(m, data.taus, data.x.shape[3]))
        ys.append(wsn.mirror(y, fh, fw, sign))
        ss.append(m)
    return torch.cat(xs), torch.cat(ys), torch.cat(ss)


def train(net, data, scales, epochs=20, lr=1e-3, lr_end=1e-5, seed=0, log=None, augment=False):
    """Adam on the masked MSE; minibatches are contiguous slices of the data in a
    shuffled order per epoch, learning rate decayed geometrically to lr_end.
    augment: train on the data and its three mirror images (``augmented``).
    Returns the mean loss of every epoch."""
    import torch
    B = net.batch
    x_all, y_all, s_all = data.x, data.targets(scales), data.solid
    if augment:
        x_all, y_all, s_all = augmented(data, y_all)
    nb = len(x_all) // B
    rng = np.random.default_rng(seed)
    total = epochs * nb
    hist = []
    it = 0
    for ep in range(epochs):
        losses = []
        for i in rng.permutation(nb):
            sl = slice(i * B, (i + 1) * B)
            rate = lr * (lr_end / lr) ** (it / max(total - 1, 1))
            losses.append(net.train_step(x_all[sl], y_all[sl], s_all[sl], rate))
            it += 1
        ep_loss = float(torch.stack(losses).mean().item())
        hist.append(ep_loss)
        if log:
            log(f"epoch {ep + 1}/{epochs}: loss {ep_loss:.4e}")
    return hist


def predict(net, masks, taus, scales, tta=False):
    """Fields (rho [B,H,W], u [B,2,H,W]) and the non-finite flags of the network's
    prediction for the samples (any number; run in chunks of the net's batch).
    tta: average the predictions for the mask and its three mirror images
    (MIRRORS), each mirrored back.  The velocity is set to zero in fluid
    pockets that no path along lattice links joins to the inlet or outlet: the
    steady flow there is exactly zero, and a closed pocket keeps whatever
    momentum it starts with."""
    import torch
    from .qsgs import open_fluid
    n = len(masks)
    rho = torch.empty((n, NY, NX), dtype=torch.float32, device="cuda")
    u = torch.empty((n, 2, NY, NX), dtype=torch.float32, device="cuda")
    bad = torch.empty(n, dtype=torch.int32, device="cuda")
    shift, slope, _, inv = target_maps(taus, NX, scales)
    for c0 in range(0, n, net.batch):
        m = min(net.batch, n - c0)
        solid = _dev(np.stack(masks[c0:c0 + m]).astype(np.uint8))
        keep = _dev(np.stack([open_fluid(mk) for mk in masks[c0:c0 + m]]))
        tm = taus[c0:c0 + m]
        y = net.infer(inputs(solid, tm, net.cfg.in_ch))
        if tta:
            w = 1.0 / (1 + len(MIRRORS))
            y = wsn.mirror(y, 0, 0, (w, w, w))
            for (fh, fw), sign in MIRRORS:
                xv = inputs(wsn.mirror(solid, fh, fw), tm, net.cfg.in_ch)
                wsn.mirror(net.infer(xv), fh, fw, [w * v for v in sign], out=y, accumulate=True)
        wsn.nhwc_to_fields(y, _dev(shift[c0:c0 + m]), _dev(inv[c0:c0 + m]),
                           slope=_dev(slope[c0:c0 + m]), keep_u=keep,
                           out=(rho[c0:c0 + m], u[c0:c0 + m], bad[c0:c0 + m]))
    return rho, u, bad


ONE_STEP_TOL = 1e-6   # relative flux change over one step that marks a period-2 mode
K_TOL = 1e-4          # permeability accuracy of the "accurate permeability" measure


def steps_to_accuracy(q_log, q_final, start_steps, K, rtol=K_TOL):
    """First step count after which the logged flux stays within rtol of its
    converged value (the permeability is proportional to the flux)."""
    out = np.zeros(len(q_final), np.int64)
    for d in range(len(q_final)):
        q = q_log[:, d]
        q = q[np.isfinite(q)]
        err = np.abs(q - q_final[d]) / abs(q_final[d])
        bad = np.nonzero(err > rtol)[0]
        w = 0 if len(bad) == 0 else bad[-1] + 1
        out[d] = start_steps[d] + (w + 1) * K
    return out


def run_checked(masks, taus, start, precision, tol, max_steps, rerun_failed=True, after=None,
                K=100):
    """Runs the samples in one batch from `start(batch)` (which sets every
    solver's initial state and may take time of its own) to the flux residual
    tol, then checks one more step: a converged state whose flux changes by
    more than ONE_STEP_TOL in a single step carries a period-2 oscillation
    that the residual, taken every K (even) steps, cannot see; such samples
    are rerun from the zero-velocity start, their steps added.  Also reports,
    from the flux after every check window, the steps after which the
    permeability stays within K_TOL of its converged value.  `after(batch)`
    runs before the batch is released.  Returns a dict of per-sample results."""
    import torch
    b = lbm.Batch.from_masks(masks, taus, RHO_IN, RHO_OUT, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start(b)
    torch.cuda.synchronize()
    sec_start = time.perf_counter() - t0
    start_steps = np.array([s.steps for s in b.solvers])
    status, steps, _, qlog = b.run_to_steady(tol, max_steps, log_windows=max_steps // K + 1)
    sec_main = time.perf_counter() - t0
    k, _ = b.permeability()
    q0 = b.flux()
    b.step(1)
    q1 = b.flux()
    one = np.abs(q1 - q0) / np.abs(q0)
    flagged = (status == lbm.LBM_OK) & (one > ONE_STEP_TOL)
    rerun = flagged & rerun_failed
    acc = steps_to_accuracy(qlog, q0, start_steps, K)
    steps = steps + 1
    if rerun.any():
        idx = np.nonzero(rerun)[0]
        for j in idx:
            b.solvers[j].reset("uniform")
        b2 = lbm.Batch([b.solvers[j] for j in idx])
        st2, steps2, _, qlog2 = b2.run_to_steady(tol, max_steps, log_windows=max_steps // K + 1)
        k2, _ = b2.permeability()
        q2 = b2.flux()
        acc2 = steps_to_accuracy(qlog2, q2, np.zeros(len(idx), np.int64), K)
        acc[idx] = steps[idx] + acc2
        status[idx], steps[idx], k[idx] = st2, steps[idx] + steps2, k2
        b2.close()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    if after is not None:
        after(b)
    b.close()
    return dict(status=status.tolist(), steps=steps.tolist(), k=k.tolist(), seconds=sec,
                seconds_to_residual=sec_main, start_seconds=sec_start,
                steps_to_k_tol=acc.tolist(),
                one_step_change=one.tolist(), flagged=int(flagged.sum()), reruns=int(rerun.sum()))


def field_errors(pred_rho, pred_u, ref_rho, ref_u, solid, taus, scales):
    """RMS error of the prediction over fluid nodes in the network's units
    (the targets rho', u'), per channel, over all samples, with the RMS of the
    reference targets; and per sample the ratio of the predicted to the
    reference sum of u_x over the fluid nodes (the start's flux against the
    converged one)."""
    shift, slope, fwd, _ = target_maps(taus, NX, scales)
    xp = np.arange(1, NX + 1, dtype=np.float64)[None, None, :]
    fl = solid == 0
    out = {}
    for c, (p, r) in enumerate(((pred_rho, ref_rho), (pred_u[:, 0], ref_u[:, 0]),
                                (pred_u[:, 1], ref_u[:, 1]))):
        base = shift[:, c][:, None, None] + slope[:, c][:, None, None] * xp
        e = (p - r) * fwd[:, c][:, None, None]
        ref = (r - base) * fwd[:, c][:, None, None]
        out[("rho", "ux", "uy")[c]] = dict(rms_err=float(np.sqrt((e[fl] ** 2).mean())),
                                           rms_ref=float(np.sqrt((ref[fl] ** 2).mean())))
    ratio = (np.where(fl, pred_u[:, 0], 0.0).sum(axis=(1, 2)) /
             np.where(fl, ref_u[:, 0], 0.0).sum(axis=(1, 2)))
    out["ux_sum_ratio"] = dict(median=float(np.median(ratio)),
                               p10=float(np.percentile(ratio, 10)),
                               p90=float(np.percentile(ratio, 90)),
                               per_sample=[float(v) for v in ratio])
    return out


def step_seconds(mask, tau, precision, steps=2000):
    """Wall time of one time step of one sample run alone (HIP events)."""
    import torch
    s = lbm.Solver(mask, tau, RHO_IN, RHO_OUT, precision=precision)
    s.step(200)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s.step(steps)
    e1.record()
    torch.cuda.synchronize()
    s.close()
    return e0.elapsed_time(e1) / 1e3 / steps


def evaluate(net, seeds, scales, tol=1e-9, max_steps=600000, precision="fp64", log=None,
             tta=False):
    """Zero, linear-density and learned starts on the samples `seeds`: per-sample
    steps and permeabilities, the wall time of each batch job (the learned
    start's includes inference, the field conversion and lbm_set_macro), and
    per sample the time until its permeability stays within K_TOL of the
    converged value, as if it ran alone: its steps to that point times the
    step time of one sample alone, plus its share of the start's own work.
    tta: the learned start averages the predictions of the mirror images."""
    smp = [sample(s) for s in seeds]
    masks = [m for m, _, _ in smp]
    taus = [t for _, t, _ in smp]
    out = {"seeds": list(seeds), "tau": taus, "precision": precision}
    out["step_seconds_alone"] = step_seconds(masks[0], taus[0], precision)

    def zero(b):
        pass

    def linear(b):
        for s in b.solvers:
            s.reset("linear")

    info = {}
    ref = {}

    def keep_fields(b):
        for s in b.solvers:
            s.smooth(SMOOTH_PASSES)
        rho = np.stack([s.macro("float32")[0].cpu().numpy()[0] for s in b.solvers])
        u = np.stack([s.macro("float32")[1].cpu().numpy()[:, 0] for s in b.solvers])
        ref["rho"], ref["u"] = rho, u

    def learned(b):
        rho, u, bad = predict(net, masks, taus, scales, tta=tta)
        info["pred"] = (rho.cpu().numpy(), u.cpu().numpy())
        badh = bad.cpu().numpy()
        for j, s in enumerate(b.solvers):
            if badh[j]:
                s.reset("uniform")                 # fallback: the plain start
            else:
                s.set_macro(rho[j], u[j])
                s.smooth(SMOOTH_PASSES)
        info["fallbacks"] = int(badh.sum())

    # the zero start is the plain method: judged by the same check, never rerun
    for name, fn in (("zero", zero), ("linear", linear), ("learned", learned)):
        out[name] = run_checked(masks, taus, fn, precision, tol, max_steps,
                                rerun_failed=name != "zero",
                                after=keep_fields if name == "zero" else None)
    out["learned"]["fallbacks"] = info["fallbacks"]
    for name in ("zero", "linear", "learned"):
        r = out[name]
        r["seconds_to_k_tol"] = (np.array(r["steps_to_k_tol"]) * out["step_seconds_alone"] +
                                 r["start_seconds"] / len(masks)).tolist()
    out["prediction_error"] = field_errors(info["pred"][0], info["pred"][1], ref["rho"], ref["u"],
                                           np.stack(masks), np.asarray(taus), scales)
    kz = np.array(out["zero"]["k"])
    okz = np.array(out["zero"]["status"]) == lbm.LBM_OK
    for name in ("linear", "learned"):
        both = okz & (np.array(out[name]["status"]) == lbm.LBM_OK)
        e = np.abs(np.array(out[name]["k"]) - kz) / np.abs(kz)
        out[name]["k_rel_err_max"] = float(e[both].max()) if both.any() else float("nan")
        out[name]["k_compared"] = int(both.sum())
    if log:
        for name in ("zero", "linear", "learned"):
            s = np.array(out[name]["steps"])
            a = np.array(out[name]["steps_to_k_tol"])
            t = np.array(out[name]["seconds_to_k_tol"])
            log(f"{name:8s}: steps median {np.median(s):.0f} p90 {np.percentile(s, 90):.0f}, "
                f"to k within {K_TOL:g}: median {np.median(a):.0f} steps, "
                f"{np.median(t) * 1e3:.1f} ms per sample alone (sum {t.sum():.2f} s); batch "
                f"{out[name]['seconds']:.2f} s, reruns {out[name]['reruns']}")
        pe = {k: ({kk: vv for kk, vv in v.items() if kk != "per_sample"}) for k, v in
              out["prediction_error"].items()}
        log(f"prediction error (network units): {pe}")
    return out


def start_gains(ev, keys=("steps_to_k_tol", "seconds_to_k_tol", "steps")):
    """The learned start against the zero and linear starts of an `evaluate`
    result, over the samples that all three bring to the residual: for each
    measure the ratio of the sums and of the medians (below 1: the learned
    start is faster) and the share of samples on which it is faster."""
    names = ("zero", "linear", "learned")
    ok = np.ones(len(ev["seeds"]), bool)
    for n in names:
        ok &= np.array(ev[n]["status"]) == lbm.LBM_OK
    out = {"samples": int(ok.sum())}
    for key in keys:
        a = {n: np.asarray(ev[n][key], float)[ok] for n in names}
        r = {}
        for base in ("zero", "linear"):
            r[f"sum_vs_{base}"] = float(a["learned"].sum() / a[base].sum())
            r[f"median_vs_{base}"] = float(np.median(a["learned"]) / np.median(a[base]))
            r[f"faster_than_{base}"] = float(np.mean(a["learned"] < a[base]))
        out[key] = r
    return out
