"""Throughput benchmark of the lattice Boltzmann step on one MI355X.

Default workload: D3Q19 BGK, FP32 deviation storage, 512^3 QSGS porous mask
(porosity 0.6, seed 0), tau = 0.6, density drop 1e-4 along x, symmetric y/z
planes.  One step = one launch of the fused stream-collide kernel over the
whole lattice.  Prints one JSON line with MLUPS (all nodes), the roofline of
the step kernel against HBM bandwidth, and the CPU checker's throughput on a
bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
METRIC = "MLUPS + % HBM roofline (D3Q19 FP32); time-to-converged k, warm vs plain"

WORKLOADS = {
    # name: (lattice, shape (nz, ny, nx), porosity, tau, rho_in, rho_out, precision)
    "d3q19_512_fp32": (19, (512, 512, 512), 0.6, 0.6, 1.00005, 0.99995, "fp32"),
    "d3q19_256_fp32": (19, (256, 256, 256), 0.6, 0.6, 1.00005, 0.99995, "fp32"),
    "d2q9_400x200_fp32": (9, (1, 200, 400), 0.74, 0.8, 1.0005, 0.9995, "fp32"),
    "d2q9_400x200_fp64": (9, (1, 200, 400), 0.74, 0.8, 1.0005, 0.9995, "fp64"),
    "d2q9_100x50_fp64": (9, (1, 50, 100), 0.74, 0.8, 1.0005, 0.9995, "fp64"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_mask(Q, shape, porosity, seed=0):
    from paper_1609_09685_amd.qsgs import qsgs_2d, qsgs_3d
    nz, ny, nx = shape
    if Q == 9:
        return qsgs_2d(nx, ny, porosity, seed)
    return qsgs_3d(nx, ny, nz, porosity, seed)


def cpu_baseline(Q, mask, tau, rho_in, rho_out, budget_s=12.0, threads=None):
    """The CPU checker, as it stands, on a bounded sub-box of the workload, with
    `threads` OpenMP threads (None: all the host offers)."""
    import oracle
    if Q == 19:
        sub = np.ascontiguousarray(mask[:256, :256, :256])
    else:
        sub = mask
    prev = oracle.threads()
    if threads is not None:
        oracle.set_threads(threads)
    try:
        o = oracle.Oracle(Q, sub, tau, rho_in, rho_out)
        o.step(1)
        steps, t0 = 0, time.perf_counter()
        while True:
            o.step(1)
            steps += 1
            dt = time.perf_counter() - t0
            if dt >= budget_s or steps >= 10000:
                break
        used = oracle.threads()
    finally:
        oracle.set_threads(prev)
    n = sub.size
    shape = "x".join(str(s) for s in sub.shape[::-1])
    return {"value": n * steps / dt / 1e6, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"{steps} FP64 steps on the {shape} corner sub-box of the same mask "
                      f"({dt:.1f} s wall)"}


def _function_text(text, signature):
    """Source text of the function that starts with `signature` (up to its
    matching closing brace)."""
    i = text.index(signature)
    j = text.index("{", i)
    depth = 0
    for k in range(j, len(text)):
        if text[k] == "{":
            depth += 1
        elif text[k] == "}":
            depth -= 1
            if depth == 0:
                return text[i:k + 1]
    raise ValueError(signature)


def kernel_source_hash(extra=()):
    """Short hash of what fixes the step kernel's code and launch: its device
    sources, its compiler flags, the step arguments and grid, and the slot
    layout, so that profiled counters are tied to them (host code elsewhere
    may change).
    `extra`: further source files of csrc/ (the batched launcher)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1609_09685_amd", "csrc")
    h = hashlib.sha256()
    for f in ("kernels.h", "pull_index.h", "lattice.h", "step_launch.h", "step_launch.hip",
              *extra):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    ctx = open(os.path.join(csrc, "context.h")).read()
    api = open(os.path.join(csrc, "lbm_api.hip")).read()
    from paper_1609_09685_amd import build as _b
    h.update(repr((_b.HIPCC_FLAGS, _b.STEP_FLAGS)).encode())   # how the step objects are compiled
    for part in (_function_text(ctx, "StepArgs<T> step_args(const lbm_ctx* c)"),
                 _function_text(ctx, "int step_grid(const lbm_ctx* c, const StepArgs<T>& a)"),
                 _function_text(api, "lbm_status make_layout(const lbm_geom* g, Layout* L)")):
        h.update(part.encode())
    return h.hexdigest()[:16]


BATCH_PROFILE = "k_step_batch_c3_fp32"     # counter summary of the batched workload
BATCH_SOURCES = ("lbm_batch.hip",)


def profiled_traffic(name, extra=()):
    """HBM bytes per launch from the committed counter summary
    profiles/<name>_pmc.md, if it was taken on the current kernel sources
    (else None)."""
    path = os.path.join(ROOT, "profiles", f"{name}_pmc.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0].strip() in ("traffic_bytes_per_launch",
                                                              "kernel_source_sha256_16"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256_16") != kernel_source_hash(extra):
        return None
    return int(fields["traffic_bytes_per_launch"])


def stream_ceilings(n_per_array=80_530_432, arrays=19, reps=5):
    """What plain streaming of the step's kind of data reaches on this GPU: the
    hand-written kernels of liblbmprobe.so (include/lbm_probe.h) over `arrays`
    arrays of n floats (the 512^3 workload's fluid populations), timed with HIP
    events on torch's current stream.  GB/s counts the bytes each pass moves."""
    import ctypes
    import torch
    from paper_1609_09685_amd import build as _b
    lib = ctypes.CDLL(_b.PROBE_LIB)
    lib.lbm_probe_stream.restype = ctypes.c_int
    lib.lbm_probe_stream.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]
    n = n_per_array // 1024 * 1024
    src = torch.zeros(arrays * n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(4, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    out = {"arrays": arrays, "floats_per_array": n}
    for name, mode, vec, nt in (("copy_dword_nt", 0, 1, 1), ("copy_dwordx4_nt", 0, 4, 1),
                                ("copy_dword", 0, 1, 0), ("read_dword", 1, 1, 0),
                                ("read_dwordx4", 1, 4, 0), ("write_dword_nt", 2, 1, 1),
                                ("write_dwordx4_nt", 2, 4, 1)):
        def run():
            rc = lib.lbm_probe_stream(mode, vec, nt, arrays, n, src.data_ptr(), dst.data_ptr(),
                                      sink.data_ptr(), ctypes.c_void_p(st.cuda_stream))
            if rc != 0:
                raise RuntimeError(f"lbm_probe_stream failed ({rc})")
        run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        moved = arrays * n * 4 * (2 if mode == 0 else 1)
        out[name] = round(moved / (ms / 1e3) / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    return out


C3_SIZES = [(400, 200), (800, 400), (1200, 600)]


def c3_samples(n=256, seed0=1000):
    """Batched D2Q9 workload: sample j uses seed 1000 + j for its size (uniform over
    400x200, 800x400, 1200x600), porosity U[0.6, 0.9], tau U[0.51, 1.0] and mask."""
    from paper_1609_09685_amd.qsgs import qsgs_2d
    out = []
    for j in range(n):
        rng = np.random.default_rng(seed0 + j)
        nx, ny = C3_SIZES[int(rng.integers(0, 3))]
        phi = float(rng.uniform(0.6, 0.9))
        tau = float(rng.uniform(0.51, 1.0))
        out.append((qsgs_2d(nx, ny, phi, seed0 + j), tau, phi))
    return out


def bench_batch(args):
    """256 independent D2Q9 FP32 samples advanced by one launch per step; the
    timed region is whole check windows (K = 100 steps each, replayed as a HIP
    graph, with the batched FP64 flux reduction and the host residual check)."""
    import torch
    from paper_1609_09685_amd import lbm
    t0 = time.time()
    samples = c3_samples(args.batch)
    log(f"{len(samples)} masks in {time.time() - t0:.1f} s")
    torch.cuda.set_device(0)
    masks = [m for m, _, _ in samples]
    taus = [t for _, t, _ in samples]
    t0 = time.time()
    b = lbm.Batch.from_masks(masks, taus, 1.0005, 0.9995, precision="fp32",
                             autotune=args.autotune, graph=not args.no_graph)
    log(f"batch of {b.n} solvers in {time.time() - t0:.1f} s")
    N = sum(int(m.size) for m in masks)
    n_fluid = sum(s.n_fluid for s in b.solvers)
    K = 100
    warm = max(K, (args.warmup + K - 1) // K * K)
    steps = max(K, (args.steps + K - 1) // K * K)
    b.run_to_steady(0.0, warm)          # tol 0: never converges, runs whole windows
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    b.run_to_steady(0.0, warm + steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_step = ms / steps
    # plain stepping without checks, for comparison
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms_plain = e0.elapsed_time(e1) / steps
    alg_bytes = n_fluid * 2 * 9 * 4 + N
    achieved = alg_bytes / (ms_step / 1e3) / 1e9
    to_steady = c3_to_steady(b, masks, taus, n_fluid) if args.to_steady else None
    out = {
        "metric": METRIC,
        "value": round(N * steps / (ms / 1e3) / 1e6, 1),
        "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": warm,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched D2Q9 BGK fp32 deviation storage: {b.n} QSGS samples, "
                               "sizes 400x200/800x400/1200x600, porosity U[0.6,0.9], tau "
                               "U[0.51,1.0], rho 1.0005/0.9995; check windows of 100 steps as "
                               "HIP graphs" + (" (off)" if args.no_graph else ""),
                   "name": "c3_batch_fp32", "samples": b.n, "nodes": N, "fluid_nodes": n_fluid,
                   "mflups": round(n_fluid * steps / (ms / 1e3) / 1e6, 1),
                   "ms_per_step_without_checks": round(ms_plain, 5),
                   "autotune": bool(args.autotune)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(BATCH_PROFILE, BATCH_SOURCES)
                     if (b.n, args.autotune, args.no_graph) == (256, False, False) else None,
                     "kernel": "k_step_batch", "algorithmic_bytes_per_launch": alg_bytes},
    }
    if to_steady is not None:
        out["to_steady"] = to_steady
    # the same probes as the headline, over 9 arrays of the batch's fluid size
    out["stream_ceilings"] = stream_ceilings(n_per_array=n_fluid, arrays=9)
    log(f"stream ceilings (GB/s): {out['stream_ceilings']}")
    print(json.dumps(out), flush=True)


def c3_to_steady(b, masks, taus, n_fluid, tol=1e-9, max_steps=3_000_000, n_check=4):
    """Every sample of the batch from rest to the flux residual tol (K = 100):
    wall time, outcome counts, the steps distribution, and, for n_check samples
    spread over the batch, k and steps against the same solver run alone."""
    import torch
    from paper_1609_09685_amd import lbm
    for s in b.solvers:
        s.reset("uniform")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, steps, resid = b.run_to_steady(tol, max_steps)
    k, kst = b.permeability()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ok = status == lbm.LBM_OK
    log(f"to steady: {int(ok.sum())}/{b.n} converged in {wall:.1f} s")
    updates = sum(s.n_fluid * int(n) for s, n in zip(b.solvers, steps))
    picks = sorted({int(round(j)) for j in np.linspace(0, b.n - 1, n_check)})
    checks = []
    for j in picks:
        s = lbm.Solver(masks[j], taus[j], 1.0005, 0.9995, precision=b.solvers[j].precision)
        st, n1, _ = s.run_to_steady(tol, max_steps, raise_on_notconv=False)
        k1 = s.permeability() if st else float("nan")
        checks.append({"sample": j, "steps_batch": int(steps[j]), "steps_alone": int(n1),
                       "k_batch": float(k[j]), "k_alone": float(k1),
                       "bitwise_equal": bool(np.float64(k[j]).view(np.uint64) ==
                                             np.float64(k1).view(np.uint64))})
        s.close()
    q = np.percentile(steps[ok], [0, 50, 90, 100]) if ok.any() else [0, 0, 0, 0]
    return {"tol": tol, "wall_s": round(wall, 2), "converged": int(ok.sum()),
            "not_converged": int((status == lbm.LBM_ENOTCONV).sum()),
            "non_finite": int((status == lbm.LBM_ENONFINITE).sum()),
            "non_finite_taus": [round(float(taus[j]), 4) for j in np.flatnonzero(
                status == lbm.LBM_ENONFINITE)],
            "steps_min_median_p90_max": [int(v) for v in q],
            "fluid_node_updates": int(updates),
            "mflups_over_run": round(updates / wall / 1e6, 1),
            "single_run_checks": checks}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="d3q19_512_fp32",
                    choices=sorted(WORKLOADS) + ["c3_batch_fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--xcd-remap", type=int, default=1)
    ap.add_argument("--band", type=int, default=16, help="banded tile order (tile rows per band; 0: off)")
    ap.add_argument("--batch", type=int, default=256, help="samples of the batched workload")
    ap.add_argument("--autotune", action="store_true", help="batched workload: tune tile orders")
    ap.add_argument("--no-graph", action="store_true", help="batched workload: plain launches")
    ap.add_argument("--to-steady", action="store_true",
                    help="batched workload: also run every sample to the 1e-9 residual")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the multi-GPU slab "
                                   "decomposition is not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "c3_batch_fp32":
        return bench_batch(args)

    import torch
    from paper_1609_09685_amd import lbm

    Q, shape, phi, tau, rin, rout, prec = WORKLOADS[args.workload]
    t0 = time.time()
    mask = make_mask(Q, shape, phi)
    log(f"mask {shape} porosity {1 - mask.mean():.4f} in {time.time() - t0:.1f} s")
    torch.cuda.set_device(0)
    s = lbm.Solver(mask, tau, rin, rout, precision=prec, lattice=Q)
    s.configure(xcd_remap=args.xcd_remap, band=args.band)
    N = int(mask.size)
    n_fluid = int((mask == 0).sum())
    esize = 8 if prec == "fp64" else 4
    s.step(args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} steps done")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    s.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_step = ms / args.steps
    log(f"timed {args.steps} steps: {ms_step:.4f} ms/step")
    k = s.permeability()
    log(f"k after {s.steps} steps = {k:.6e}")
    mlups = N * args.steps / (ms / 1e3) / 1e6
    alg_bytes = n_fluid * 2 * Q * esize + N * 1
    achieved = alg_bytes / (ms_step / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"D{'3Q19' if Q == 19 else '2Q9'} BGK {prec} deviation storage, "
                               f"{'x'.join(map(str, shape[::-1]))} QSGS mask porosity {phi}, "
                               f"tau {tau}, rho {rin}/{rout}, pressure x, symmetric y/z",
                   "name": args.workload, "nodes": N, "fluid_nodes": n_fluid,
                   "mflups": round(n_fluid * args.steps / (ms / 1e3) / 1e6, 1)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": profiled_traffic(f"k_step_{args.workload}")
                     if (args.band, args.xcd_remap) == (16, 1) else None,
                     "kernel": "k_step", "algorithmic_bytes_per_launch": alg_bytes},
    }
    out["stream_ceilings"] = stream_ceilings(arrays=Q)
    log(f"stream ceilings (GB/s): {out['stream_ceilings']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (all host threads, then one) ...")
        out["cpu_baseline"] = cpu_baseline(Q, mask, tau, rin, rout)
        out["cpu_baseline"]["single_core"] = cpu_baseline(Q, mask, tau, rin, rout, threads=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
