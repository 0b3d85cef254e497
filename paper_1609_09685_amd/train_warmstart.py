"""Trains the warm-start network on solver steady states and measures the start
it gives (zero vs linear-density vs learned), all on one GPU.

    python -m paper_1609_09685_amd.train_warmstart --train 4096 --test 256 \
        --epochs 20 --out warmstart.npz --report report.json

Training samples use seeds 10000 + j, held-out samples 20000 + j (porosity
U[0.6, 0.9], tau U[0.51, 1.0], 256 x 128 QSGS masks).  The parameters, the
velocity scale and the measurements are written to --out (NumPy .npz, no
pickles) and --report (JSON).  --augment adds the three mirror images of every
training state (``warmstart.MIRRORS``); --tta averages the learned start's
predictions over the mask's mirror images; --profile gives the network the
masks' resistance profile along x as a third input.
"""
import argparse
import json
import sys
import time

import numpy as np


def log(msg):
    print(f"[warmstart] {msg}", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=4096)
    ap.add_argument("--test", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-end", type=float, default=2e-5)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"],
                    help="solver storage for the training data")
    ap.add_argument("--eval-precision", default="fp64", choices=["fp32", "fp64"],
                    help="solver storage for the start comparison")
    ap.add_argument("--max-steps", type=int, default=200000)
    ap.add_argument("--eval-max-steps", type=int, default=600000)
    ap.add_argument("--chunk", type=int, default=1024, help="samples per data-generation batch")
    ap.add_argument("--augment", action="store_true",
                    help="train on the data and its three mirror images (symmetries of the setup)")
    ap.add_argument("--levels", type=int, default=4,
                    help="U-Net levels (4: the configuration's network)")
    ap.add_argument("--profile", action="store_true",
                    help="third network input: the masks' resistance profile along x")
    ap.add_argument("--rho-weight", type=float, default=1.0,
                    help="weight of the density channel in the loss (its target scale / sqrt(w))")
    ap.add_argument("--tta", action="store_true",
                    help="learned start: average the predictions of the mask's mirror images")
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    args = ap.parse_args(argv)

    import torch
    from . import warmstart as ws

    torch.cuda.set_device(0)
    rep = {"args": vars(args)}
    t0 = time.perf_counter()
    in_ch = 3 if args.profile else 2
    data = ws.generate(range(10000, 10000 + args.train), chunk=args.chunk,
                       precision=args.precision, max_steps=args.max_steps, log=log, in_ch=in_ch)
    torch.cuda.synchronize()
    rep["data_seconds"] = time.perf_counter() - t0
    rep["train_samples_kept"] = len(data)
    rep["train_samples_dropped"] = data.dropped
    rep["train_steps_median"] = float(np.median(data.steps))
    log(f"data: {len(data)} samples kept in {rep['data_seconds']:.1f} s, dropped {data.dropped}")
    scales = ws.scales_of(data)
    if args.rho_weight <= 0:
        raise SystemExit("--rho-weight must be > 0")
    scales = (scales[0], scales[1] / float(np.sqrt(args.rho_weight)))
    rep["u_scale"], rep["rho_scale"] = scales
    net = ws.new_network(args.batch, seed=0, levels=args.levels, in_ch=in_ch)
    t0 = time.perf_counter()
    hist = ws.train(net, data, scales, epochs=args.epochs, lr=args.lr, lr_end=args.lr_end, log=log,
                    augment=args.augment)
    torch.cuda.synchronize()
    rep["train_seconds"] = time.perf_counter() - t0
    rep["loss_per_epoch"] = hist
    iters = args.epochs * ((4 if args.augment else 1) * len(data) // args.batch)
    rep["train_iterations"] = iters
    rep["ms_per_iteration"] = 1e3 * rep["train_seconds"] / max(iters, 1)
    log(f"training: {iters} iterations in {rep['train_seconds']:.1f} s "
        f"({rep['ms_per_iteration']:.1f} ms each)")
    del data
    torch.cuda.empty_cache()
    ev = ws.evaluate(net, range(20000, 20000 + args.test), scales, max_steps=args.eval_max_steps,
                     precision=args.eval_precision, log=log, tta=args.tta)
    rep["eval"] = ev
    summary = {}
    for name in ("zero", "linear", "learned"):
        s = np.array(ev[name]["steps"])
        a = np.array(ev[name]["steps_to_k_tol"])
        summary[name] = {"steps_median": float(np.median(s)), "steps_p90": float(np.percentile(s, 90)),
                         "steps_total": int(s.sum()), "seconds": ev[name]["seconds"],
                         "steps_to_k_tol_median": float(np.median(a)),
                         "steps_to_k_tol_p90": float(np.percentile(a, 90)),
                         "steps_to_k_tol_total": int(a.sum()),
                         "seconds_to_k_tol_median": float(np.median(ev[name]["seconds_to_k_tol"])),
                         "seconds_to_k_tol_total": float(np.sum(ev[name]["seconds_to_k_tol"])),
                         "converged": int(sum(1 for v in ev[name]["status"] if v == 0))}
    for name in ("linear", "learned"):
        summary[name]["k_rel_err_max"] = ev[name]["k_rel_err_max"]
    summary["learned"]["fallbacks"] = ev["learned"]["fallbacks"]
    for name in ("zero", "linear", "learned"):
        summary[name]["reruns"] = ev[name]["reruns"]
    z, l = np.array(ev["zero"]["steps"]), np.array(ev["learned"]["steps"])
    summary["learned"]["step_ratio_median"] = float(np.median(l / z))
    za, la = np.array(ev["zero"]["steps_to_k_tol"]), np.array(ev["learned"]["steps_to_k_tol"])
    summary["learned"]["k_tol_step_ratio_median"] = float(np.median(la / za))
    summary["prediction_error"] = ev["prediction_error"]
    summary["gains"] = ws.start_gains(ev)
    summary["step_seconds_alone"] = ev["step_seconds_alone"]
    rep["summary"] = summary
    log(json.dumps(summary))
    if args.out:
        np.savez(args.out, params=net.params.cpu().numpy(), u_scale=np.array(scales[0]),
                 rho_scale=np.array(scales[1]),
                 levels=np.array(args.levels), base=np.array(32), in_ch=np.array(in_ch))
    if args.report:
        with open(args.report, "w") as fh:
            json.dump(rep, fh, indent=1)
    return rep


if __name__ == "__main__":
    main(sys.argv[1:])
