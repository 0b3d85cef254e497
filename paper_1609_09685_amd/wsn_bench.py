"""Timing of the warm-start U-Net's training iteration on the GPU, and the
multiply-add count of its convolutions (the network's dense contractions,
which run on the FP32 matrix cores).

    python -m paper_1609_09685_amd.wsn_bench [--batch 32] [--iters 20]

Inputs are seeded random masks, features and targets of the warm-start size
(256 x 128); the timing does not depend on the values.  Under a kernel trace
the per-kernel times divided into conv_flops() give each convolution kernel's
rate.
"""
import argparse
import json
import sys
import time

import numpy as np


def conv_flops(batch, height=128, width=256, levels=4, base=32, in_ch=2, out_ch=3):
    """FLOPs (2 per multiply-add) of one forward pass through every
    convolution: {"conv3x3": ..., "conv1x1": ...}.  The data and weight
    gradients of a 3x3 layer cost the same as its forward pass each."""
    ch = [base * 2 ** l for l in range(levels)]
    f3 = 0
    cin = in_ch
    for l in range(levels):
        px = batch * (height >> l) * (width >> l)
        f3 += 2 * px * 9 * (cin * ch[l] + ch[l] * ch[l])
        cin = ch[l]
    for l in range(levels - 2, -1, -1):
        px = batch * (height >> l) * (width >> l)
        f3 += 2 * px * 9 * ((ch[l + 1] + ch[l]) * ch[l] + ch[l] * ch[l])
    f1 = 2 * batch * height * width * ch[0] * out_ch
    return {"conv3x3": f3, "conv1x1": f1}


def main(argv=None):
    import torch

    from . import warmstart, wsn

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    B, H, W = a.batch, warmstart.NY, warmstart.NX
    net = warmstart.new_network(B, seed=0)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    solid = (torch.rand((B, H, W), generator=g, device="cuda") < 0.3).to(torch.uint8)
    feat = torch.rand((B,), generator=g, device="cuda")
    x = wsn.pack_input(solid, feat)
    target = torch.randn((B, H, W, 3), generator=g, device="cuda")
    for _ in range(a.warmup):
        net.train_step(x, target, solid, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.iters):
        net.train_step(x, target, solid, 1e-4)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / a.iters * 1e3
    f = conv_flops(B, H, W)
    out = {"batch": B, "height": H, "width": W, "ms_per_iteration": ms,
           "conv3x3_forward_gflop": f["conv3x3"] / 1e9,
           "iteration_conv3x3_gflop": 3 * f["conv3x3"] / 1e9,
           "iteration_tflops_conv3x3": 3 * f["conv3x3"] / (ms * 1e-3) / 1e12}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
