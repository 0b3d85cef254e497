"""The learned warm start end to end on the GPU, at the warm-start size
(256 x 128 D2Q9 masks): solver-generated steady states, U-Net training with
the HIP kernels, and the start it gives against the zero and linear starts.

Reduced budget (4096 training samples, 20 epochs, 96 held-out samples) so
that the module runs in about a minute and a half; the full-size figures come from
``python -m paper_1609_09685_amd.train_warmstart``.  Everything is seeded and
the kernels are deterministic, so the figures repeat exactly.

Checked: training lowers the held-out loss well below the untrained
network's; all but a few held-out samples (the smallest tau, whose zero start
can need more than the 300,000-step budget) converge from every start, the
learned start to the zero start's permeability within 1e-4, with no
fallback; and on the samples all three starts bring to the residual the
learned start gains over both the method without it (the zero start) and
the cheap linear-density start: summed and median steps until k stays within 1e-4 of
its converged value, and the same for the per-sample time to that point
(steps times the step time of one sample alone, plus the start's own work,
inference included), each at most GAIN_BAR times the other start's.
"""
import numpy as np
import pytest
import torch

from paper_1609_09685_amd import lbm, warmstart as ws, wsn

# data and training take about 130 s of the first test's time
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

GAIN_BAR = 0.95     # learned / other start, on sums and medians
N_TRAIN, EPOCHS, N_EVAL = 4096, 20, 96
MAX_UNCONVERGED = 4  # held-out samples allowed to miss the step budget from some start


def _heldout_loss(net, data, scales):
    y = data.targets(scales)
    losses = []
    B = net.batch
    for c0 in range(0, len(data) - B + 1, B):
        p = net.infer(data.x[c0:c0 + B])
        loss, _ = wsn.masked_mse(p, y[c0:c0 + B].contiguous(), data.solid[c0:c0 + B].contiguous())
        losses.append(loss.item())
    return float(np.mean(losses))


@pytest.fixture(scope="module")
def trained():
    torch.cuda.set_device(0)
    log = lambda msg: print(msg, flush=True)    # progress (visible with -s)
    data = ws.generate(range(10000, 10000 + N_TRAIN), chunk=N_TRAIN // 2, max_steps=200000,
                       log=log)
    # ~1 % of random samples (the smallest tau) do not reach the residual
    # within 200,000 steps; they are dropped, not trained on
    assert len(data) >= 0.97 * N_TRAIN, data.dropped
    scales = ws.scales_of(data)
    held = ws.generate(range(21000, 21032), chunk=32, max_steps=200000)
    net = ws.new_network(16, seed=0)
    before = _heldout_loss(net, held, scales)
    hist = ws.train(net, data, scales, epochs=EPOCHS, lr=1e-3, lr_end=5e-5, log=log)
    after = _heldout_loss(net, held, scales)
    del data, held
    torch.cuda.empty_cache()
    return net, scales, hist, before, after


def test_training_lowers_the_loss(trained):
    _, scales, hist, before, after = trained
    print(f"scales {scales}; training loss {hist[0]:.3f} -> {hist[-1]:.4f}; "
          f"held-out {before:.3f} -> {after:.4f}")
    assert hist[-1] < 0.5 * hist[0]
    assert after < 0.35 * before, (before, after)


def test_learned_start_beats_zero_and_linear_starts(trained):
    net, scales = trained[0], trained[1]
    ev = ws.evaluate(net, range(20000, 20000 + N_EVAL), scales, max_steps=300000,
                     log=lambda msg: print(msg, flush=True))
    learned = ev["learned"]
    assert learned["fallbacks"] == 0
    assert learned["k_compared"] >= N_EVAL - MAX_UNCONVERGED
    assert learned["k_rel_err_max"] <= 1e-4, learned["k_rel_err_max"]
    g = ws.start_gains(ev)
    print(f"gains {g}; prediction errors "
          f"{ {k: v for k, v in ev['prediction_error'].items() if k != 'ux_sum_ratio'} }")
    assert g["samples"] >= N_EVAL - MAX_UNCONVERGED
    for key in ("steps_to_k_tol", "seconds_to_k_tol"):
        for ratio in ("sum_vs_zero", "sum_vs_linear", "median_vs_zero", "median_vs_linear"):
            assert g[key][ratio] <= GAIN_BAR, (key, ratio, g[key])
