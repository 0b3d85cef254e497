"""The learned warm start end to end on the GPU, at the warm-start size
(256 x 128 D2Q9 masks): solver-generated steady states, U-Net training with
the HIP kernels, and the start it gives against the zero and linear starts.

Reduced budget (2048 training samples, 10 epochs, 48 held-out samples) so the
test runs in about a minute; the full-size figures come from
``python -m paper_1609_09685_amd.train_warmstart``.  Checked: training lowers
the held-out loss well below the untrained network's; every held-out sample
that converges from the zero start converges from the learned start to the
same permeability within 1e-4; no prediction needed the fallback; and the
learned start does not need more steps than the zero start.
"""
import numpy as np
import pytest
import torch

from paper_1609_09685_amd import lbm, warmstart as ws, wsn

pytestmark = pytest.mark.gpu


def _heldout_loss(net, data, u_scale):
    y = data.targets(u_scale)
    losses = []
    B = net.batch
    for c0 in range(0, len(data) - B + 1, B):
        p = net.infer(data.x[c0:c0 + B])
        loss, _ = wsn.masked_mse(p, y[c0:c0 + B].contiguous(), data.solid[c0:c0 + B].contiguous())
        losses.append(loss.item())
    return float(np.mean(losses))


def test_learned_start_end_to_end():
    torch.cuda.set_device(0)
    data = ws.generate(range(10000, 12048), chunk=2048, max_steps=200000)
    assert len(data) >= 2000
    u_scale = ws.u_scale_of(data)
    held = ws.generate(range(21000, 21032), chunk=32, max_steps=200000)
    net = ws.new_network(16, seed=0)
    before = _heldout_loss(net, held, u_scale)
    hist = ws.train(net, data, u_scale, epochs=10, lr=1e-3, lr_end=5e-5)
    after = _heldout_loss(net, held, u_scale)
    assert hist[-1] < 0.5 * hist[0]
    assert after < 0.2 * before, (before, after)

    ev = ws.evaluate(net, range(20000, 20048), u_scale, max_steps=300000)
    zero, learned = ev["zero"], ev["learned"]
    assert learned["fallbacks"] == 0
    assert learned["k_rel_err_max"] <= 1e-4, learned["k_rel_err_max"]
    assert learned["k_compared"] >= 45
    z, l = np.array(zero["steps"]), np.array(learned["steps"])
    za, la = np.array(zero["steps_to_k_tol"]), np.array(learned["steps_to_k_tol"])
    both = (np.array(zero["status"]) == lbm.LBM_OK) & (np.array(learned["status"]) == lbm.LBM_OK)
    print(f"held-out loss {before:.3f} -> {after:.4f}; steps to the residual: zero "
          f"{z[both].sum()} learned {l[both].sum()}; steps to k within 1e-4: zero "
          f"{za[both].sum()} learned {la[both].sum()}; errors {ev['prediction_error']}")
    assert la[both].sum() <= 1.02 * za[both].sum()
    assert l[both].sum() <= 1.02 * z[both].sum()
