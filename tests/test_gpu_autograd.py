"""torch.autograd through the HIP operator: gradients against the FP64 oracle
and FP64 central finite differences of the oracle's loss."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rand_image, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_phi_backward_is_adjoint_small():
    import torch
    import paper_2108_01438_amd as P
    from paper_2108_01438_amd.autograd import phi
    flush("[autograd] small B-scan, masked")
    og, pg = both_geoms(n_depth=128, n_x=40, n_k=160, batch=2, disp_b=1e-6)
    rng = np.random.default_rng(21)
    mask = (rng.random((1, 40, 160)) < 0.6).astype(np.uint8)
    plan = P.Plan(pg, mask)
    x32, x64 = rand_image(rng, O.img_shape(og))
    y32 = (rng.standard_normal(O.meas_shape(og)) * mask[None]).astype(np.float32)
    x = to_dev(x32).requires_grad_(True)
    yd = to_dev(y32)
    loss = 0.5 * ((phi(x, plan) - yd) ** 2).sum()
    loss.backward()
    g_or, _ = O.grad(x64, y32.astype(np.float64), og, mask)
    assert rel(to_host(x.grad), g_or) <= 1e-5
    # the data-loss function: FP64 loss and fused gradient
    from paper_2108_01438_amd.autograd import data_loss
    x2 = to_dev(x32).requires_grad_(True)
    l2 = data_loss(x2, yd, plan)
    l2.backward()
    lo = O.data_loss(x64, y32.astype(np.float64), og, mask)
    assert abs(float(l2.item()) - lo) <= 1e-5 * lo
    assert rel(to_host(x2.grad), g_or) <= 1e-5
    assert l2.dtype == torch.float64


def test_batch32_gradient_oracle_and_finite_differences():
    """32 B-scans of 1024 x 512, x0 ~ CN(0,1), y = Phi x0 + 1% noise: the
    gradient of 1/2||Phi x - y||^2 at a random x against the oracle gradient
    (relative L2 <= 1e-5) and against FP64 central differences of the oracle
    loss along 20 random directions (step 1e-6, relative error <= 1e-5); each
    direction lives on one batch item, so each difference needs that item only."""
    import paper_2108_01438_amd as P
    from paper_2108_01438_amd.autograd import data_loss
    pr = synth.preset("batch32_1024x512_grad")
    og, pg = both_geoms(**pr["geom"])
    rng = np.random.default_rng(3)
    flush("[autograd] batch 32 x 1024 x 512: oracle data")
    x0 = synth.complex_normal(rng, O.img_shape(og))
    y_clean = O.forward(x0, og)
    y32 = synth.noisy(y_clean, synth.standard_normal(rng, y_clean.shape), None, pr["noise"]).astype(np.float32)
    x32, x64 = rand_image(rng, O.img_shape(og))
    plan = P.Plan(pg)
    x = to_dev(x32).requires_grad_(True)
    loss = data_loss(x, to_dev(y32), plan)
    loss.backward()
    g = to_host(x.grad).astype(np.complex128)
    flush("[autograd] oracle gradient")
    g_or, _ = O.grad(x64, y32.astype(np.float64), og)
    err = rel(g, g_or)
    print(f"[autograd] batch32 gradient rel err vs oracle {err:.3e}")
    assert err <= 1e-5
    flush("[autograd] 20 central differences")
    og1 = og.with_(batch=1)
    h = 1e-6
    worst = 0.0
    for _ in range(20):
        b = int(rng.integers(0, og.batch))
        d = synth.complex_normal(rng, O.img_shape(og1))
        yb = y32[b:b + 1].astype(np.float64)
        fp = O.data_loss(x64[b:b + 1] + h * d, yb, og1)
        fm = O.data_loss(x64[b:b + 1] - h * d, yb, og1)
        fd = (fp - fm) / (2 * h)
        an = float(np.real(np.vdot(g[b:b + 1], d)))
        worst = max(worst, abs(fd - an) / abs(fd))
    print(f"[autograd] worst FD relative error {worst:.3e}")
    assert worst <= 1e-5
