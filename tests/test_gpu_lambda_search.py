"""The lambda search of Sec. 3.2 with its coarse scan as one batched solve
(per-item weights, the measurement replicated over the batch) against an
oracle-side scan over the same lambda values: every item's z^K matches the
oracle's FISTA solution, its NCC with the reference (eq. (17)) matches the
oracle's, and both pick the same lambda.  Per-item solves also equal the
one-at-a-time GPU solves."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pen", ["l1", "tv", "haar"])
def test_batched_lambda_scan_matches_oracle_scan(pen):
    import torch
    import paper_2108_01438_amd as P
    from paper_2108_01438_amd.tune import scan_lambda_batched
    kw = dict(n_depth=128, n_x=48, n_k=128)
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(61)
    x_true = synth.scatterers(rng, O.img_shape(og), 15)
    y_full = synth.noisy(O.forward(x_true, og), synth.standard_normal(rng, O.meas_shape(og)), None, 0.01)
    mask = synth.mask_equispaced((1, og.n_x), og.n_k)
    y32 = (y_full * mask[None]).astype(np.float32)
    y64 = y32.astype(np.float64)
    ref64 = O.direct_isam(y_full.astype(np.float32).astype(np.float64), og)
    ref32 = ref64.astype(np.complex64)
    lam_max = O.lambda_max(y64, og, mask)
    delta = O.step_size(O.lipschitz(og, mask, iters=30))
    us = list(np.linspace(-4.0, -0.5, 8))
    pid = {"l1": O.PEN_L1, "tv": O.PEN_TV, "haar": O.PEN_HAAR}[pen]
    iters = 30
    flush(f"[lambda scan] oracle, {pen}")
    zo, no = [], []
    for u in us:
        z, _ = O.fista(y64, og, mask, pid, lam_max * 10.0 ** u, delta, iters, tv_inner=10, haar_levels=3)
        zo.append(z)
        no.append(O.ncc(z, ref64))
    flush(f"[lambda scan] batched GPU scan, {pen}")
    import dataclasses
    plan_b = P.Plan(dataclasses.replace(pg, batch=len(us)), mask)
    scan, zb = scan_lambda_batched(plan_b, to_dev(y32), to_dev(ref32), pen, lam_max, delta, us, iters)
    zb = to_host(zb)
    ng = [v for _, v in scan]
    plan1 = P.Plan(pg, mask)
    for b, u in enumerate(us):
        e = rel(zb[b:b + 1], zo[b])
        assert e <= 1e-4, (u, e)
        assert abs(ng[b] - no[b]) <= 1e-5, (u, ng[b], no[b])
        z1, _ = plan1.mbir_solve(to_dev(y32), pen, lam_max * 10.0 ** u, iters, delta=delta)
        assert rel(zb[b:b + 1], to_host(z1)) <= 1e-5
    assert int(np.argmax(ng)) == int(np.argmax(no))
    top = sorted(no)[-2:]
    print(f"[lambda scan] {pen}: best u {us[int(np.argmax(no))]:.2f}, NCC {max(no):.5f} "
          f"(runner-up {top[0]:.5f}); worst |dNCC| {max(abs(a - b) for a, b in zip(ng, no)):.2e}")
    torch.cuda.synchronize()


def test_per_item_weights_reject_unsupported():
    import dataclasses
    import paper_2108_01438_amd as P
    og, pg = both_geoms(n_depth=64, n_x=16, n_k=64)
    plan = P.Plan(dataclasses.replace(pg, batch=2))
    y = to_dev(np.zeros((2, 1, 16, 64), np.float32))
    for kw, st in ((dict(objective=True), P.OCT_E_UNSUPPORTED), (dict(bound=1.0), P.OCT_E_UNSUPPORTED)):
        with pytest.raises(P.OctError) as e:
            plan.mbir_solve(y, "l1", [1.0, 2.0], 3, delta=1e-3, **kw)
        assert e.value.status == st
    with pytest.raises(P.OctError) as e:
        plan.mbir_solve(y, "l1", [1.0, -2.0], 3, delta=1e-3)
    assert e.value.status == P.OCT_E_INVALID


def test_per_item_weights_fully_observed_match_oracle():
    """Per-item weights on a fully observed plan (the residual seam in the
    lateral-frequency domain, the measurement's lateral spectrum formed from
    the per-item scaled measurements): every item's z^K matches the oracle's
    FISTA at its own lambda (eq. (15))."""
    import dataclasses
    import paper_2108_01438_amd as P
    og, pg = both_geoms(n_depth=64, n_x=16, n_k=64)
    rng = np.random.default_rng(67)
    x_true = synth.scatterers(rng, O.img_shape(og), 8)
    y = synth.noisy(O.forward(x_true, og), synth.standard_normal(rng, O.meas_shape(og)), None, 0.01)
    y32 = y.astype(np.float32)
    y64 = y32.astype(np.float64)
    lam_max = O.lambda_max(y64, og, None)
    delta = O.step_size(O.lipschitz(og, None, iters=30))
    lams = [lam_max * f for f in (0.02, 0.1, 0.3)]
    flush("[per-item weights, fully observed] oracle")
    zo = [O.fista(y64, og, None, O.PEN_L1, lam, delta, 20)[0] for lam in lams]
    plan = P.Plan(dataclasses.replace(pg, batch=len(lams)))
    yb = np.repeat(y32, len(lams), axis=0)
    z, _ = plan.mbir_solve(to_dev(yb), "l1", lams, 20, delta=delta)
    z = to_host(z)
    for b in range(len(lams)):
        assert rel(z[b:b + 1], zo[b]) <= 1e-4, b
