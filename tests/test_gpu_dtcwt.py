"""The DT-CWT penalty of Sec. 2.2 (B-scans and volumes) through the C ABI
against the FP64 oracle on the same float32 inputs: the shrinkage step at
several sizes and levels (and the full B-scan), perfect reconstruction at
tau = 0, FISTA with its objective history, and the rejected cases."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rand_image, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

PROX_TOL = 1e-5
SOLVE_TOL = 1e-4

CASES = [
    (dict(n_depth=64, n_x=40, n_k=64, batch=2), 3, 0.3),
    (dict(n_depth=96, n_x=24, n_k=64), 1, 0.2),
    (dict(n_depth=128, n_x=64, n_k=64), 4, 0.5),
    (dict(n_depth=32, n_x=32, n_k=32), 5, 0.1),
    (dict(n_depth=1024, n_x=600, n_k=64), 3, 0.3),
]


@pytest.mark.parametrize("kw,levels,tau", CASES)
def test_prox_dtcwt_matches_oracle(kw, levels, tau):
    import paper_2108_01438_amd as P
    flush(f"[dtcwt prox] {kw} levels={levels}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(90)
    v32, v64 = rand_image(rng, O.img_shape(og))
    plan = P.Plan(pg)
    z = to_host(plan.prox("dtcwt", tau, 1.0, to_dev(v32), haar_levels=levels))
    assert rel(z, O.prox_dtcwt(v64, tau, (3, 2), levels)) <= PROX_TOL
    z0 = to_host(plan.prox("dtcwt", 0.0, 1.0, to_dev(v32), haar_levels=levels))
    assert rel(z0, v64) <= 2e-6
    plan.close()


def test_prox_dtcwt_full_bscan():
    import paper_2108_01438_amd as P
    flush("[dtcwt prox] 2048 x 1000")
    og, pg = both_geoms(n_depth=2048, n_x=1000, n_k=2048)
    rng = np.random.default_rng(91)
    v32, v64 = rand_image(rng, O.img_shape(og))
    plan = P.Plan(pg)
    z = to_host(plan.prox("dtcwt", 0.4, 1.0, to_dev(v32), haar_levels=3))
    assert rel(z, O.prox_dtcwt(v64, 0.4, (3, 2), 3)) <= PROX_TOL
    plan.close()


VOL_CASES = [
    (dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=32), 2, 0.3),
    (dict(n_depth=64, n_x=32, n_y=16, lateral_dims=2, n_k=32, batch=2), 3, 0.2),
    (dict(n_depth=16, n_x=16, n_y=16, lateral_dims=2, n_k=16), 4, 0.1),
]


@pytest.mark.parametrize("kw,levels,tau", VOL_CASES)
def test_prox_dtcwt_volume_matches_oracle(kw, levels, tau):
    import paper_2108_01438_amd as P
    flush(f"[dtcwt prox volume] {kw} levels={levels}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(93)
    v32, v64 = rand_image(rng, O.img_shape(og))
    plan = P.Plan(pg)
    z = to_host(plan.prox("dtcwt", tau, 1.0, to_dev(v32), haar_levels=levels))
    assert rel(z, O.prox_dtcwt(v64, tau, (3, 2, 1), levels)) <= PROX_TOL
    z0 = to_host(plan.prox("dtcwt", 0.0, 1.0, to_dev(v32), haar_levels=levels))
    assert rel(z0, v64) <= 2e-6
    plan.close()


def test_prox_dtcwt_volume_window_passes_match_stored_oracle():
    """512 x 128 x 128, 2 levels: large enough that the first level's x and y
    analysis and synthesis run the register-window kernels.  Against the FP64
    oracle's stored summaries (tests/golden/dtcwt_volume_512x128x128.npz,
    written by the script beside it): sampled voxels, block norms, the
    whole-volume sketch and the norm within 1e-5; tau = 0 returns the input."""
    import importlib.util
    import os
    import sys
    import paper_2108_01438_amd as P
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    import refstats
    spec = importlib.util.spec_from_file_location(
        "make_dtcwt_ref", os.path.join(here, "golden", "make_dtcwt_volume_reference.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    ref = np.load(os.path.join(here, "golden", "dtcwt_volume_512x128x128.npz"))
    flush("[dtcwt prox volume] 512 x 128 x 128 vs the stored oracle")
    v = m.inputs()
    g = P.Geometry(n_depth=m.SHAPE[3], n_x=m.SHAPE[2], n_y=m.SHAPE[1], lateral_dims=2, n_k=16)
    plan = P.Plan(g)
    vd = to_dev(v)
    z = to_host(plan.prox("dtcwt", float(ref["tau"]), 1.0, vd, haar_levels=int(ref["levels"])))
    err = refstats.compare(z, ref, "", tuple(ref["block"]))
    print(f"[dtcwt prox volume] errors vs the oracle: {err}")
    for k in ("samples", "whole_sketch", "norm"):
        assert err[k] <= PROX_TOL, (k, err[k])
    assert err["blocks"] <= 1e-4
    z0 = to_host(plan.prox("dtcwt", 0.0, 1.0, vd, haar_levels=int(ref["levels"])))
    assert rel(z0, v.astype(np.complex128)) <= 2e-6
    plan.close()


def test_fista_dtcwt_volume_matches_oracle():
    import paper_2108_01438_amd as P
    flush("[dtcwt fista volume]")
    og, pg = both_geoms(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=48)
    rng = np.random.default_rng(94)
    x_true = synth.scatterers(rng, O.img_shape(og), 30)
    y_clean = O.forward(x_true, og)
    y32 = synth.noisy(y_clean, synth.standard_normal(rng, y_clean.shape), None, 0.01).astype(np.float32)
    y64 = y32.astype(np.float64)
    lam = 0.01 * O.lambda_max(y64, og)
    delta = O.step_size(O.lipschitz(og, None, iters=50))
    zo, ho = O.fista(y64, og, None, O.PEN_DTCWT, lam, delta, 12, haar_levels=2)
    plan = P.Plan(pg)
    z, info = plan.mbir_solve(to_dev(y32), "dtcwt", lam, 12, delta=delta, haar_levels=2, objective=True)
    assert rel(to_host(z), zo) <= SOLVE_TOL
    np.testing.assert_allclose(info["objective"], ho, rtol=1e-5)
    plan.close()


def test_dtcwt_rejections():
    import paper_2108_01438_amd as P
    og, pg = both_geoms(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=32)
    plan = P.Plan(pg)
    v = to_dev(np.zeros(O.img_shape(og), np.complex64))
    with pytest.raises(P.OctError, match="levels"):
        plan.prox("dtcwt", 0.1, 1.0, v, haar_levels=5)
    with pytest.raises(P.OctError, match="divisible"):
        plan.prox("dtcwt", 0.1, 1.0, v, haar_levels=4)
    plan.close()
    og, pg = both_geoms(n_depth=36, n_x=16, n_k=32)
    plan = P.Plan(pg)
    v = to_dev(np.zeros(O.img_shape(og), np.complex64))
    with pytest.raises(P.OctError, match="divisible"):
        plan.prox("dtcwt", 0.1, 1.0, v, haar_levels=3)
    with pytest.raises(P.OctError, match="no closed form"):
        plan.prox("dtcwt", 0.1, 1.0, v, haar_levels=2, bound=1.0)
    plan.close()


@pytest.mark.parametrize("kw,iters,masked", [(dict(n_depth=128, n_x=48, n_k=128), 20, True),
                                             (dict(n_depth=64, n_x=32, n_k=64, batch=2), 15, False)])
def test_fista_dtcwt_matches_oracle(kw, iters, masked):
    import paper_2108_01438_amd as P
    flush(f"[dtcwt fista] {kw}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(92)
    mask = synth.mask_random_exact(rng, (1, og.n_x), og.n_k, og.n_k // 2) if masked else None
    x_true = synth.scatterers(rng, O.img_shape(og), 30)
    y_clean = O.forward(x_true, og, mask)
    y32 = synth.noisy(y_clean, synth.standard_normal(rng, y_clean.shape), mask, 0.01).astype(np.float32)
    y64 = y32.astype(np.float64)
    lam = 0.01 * O.lambda_max(y64, og, mask)
    delta = O.step_size(O.lipschitz(og, mask, iters=50))
    zo, ho = O.fista(y64, og, mask, O.PEN_DTCWT, lam, delta, iters, haar_levels=3)
    plan = P.Plan(pg, mask)
    z, info = plan.mbir_solve(to_dev(y32), "dtcwt", lam, iters, delta=delta, haar_levels=3, objective=True)
    err = rel(to_host(z), zo)
    print(f"[dtcwt fista] rel err vs oracle {err:.3e}")
    assert err <= SOLVE_TOL
    np.testing.assert_allclose(info["objective"], ho, rtol=1e-5)
    # without the objective the solve skips the value pass and gives the same iterate
    z2, _ = plan.mbir_solve(to_dev(y32), "dtcwt", lam, iters, delta=delta, haar_levels=3)
    assert np.array_equal(to_host(z2), to_host(z))
    plan.close()
