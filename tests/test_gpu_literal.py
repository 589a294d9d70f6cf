"""The paper's literal K, Q, D chain (operator model 1, n_k = 2 n_depth)
through the C ABI against the FP64 oracle on the same float32 inputs: forward,
adjoint, gradient, the paper's backward operator, FISTA and the power
iteration."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rand_image, rand_meas, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-5
SOLVE_TOL = 1e-4

GEOMS = [
    dict(n_depth=64, n_x=40, n_k=128, disp_b=1e-6, model=1),
    dict(n_depth=96, n_x=24, n_k=192, batch=2, model=1),           # radix 3 in both transforms
    dict(n_depth=32, n_x=12, n_y=10, lateral_dims=2, n_k=64, model=1),
    dict(n_depth=1024, n_x=64, n_k=2048, model=1),                 # compile-time transforms
    dict(n_depth=2016, n_x=8, n_k=4032, model=1),                  # radix 7, two butterflies per thread
]


@pytest.mark.parametrize("gk", range(len(GEOMS)))
def test_literal_operators_match_oracle(gk):
    import paper_2108_01438_amd as P
    kw = GEOMS[gk]
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(80 + gk)
    lat = (og.n_y, og.n_x)
    mask = synth.mask_bernoulli(rng, lat, og.n_k, 0.5)
    x32, x64 = rand_image(rng, O.img_shape(og))
    r32, r64 = rand_meas(rng, O.meas_shape(og))
    flush(f"[literal] geom {gk}")
    plan = P.Plan(pg, mask)
    y = to_host(plan.forward(to_dev(x32)))
    assert rel(y, O.forward(x64, og, mask)) <= TOL
    xa = to_host(plan.adjoint(to_dev(r32)))
    assert rel(xa, O.adjoint(r64, og, mask)) <= TOL
    xp = to_host(plan.adjoint_paper(to_dev(r32)))
    assert rel(xp, O.paper_backward(r64, og, mask)) <= TOL
    g, _ = plan.grad(to_dev(x32), to_dev(r32))
    go, _ = O.grad(x64, r64, og, mask)
    assert rel(to_host(g), go) <= TOL
    plan.close()


def test_literal_even_pixels_equal_the_direct_model_on_the_gpu():
    """The even detector pixels of the literal chain are the direct model's
    (same NUFFT samples); the odd ones differ when q != 0."""
    import paper_2108_01438_amd as P
    og, pg = both_geoms(n_depth=128, n_x=48, n_k=256, model=1)
    rng = np.random.default_rng(88)
    x32, _ = rand_image(rng, O.img_shape(og))
    lit = P.Plan(pg)
    pd = P.Geometry(**{**pg.__dict__, "model": 0})
    direct = P.Plan(pd)
    yl = to_host(lit.forward(to_dev(x32)))
    yd = to_host(direct.forward(to_dev(x32)))
    assert rel(yl[..., ::2], yd[..., ::2]) <= 1e-6
    assert rel(yl[..., 1::2], yd[..., 1::2]) > 1e-3
    lit.close()
    direct.close()


def test_literal_model_validation():
    import paper_2108_01438_amd as P
    with pytest.raises(P.OctError, match="n_k = 2 n_depth"):
        P.Plan(P.Geometry(n_depth=32, n_x=8, n_k=48, model=1))
    with pytest.raises(P.OctError, match="model"):
        P.Plan(P.Geometry(n_depth=32, n_x=8, n_k=64, model=2))


def _problem(og, rng, n_scat, mask=None, noise=0.01):
    x_true = synth.scatterers(rng, O.img_shape(og), n_scat)
    y_clean = O.forward(x_true, og, mask)
    return synth.noisy(y_clean, synth.standard_normal(rng, y_clean.shape), mask, noise)


SOLVES = {
    "bscan_128x48_l1_30": (dict(n_depth=128, n_x=48, n_k=256, model=1), "l1", 0.01, 30, 20, False),
    "bscan_128x48_tv_20": (dict(n_depth=128, n_x=48, n_k=256, model=1), "tv", 0.005, 20, 30, True),
    "volume_32x16x8_haar_15": (dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=64, model=1), "haar", 0.01,
                               15, 30, False),
}


@pytest.mark.parametrize("name", list(SOLVES))
def test_literal_fista_matches_oracle(name):
    import paper_2108_01438_amd as P
    kw, pen, lam_frac, iters, nsc, masked = SOLVES[name]
    flush(f"[literal fista] {name}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(89)
    mask = None
    if masked:
        lat = (og.n_y if og.lateral_dims == 2 else 1, og.n_x)
        mask = synth.mask_random_exact(rng, lat, og.n_k, og.n_k // 2)
    y32 = _problem(og, rng, nsc, mask).astype(np.float32)
    y64 = y32.astype(np.float64)
    lam = lam_frac * O.lambda_max(y64, og, mask)
    Lo = O.lipschitz(og, mask, iters=50, seed=2)
    delta = O.step_size(Lo)
    penc = {"l1": O.PEN_L1, "tv": O.PEN_TV, "haar": O.PEN_HAAR}[pen]
    zo, ho = O.fista(y64, og, mask, penc, lam, delta, iters, tv_inner=10, haar_levels=3)
    plan = P.Plan(pg, mask)
    L = plan.lipschitz(50, seed=2)
    assert abs(L - Lo) <= 1e-5 * Lo
    z, info = plan.mbir_solve(to_dev(y32), pen, lam, iters, delta=delta, tv_inner=10, haar_levels=3,
                              objective=True)
    err = rel(to_host(z), zo)
    print(f"[literal fista] {name}: rel err vs oracle {err:.3e}")
    assert err <= SOLVE_TOL
    np.testing.assert_allclose(info["objective"], ho, rtol=1e-5)
    plan.close()
