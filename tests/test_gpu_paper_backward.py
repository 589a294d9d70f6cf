"""The paper's backward operator of eq. (10)-(11) (conjugate analytic signal
along k, then the adjoint's NUFFT and lateral parts) and FISTA driven by it,
through the C ABI against the FP64 oracle on the same float32 inputs."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-5
SOLVE_TOL = 1e-4

GEOMS = [
    dict(n_depth=128, n_x=40, n_k=160, disp_b=1e-6),        # even n_k, radix 5
    dict(n_depth=96, n_x=24, n_k=105, batch=2),              # odd n_k (3 5 7): no Nyquist bin
    dict(n_depth=64, n_x=12, n_y=10, lateral_dims=2, n_k=64),
    dict(n_depth=512, n_x=64, n_k=1024),                     # compile-time spectral transform
]


@pytest.mark.parametrize("gk", range(len(GEOMS)))
def test_adjoint_paper_matches_oracle(gk):
    import paper_2108_01438_amd as P
    kw = GEOMS[gk]
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(70 + gk)
    lat = (og.n_y, og.n_x)
    r32 = rng.standard_normal(O.meas_shape(og)).astype(np.float32)
    r64 = r32.astype(np.float64)
    masks = {"none": None, "random": synth.mask_bernoulli(rng, lat, og.n_k, 0.5),
             "partial": synth.mask_partial(lat, og.n_k)}
    for mname, mask in masks.items():
        flush(f"[paper backward] geom {gk} mask {mname}")
        plan = P.Plan(pg, mask)
        x = to_host(plan.adjoint_paper(to_dev(r32)))
        err = rel(x, O.paper_backward(r64, og, mask))
        print(f"[paper backward] geom {gk} mask {mname}: rel err {err:.3e}")
        assert err <= TOL, (mname, err)
        plan.close()


def test_adjoint_paper_full_size_bscan():
    """2048 spectral px x 1000 A-scans with the random 50% mask, every pixel."""
    import paper_2108_01438_amd as P
    pr = synth.preset("bscan_2048x1000_tv")
    og, pg = both_geoms(**pr["geom"])
    rng = np.random.default_rng(77)
    mask = synth.mask_random_exact(rng, (1, og.n_x), og.n_k, og.n_k // 2)
    r32 = rng.standard_normal(O.meas_shape(og)).astype(np.float32)
    flush("[paper backward] full-size B-scan")
    plan = P.Plan(pg, mask)
    x = to_host(plan.adjoint_paper(to_dev(r32)))
    err = rel(x, O.paper_backward(r32.astype(np.float64), og, mask))
    print(f"[paper backward] full size: rel err {err:.3e}")
    assert err <= TOL
    plan.close()


def test_adjoint_paper_differs_from_the_exact_adjoint_by_the_hilbert_term():
    """For real r, Phi^H r is the complex adjoint applied to s r, so
    Phi* r - Phi^H r is that adjoint applied to -j H(s r): the Hilbert term
    alone, compared with the oracle's difference."""
    import paper_2108_01438_amd as P
    og, pg = both_geoms(n_depth=64, n_x=16, n_k=128)
    rng = np.random.default_rng(78)
    r32 = rng.standard_normal(O.meas_shape(og)).astype(np.float32)
    r64 = r32.astype(np.float64)
    plan = P.Plan(pg)
    rd = to_dev(r32)
    d_gpu = to_host(plan.adjoint_paper(rd)).astype(np.complex128) - to_host(plan.adjoint(rd))
    d_ref = O.paper_backward(r64, og) - O.adjoint(r64, og)
    assert rel(d_gpu, d_ref) <= 1e-4
    plan.close()


def _problem(og, rng, n_scat, mask=None, noise=0.01):
    x_true = synth.scatterers(rng, O.img_shape(og), n_scat)
    y_clean = O.forward(x_true, og, mask)
    return synth.noisy(y_clean, synth.standard_normal(rng, y_clean.shape), mask, noise)


SOLVES = {
    "bscan_256x48_l1_30": (dict(n_depth=256, n_x=48, n_k=256), "l1", 0.01, 30, 20, False),
    "bscan_128x48_tv_20": (dict(n_depth=128, n_x=48, n_k=128), "tv", 0.005, 20, 30, True),
    "volume_32x16x8_haar_15": (dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=48), "haar", 0.01, 15, 30,
                               False),
}


@pytest.mark.parametrize("name", list(SOLVES))
def test_fista_paper_backward_matches_oracle(name):
    import paper_2108_01438_amd as P
    kw, pen, lam_frac, iters, nsc, masked = SOLVES[name]
    flush(f"[fista paper backward] {name}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(9)
    mask = None
    if masked:
        lat = (og.n_y if og.lateral_dims == 2 else 1, og.n_x)
        mask = synth.mask_random_exact(rng, lat, og.n_k, og.n_k // 2)
    y32 = _problem(og, rng, nsc, mask).astype(np.float32)
    y64 = y32.astype(np.float64)
    lam = lam_frac * O.lambda_max(y64, og, mask)
    delta = O.step_size(O.lipschitz(og, mask, iters=50, backward="paper"))
    penc = {"l1": O.PEN_L1, "tv": O.PEN_TV, "haar": O.PEN_HAAR}[pen]
    zo, ho = O.fista(y64, og, mask, penc, lam, delta, iters, tv_inner=10, haar_levels=3, backward="paper")
    plan = P.Plan(pg, mask)
    z, info = plan.mbir_solve(to_dev(y32), pen, lam, iters, delta=delta, tv_inner=10, haar_levels=3,
                              objective=True, paper_backward=True)
    err = rel(to_host(z), zo)
    print(f"[fista paper backward] {name}: rel err vs oracle {err:.3e}")
    assert err <= SOLVE_TOL
    np.testing.assert_allclose(info["objective"], ho, rtol=1e-5)
    plan.close()


def test_power_iteration_on_the_paper_normal_operator():
    """L of Phi* Phi on a masked B-scan and on a volume against the oracle, and
    the solver's own step (delta <= 0) with the paper backward."""
    import paper_2108_01438_amd as P
    for kw, masked in ((dict(n_depth=128, n_x=48, n_k=128), True),
                       (dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=48), False)):
        flush(f"[paper power iteration] {kw}")
        og, pg = both_geoms(**kw)
        rng = np.random.default_rng(12)
        mask = None
        if masked:
            mask = synth.mask_random_exact(rng, (1, og.n_x), og.n_k, og.n_k // 2)
        plan = P.Plan(pg, mask)
        L = plan.lipschitz(50, seed=4, paper_backward=True)
        Lo = O.lipschitz(og, mask, iters=50, seed=4, backward="paper")
        assert abs(L - Lo) <= 1e-5 * Lo, (L, Lo)
        y = to_dev(rng.standard_normal(O.meas_shape(og)).astype(np.float32))
        _, info = plan.mbir_solve(y, "l1", 0.01, 2, delta=0.0, power_iters=50, seed=4, paper_backward=True)
        assert abs(info["lipschitz"] - Lo) <= 1e-5 * Lo
        plan.close()


def test_paper_backward_rejects_a_spectral_length_with_a_large_prime():
    import paper_2108_01438_amd as P
    og, pg = both_geoms(n_depth=32, n_x=8, n_k=44)   # 44 = 4 x 11
    plan = P.Plan(pg)
    r = to_dev(np.zeros(O.meas_shape(og), np.float32))
    with pytest.raises(P.OctError, match="7-smooth"):
        plan.adjoint_paper(r)
    with pytest.raises(P.OctError, match="7-smooth"):
        plan.mbir_solve(r, "l1", 0.1, 2, delta=1.0, paper_backward=True)
    plan.close()


def test_fista_paper_backward_full_size_first_iterations():
    """2048 x 1000 B-scan with the random 50% mask: 4 TV iterations driven by the
    paper's backward operator against the oracle's, same step."""
    import paper_2108_01438_amd as P
    pr = synth.preset("bscan_2048x1000_tv")
    og, pg = both_geoms(**pr["geom"])
    rng = np.random.default_rng(79)
    mask = synth.mask_random_exact(rng, (1, og.n_x), og.n_k, og.n_k // 2)
    x_true = synth.scatterers(rng, O.img_shape(og), 200)
    flush("[fista paper backward] full size: oracle measurement")
    y_clean = O.forward(x_true, og, mask)
    y32 = synth.noisy(y_clean, synth.standard_normal(rng, y_clean.shape), mask, 0.01).astype(np.float32)
    y64 = y32.astype(np.float64)
    lam = 0.005 * O.lambda_max(y64, og, mask)
    delta = 1e-4
    flush("[fista paper backward] full size: 4 oracle iterations")
    zo, ho = O.fista(y64, og, mask, O.PEN_TV, lam, delta, 4, tv_inner=10, backward="paper")
    plan = P.Plan(pg, mask)
    z, info = plan.mbir_solve(to_dev(y32), "tv", lam, 4, delta=delta, tv_inner=10, objective=True,
                              paper_backward=True)
    err = rel(to_host(z), zo)
    print(f"[fista paper backward] full size: rel err {err:.3e}")
    assert err <= SOLVE_TOL
    np.testing.assert_allclose(info["objective"], ho, rtol=1e-5)
    plan.close()
