"""Parity of the HIP proximal steps, power iteration and FISTA solve with the
FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rand_image, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

PROX_TOL = 1e-5
SOLVE_TOL = 1e-4


@pytest.mark.parametrize("kw", [dict(n_depth=64, n_x=40, n_k=64, batch=2),
                                dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=32)])
def test_prox_l1(kw):
    import paper_2108_01438_amd as P
    flush(f"[prox l1] {kw}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(1)
    plan = P.Plan(pg)
    v32, v64 = rand_image(rng, O.img_shape(og))
    z = to_host(plan.prox("l1", 0.5, 1.2, to_dev(v32)))
    assert rel(z, O.prox_l1(v64, 0.6)) <= 1e-6


@pytest.mark.parametrize("kw,levels", [
    (dict(n_depth=64, n_x=40, n_k=64, batch=2), 3),
    (dict(n_depth=96, n_x=32, n_k=64), 1),
    (dict(n_depth=64, n_x=32, n_k=64), 5),
    (dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=32, batch=2), 3),
    (dict(n_depth=32, n_x=16, n_y=16, lateral_dims=2, n_k=32), 4),
    (dict(n_depth=8, n_x=4, n_y=4, lateral_dims=2, n_k=32), 2),
])
def test_prox_haar(kw, levels):
    import paper_2108_01438_amd as P
    flush(f"[prox haar] {kw} levels={levels}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(2)
    plan = P.Plan(pg)
    v32, v64 = rand_image(rng, O.img_shape(og))
    axes = (3, 2, 1) if og.lateral_dims == 2 else (3, 2)
    z = to_host(plan.prox("haar", 0.3, 1.0, to_dev(v32), haar_levels=levels))
    assert rel(z, O.prox_haar(v64, 0.3, axes, levels)) <= PROX_TOL


TV_CASES = [
    (dict(n_depth=64, n_x=40, n_k=64, batch=2), 10),          # tiled, 2 depth tiles
    (dict(n_depth=75, n_x=35, n_k=64), 10),
    (dict(n_depth=140, n_x=160, n_k=64), 10),                 # several tiles both ways
    (dict(n_depth=140, n_x=160, n_k=64), 3),                  # small halo
    (dict(n_depth=64, n_x=40, n_k=64), 27),                   # largest tiled inner count
    (dict(n_depth=64, n_x=40, n_k=64), 30),                   # general path (per-step passes)
    (dict(n_depth=1024, n_x=600, n_k=64, batch=2), 10),       # more tiles than CUs: blocks take several
    (dict(n_depth=24, n_x=12, n_y=10, lateral_dims=2, n_k=32), 10),   # volume
    (dict(n_depth=200, n_x=1, n_k=64), 10),                   # one A-scan: TV along depth only
]


@pytest.mark.parametrize("kw,inner", TV_CASES)
def test_prox_tv_cold_and_warm(kw, inner):
    import torch
    import paper_2108_01438_amd as P
    flush(f"[prox tv] {kw} inner={inner}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(3)
    plan = P.Plan(pg)
    v32, v64 = rand_image(rng, O.img_shape(og))
    axes = (3, 2, 1) if og.lateral_dims == 2 else (3, 2)
    tau = 0.4
    z1 = to_host(plan.prox("tv", tau, 1.0, to_dev(v32), tv_inner=inner))
    zr1, p1 = O.prox_tv(v64, tau, axes, inner)
    assert rel(z1, zr1) <= PROX_TOL
    state = torch.zeros((len(axes),) + O.img_shape(og), dtype=torch.complex64, device="cuda")
    plan.prox("tv", tau, 1.0, to_dev(v32), state=state, tv_inner=inner)
    assert rel(to_host(state), p1) <= PROX_TOL
    z2 = to_host(plan.prox("tv", tau, 1.0, to_dev(v32), state=state, tv_inner=7))
    zr2, _ = O.prox_tv(v64, tau, axes, 7, p0=p1)
    assert rel(z2, zr2) <= PROX_TOL


@pytest.mark.parametrize("geom,masked", [
    (dict(n_depth=128, n_x=32, n_k=128, batch=2), True),
    # every pixel observed: the power steps take the residual seam in the lateral-frequency domain
    (dict(n_depth=128, n_x=32, n_k=128, batch=2), False),
    (dict(n_depth=64, n_x=16, n_y=12, lateral_dims=2, n_k=96), False),
])
def test_lipschitz_matches_oracle(geom, masked):
    import paper_2108_01438_amd as P
    flush(f"[lipschitz] 50 power steps {geom} masked={masked}")
    og, pg = both_geoms(**geom)
    rng = np.random.default_rng(4)
    lat = (og.n_y if og.lateral_dims == 2 else 1, og.n_x, og.n_k)
    mask = (rng.random(lat) < 0.5).astype(np.uint8) if masked else None
    plan = P.Plan(pg, mask)
    L = plan.lipschitz(50, seed=11)
    Lo = O.lipschitz(og, mask, iters=50, seed=11)
    assert abs(L - Lo) <= 1e-5 * Lo


def _problem(og, rng, n_scat, mask=None, noise=0.01):
    x_true = synth.scatterers(rng, O.img_shape(og), n_scat)
    y_clean = O.forward(x_true, og, mask)
    y = synth.noisy(y_clean, synth.standard_normal(rng, y_clean.shape), mask, noise)
    return x_true, y


SOLVES = {
    "bscan_512x64_l1_50": (dict(n_depth=512, n_x=64, n_k=512), "l1", 0.01, 50, 20),
    "bscan_128x48_tv_30": (dict(n_depth=128, n_x=48, n_k=128), "tv", 0.005, 30, 40),
    "bscan_128x48_haar_30": (dict(n_depth=128, n_x=48, n_k=128, batch=2), "haar", 0.01, 30, 40),
    "volume_64x16x16_haar_20": (dict(n_depth=64, n_x=16, n_y=16, lateral_dims=2, n_k=64), "haar", 0.01, 20, 60),
    "volume_32x16x8_tv_15": (dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=48), "tv", 0.005, 15, 30),
    "volume_32x16x8_l1_25": (dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=48), "l1", 0.01, 25, 30),
    # one iteration: z = prox(x0 - delta grad D(x0)) and the objective at x0
    "bscan_128x48_tv_1": (dict(n_depth=128, n_x=48, n_k=128), "tv", 0.005, 1, 40),
    # fully observed, odd lateral sizes (no Nyquist column in the residual norm's pair weights)
    "volume_odd_32x9x7_l1_15": (dict(n_depth=32, n_x=9, n_y=7, lateral_dims=2, n_k=48), "l1", 0.01, 15, 12),
    "bscan_odd_75x45_l1_20": (dict(n_depth=75, n_x=45, n_k=90, z_focus=20.0), "l1", 0.01, 20, 15),
}


@pytest.mark.parametrize("name", list(SOLVES))
def test_fista_matches_oracle(name):
    import paper_2108_01438_amd as P
    kw, pen, lam_frac, iters, nsc = SOLVES[name]
    flush(f"[fista] {name}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(5)
    mask = None
    if pen == "tv":
        lat = (og.n_y if og.lateral_dims == 2 else 1, og.n_x)
        mask = synth.mask_random_exact(rng, lat, og.n_k, og.n_k // 2)
    _, y = _problem(og, rng, nsc, mask)
    y32 = y.astype(np.float32)
    y64 = y32.astype(np.float64)
    lam = lam_frac * O.lambda_max(y64, og, mask)
    delta = O.step_size(O.lipschitz(og, mask, iters=50))
    penc = {"l1": O.PEN_L1, "tv": O.PEN_TV, "haar": O.PEN_HAAR}[pen]
    zo, ho = O.fista(y64, og, mask, penc, lam, delta, iters, tv_inner=10, haar_levels=3)
    plan = P.Plan(pg, mask)
    z, info = plan.mbir_solve(to_dev(y32), pen, lam, iters, delta=delta, tv_inner=10, haar_levels=3,
                              objective=True)
    err = rel(to_host(z), zo)
    print(f"[fista] {name}: rel err vs oracle {err:.3e}")
    assert err <= SOLVE_TOL
    np.testing.assert_allclose(info["objective"], ho, rtol=1e-5)


def test_zero_weight_runs_the_same_least_squares_iteration_for_every_penalty():
    """lambda = 0 takes the penalty out of eq. (15): the l1 prox (threshold 0),
    the TV prox (no TV term) and the Haar prox (threshold 0 in an orthonormal
    basis) leave v as it is, so the three solves run FISTA on the data term
    alone: all match the oracle's iteration, and each other to rounding (on a
    B-scan the l1 solve fuses the gradient step, prox and next lateral pass
    into one kernel; TV and Haar run them as separate passes)."""
    import paper_2108_01438_amd as P
    flush("[fista] lambda = 0")
    og, pg = both_geoms(n_depth=128, n_x=48, n_k=128)
    rng = np.random.default_rng(44)
    mask = synth.mask_random_exact(rng, (1, og.n_x), og.n_k, og.n_k // 2)
    _, y = _problem(og, rng, 20, mask)
    y32 = y.astype(np.float32)
    delta = O.step_size(O.lipschitz(og, mask, iters=50))
    zo, _ = O.fista(y32.astype(np.float64), og, mask, O.PEN_L1, 0.0, delta, 20)
    plan = P.Plan(pg, mask)
    zs = {}
    for pen in ("l1", "tv", "haar"):
        z, _ = plan.mbir_solve(to_dev(y32), pen, 0.0, 20, delta=delta, haar_levels=3)
        zs[pen] = to_host(z)
        err = rel(zs[pen], zo)
        print(f"[fista] lambda = 0, {pen}: rel err vs oracle {err:.3e}")
        assert err <= SOLVE_TOL
    assert rel(zs["tv"], zs["l1"]) <= 1e-5
    assert rel(zs["haar"], zs["l1"]) <= 1e-5
    plan.close()


def test_fista_power_iteration_step():
    """delta <= 0: the solver runs the power iteration itself."""
    import paper_2108_01438_amd as P
    flush("[fista] power-iteration step size")
    og, pg = both_geoms(n_depth=128, n_x=32, n_k=128)
    rng = np.random.default_rng(6)
    _, y = _problem(og, rng, 10)
    plan = P.Plan(pg)
    lam = 0.01 * O.lambda_max(y, og)
    z, info = plan.mbir_solve(to_dev(y.astype(np.float32)), "l1", lam, 5, delta=0.0, power_iters=50, seed=3)
    Lo = O.lipschitz(og, None, iters=50, seed=3)
    assert abs(info["lipschitz"] - Lo) <= 1e-5 * Lo
    assert abs(info["delta"] - O.step_size(Lo)) <= 1e-5 * O.step_size(Lo)


def test_fista_warm_start_resume():
    """Start point x0: the solver starts from it (one iteration from x0 equals
    the oracle's)."""
    import paper_2108_01438_amd as P
    flush("[fista] warm start")
    og, pg = both_geoms(n_depth=64, n_x=32, n_k=64)
    rng = np.random.default_rng(8)
    _, y = _problem(og, rng, 8)
    y32 = y.astype(np.float32)
    x032, x064 = rand_image(rng, O.img_shape(og))
    plan = P.Plan(pg)
    lam, delta = 0.1, O.step_size(O.lipschitz(og, None))
    z, _ = plan.mbir_solve(to_dev(y32), "l1", lam, 3, delta=delta, x0=to_dev(x032))
    zo, _ = O.fista(y32.astype(np.float64), og, None, O.PEN_L1, lam, delta, 3, x0=x064)
    assert rel(to_host(z), zo) <= SOLVE_TOL


@pytest.mark.parametrize("pen,kw,masked", [
    ("l1", dict(n_depth=128, n_x=48, n_k=128), False),                 # fused lateral l1 path
    ("tv", dict(n_depth=128, n_x=48, n_k=128), True),                  # tiled TV, dual carried over
    ("haar", dict(n_depth=64, n_x=16, n_y=16, lateral_dims=2, n_k=64), False),
])
def test_fista_exact_resume(pen, kw, masked):
    """Resume from the state (z^k, z^{k-1}, k): 20 iterations, then 20 more
    from x0 = z^20, z_prev0 = z^19, k0 = 20, equal one solve of 40 bitwise."""
    import torch
    import paper_2108_01438_amd as P
    flush(f"[fista] exact resume, {pen}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(14)
    mask = synth.mask_random_exact(rng, (og.n_y if og.lateral_dims == 2 else 1, og.n_x), og.n_k, og.n_k // 2) \
        if masked else None
    _, y = _problem(og, rng, 12, mask)
    plan = P.Plan(pg, mask)
    yd = to_dev(y.astype(np.float32))
    lam = (0.005 if pen == "tv" else 0.01) * O.lambda_max(y, og, mask)
    delta = O.step_size(O.lipschitz(og, mask, iters=20))
    z40, _ = plan.mbir_solve(yd, pen, lam, 40, delta=delta)
    zp = torch.empty_like(z40)
    z20, _ = plan.mbir_solve(yd, pen, lam, 20, delta=delta, z_prev_out=zp)
    z40r, _ = plan.mbir_solve(yd, pen, lam, 20, delta=delta, x0=z20, z_prev0=zp, k0=20)
    assert torch.equal(z40r, z40)
    z19, _ = plan.mbir_solve(yd, pen, lam, 19, delta=delta)
    assert torch.equal(zp, z19)


@pytest.mark.parametrize("pen", ["l1", "tv", "haar"])
def test_nothing_observed_gives_zero_lipschitz_and_zero_solution(pen):
    """An all-zero mask makes Phi = 0: the power iteration gives exactly L = 0
    (as the oracle does), the solve takes the step delta = 1 (every step is
    admissible for a constant data term) and returns exactly zero."""
    import paper_2108_01438_amd as P
    flush(f"[fista] nothing observed, {pen}")
    og, pg = both_geoms(n_depth=64, n_x=16, n_k=64)
    mask = np.zeros((1, og.n_x, og.n_k), dtype=np.uint8)
    plan = P.Plan(pg, mask)
    assert plan.lipschitz(10) == 0.0 == O.lipschitz(og, mask, iters=10)
    y = np.random.default_rng(43).standard_normal(O.meas_shape(og)).astype(np.float32)
    z, info = plan.mbir_solve(to_dev(y), pen, 0.1, 5, haar_levels=2)
    assert info["lipschitz"] == 0.0 and info["delta"] == 1.0 == O.step_size(0.0)
    assert np.all(to_host(z) == 0)
    plan.close()


@pytest.mark.parametrize("pen", ["tv", "l1", "haar"])
def test_solve_replays_bitwise_from_a_graph(pen):
    """A whole solve (batch of two) captured in a graph replays bitwise equal
    to the eager solve, with the caller's own work (zeroing the output) and
    synchronisation between the replays."""
    import torch
    import paper_2108_01438_amd as P
    flush(f"[fista] graph capture, {pen}")
    og, pg = both_geoms(n_depth=128, n_x=48, n_k=128, batch=2)
    rng = np.random.default_rng(12)
    mask = synth.mask_random_exact(rng, (1, og.n_x), og.n_k, og.n_k // 2)
    _, y = _problem(og, rng, 20, mask)
    plan = P.Plan(pg, mask)
    yd = to_dev(y.astype(np.float32))
    lam, delta = 0.005 * O.lambda_max(y, og, mask), O.step_size(O.lipschitz(og, mask, iters=20))
    z = torch.empty(O.img_shape(og), dtype=torch.complex64, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.mbir_solve(yd, pen, lam, 8, delta=delta, tv_inner=10, x_out=z)   # allocates the solver state
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    plan.mbir_solve(yd, pen, lam, 8, delta=delta, tv_inner=10, x_out=z)
    torch.cuda.synchronize()
    ref = to_host(z).copy()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.mbir_solve(yd, pen, lam, 8, delta=delta, tv_inner=10, x_out=z)
    for _ in range(3):
        z.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(to_host(z), ref)
    plan.close()
