"""Geometries drawn once from a fixed seed: 7-smooth sizes, oversampling,
KB width, batch, focus, B-scans and small volumes, random masks.  Forward,
adjoint and the TV prox (tiled and per-step paths) through the C ABI against
the FP64 oracle on the same float32 inputs.  Every run checks the same list."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rand_image, rand_meas, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5
PROX_TOL = 1e-5


def _draw(seed: int, count: int):
    """Random geometries the library accepts (its plan-size check, which
    needs no GPU, is the filter)."""
    import paper_2108_01438_amd as P
    rng = np.random.default_rng(seed)
    depths = [n for n in range(8, 161, 2) if synth.is_smooth7(n)]
    laterals = [n for n in range(1, 151) if synth.is_smooth7(n)]
    spectra = [n for n in range(8, 301) if synth.is_smooth7(n)]
    out = []
    while len(out) < count:
        vol = rng.random() < 0.3
        kw = dict(n_depth=int(rng.choice(depths)), n_k=int(rng.choice(spectra)),
                  n_x=int(rng.choice(laterals[:40] if vol else laterals)),
                  oversamp=float(rng.choice([1.5, 2.0, 2.5])), kb_width=int(rng.choice([4, 6, 8])),
                  batch=int(rng.integers(1, 4)), disp_b=float(rng.choice([0.0, 1e-6])))
        if vol:
            kw.update(lateral_dims=2, n_y=int(rng.choice(laterals[:30])))
        if rng.random() < 0.3:
            kw["z_focus"] = float(rng.uniform(0.2, 0.8)) * kw["n_depth"] * 0.5
        if P.footprint_bytes(P.Geometry(**kw)) == 0:
            continue
        out.append(kw)
    return out


CASES = _draw(20261203, 40)


@pytest.mark.parametrize("i", range(len(CASES)))
def test_random_geometry_matches_oracle(i):
    import paper_2108_01438_amd as P
    kw = CASES[i]
    flush(f"[random shape {i}] {kw}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(1000 + i)
    lat = (og.n_y if og.lateral_dims == 2 else 1, og.n_x)
    mask = synth.mask_bernoulli(rng, lat, og.n_k, 0.6) if i % 2 else None
    plan = P.Plan(pg, mask)
    x32, x64 = rand_image(rng, O.img_shape(og))
    r32, r64 = rand_meas(rng, O.meas_shape(og))
    assert rel(to_host(plan.forward(to_dev(x32))), O.forward(x64, og, mask)) <= OP_TOL
    assert rel(to_host(plan.adjoint(to_dev(r32))), O.adjoint(r64, og, mask)) <= OP_TOL
    axes = (3, 2, 1) if og.lateral_dims == 2 else (3, 2)
    for inner in (10, 30):   # B-scans: tiled path, then the per-step path
        z = to_host(plan.prox("tv", 0.3, 1.0, to_dev(x32), tv_inner=inner))
        zo, _ = O.prox_tv(x64, 0.3, axes, inner)
        assert rel(z, zo) <= PROX_TOL
    plan.close()


SOLVE_TOL = 1e-4


@pytest.mark.parametrize("i", range(0, len(CASES), 8))
@pytest.mark.parametrize("pen", ["l1", "tv"])
def test_random_geometry_fista_matches_oracle(i, pen):
    """Five FISTA iterations (power-iteration step from the oracle) on every
    eighth geometry of the list, with the objective history."""
    import paper_2108_01438_amd as P
    kw = CASES[i]
    flush(f"[random shape fista {i} {pen}] {kw}")
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(2000 + i)
    x_true = synth.scatterers(rng, O.img_shape(og), 10)
    y32 = O.forward(x_true, og).astype(np.float32)
    y64 = y32.astype(np.float64)
    lam = (0.01 if pen == "l1" else 0.005) * O.lambda_max(y64, og)
    delta = O.step_size(O.lipschitz(og, None, iters=30))
    penc = {"l1": O.PEN_L1, "tv": O.PEN_TV}[pen]
    zo, ho = O.fista(y64, og, None, penc, lam, delta, 5, tv_inner=10)
    plan = P.Plan(pg)
    z, info = plan.mbir_solve(to_dev(y32), pen, lam, 5, delta=delta, tv_inner=10, objective=True)
    assert rel(to_host(z), zo) <= SOLVE_TOL
    np.testing.assert_allclose(info["objective"], ho, rtol=1e-5)
    plan.close()
