"""Direct reconstructions (Sec. 3.1: axial "IFFT", dispersion corrected, ISAM,
interpolated ISAM) and the NCC of eq. (17) through the C ABI, against the FP64
oracle on the same float32 inputs."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rand_image, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-5
KINDS = ("axial", "dispersion", "isam", "interp_isam")


def _oracle(kind, y, og, mask):
    if kind == "axial":
        return O.direct_axial(y, og, mask, dispersion=False)
    if kind == "dispersion":
        return O.direct_axial(y, og, mask, dispersion=True)
    if kind == "isam":
        return O.direct_isam(y, og, mask)
    return O.interp_isam(y, og, mask if mask is not None else np.ones((og.n_y, og.n_x, og.n_k), np.uint8))


def _masks(rng, lat, nk):
    return {
        "none": None,
        "random": synth.mask_bernoulli(rng, lat, nk, 0.5),
        "equispaced": synth.mask_equispaced(lat, nk),
        "partial": synth.mask_partial(lat, nk),
    }


GEOMS = [
    dict(n_depth=128, n_x=40, n_k=160, disp_b=1e-6),
    dict(n_depth=96, n_x=24, n_k=96, batch=2),
    dict(n_depth=64, n_x=12, n_y=10, lateral_dims=2, n_k=64),
]


@pytest.mark.parametrize("gk", range(len(GEOMS)))
def test_direct_reconstructions_match_oracle(gk):
    import paper_2108_01438_amd as P
    kw = GEOMS[gk]
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(30 + gk)
    lat = (og.n_y, og.n_x)
    y32 = rng.standard_normal(O.meas_shape(og)).astype(np.float32)
    y64 = y32.astype(np.float64)
    for mname, mask in _masks(rng, lat, og.n_k).items():
        if mask is not None:
            mask = mask.copy()
            mask.reshape(-1, og.n_k)[3] = 0            # one A-scan with nothing observed
        plan = P.Plan(pg, mask)
        yd = to_dev(y32)
        for kind in KINDS:
            flush(f"[direct] geom {gk} mask {mname} {kind}")
            x = to_host(plan.direct(yd, kind))
            err = rel(x, _oracle(kind, y64, og, mask))
            assert err <= TOL, (kind, mname, err)
        plan.close()


def test_direct_isam_equals_adjoint_bitwise():
    import paper_2108_01438_amd as P
    og, pg = both_geoms(n_depth=64, n_x=16, n_k=80)
    rng = np.random.default_rng(40)
    mask = synth.mask_bernoulli(rng, (1, 16), 80, 0.5)
    plan = P.Plan(pg, mask)
    y = to_dev(rng.standard_normal(O.meas_shape(og)).astype(np.float32))
    assert np.array_equal(to_host(plan.direct(y, "isam")), to_host(plan.adjoint(y)))


def test_full_size_bscan_axial_on_sampled_a_scans():
    """2048 spectral px x 1000 A-scans, random 50% mask: the per-A-scan
    transforms against the oracle on 12 A-scans it computes one by one."""
    import paper_2108_01438_amd as P
    pr = synth.preset("bscan_2048x1000_tv")
    og, pg = both_geoms(**pr["geom"])
    rng = np.random.default_rng(41)
    mask = synth.mask_random_exact(rng, (1, og.n_x), og.n_k, og.n_k // 2)
    y32 = rng.standard_normal(O.meas_shape(og)).astype(np.float32)
    plan = P.Plan(pg, mask)
    yd = to_dev(y32)
    og1 = og.with_(n_x=1)
    for kind in ("axial", "dispersion"):
        flush(f"[direct] full-size B-scan {kind}")
        x = to_host(plan.direct(yd, kind))
        for l in rng.choice(og.n_x, size=12, replace=False):
            ref = O.direct_axial(y32[:, :, l:l + 1].astype(np.float64), og1, mask[:, l:l + 1],
                                 dispersion=(kind == "dispersion"))
            assert rel(x[:, :, l:l + 1], ref) <= TOL


def test_ncc_matches_oracle():
    import paper_2108_01438_amd as P
    og, pg = both_geoms(n_depth=128, n_x=40, n_k=128, batch=2)
    plan = P.Plan(pg)
    rng = np.random.default_rng(42)
    z32, z64 = rand_image(rng, O.img_shape(og))
    n32, _ = rand_image(rng, O.img_shape(og))
    for a in (0.0, 0.3, 1.0, 3.0):
        flush(f"[ncc] noise {a}")
        x32 = (z32 + np.float32(a) * n32).astype(np.complex64)
        r = plan.ncc(to_dev(x32), to_dev(z32))
        ro = O.ncc(x32.astype(np.complex128), z64)
        assert abs(r - ro) <= 1e-10, (a, r, ro)
    assert abs(plan.ncc(to_dev(z32), to_dev(z32)) - 1.0) <= 1e-12
    with pytest.raises(P.OctError):
        plan.ncc(to_dev(np.ones(O.img_shape(og), np.complex64)), to_dev(z32))


def test_lambda_search_on_device():
    """Golden-section search of lambda on NCC (Sec. 3.2) through oct_mbir_solve
    and oct_ncc: the returned lambda is the best evaluated one, inside the
    range, and its NCC is reproduced by a fresh solve."""
    import torch
    import paper_2108_01438_amd as P
    from paper_2108_01438_amd.tune import tune_lambda
    og, pg = both_geoms(n_depth=128, n_x=48, n_k=128)
    rng = np.random.default_rng(43)
    x_true = synth.scatterers(rng, O.img_shape(og), 15)
    full = P.Plan(pg)
    y = full.forward(to_dev(x_true.astype(np.complex64)))
    ref = full.direct(y, "isam")
    mask = synth.mask_equispaced((1, og.n_x), og.n_k)
    plan = P.Plan(pg, mask)
    ym = y * to_dev(mask.astype(np.float32)[None])
    lam_max = float(plan.adjoint(ym).abs().max())
    delta = 1.0 / (1.05 * plan.lipschitz(30))
    flush("[tune] golden-section search, 6 reductions")
    r = tune_lambda(plan, ym, ref, "l1", lam_max, delta, iters=30, u_range=(-4.0, -0.5), search_iters=6)
    assert len(r["evaluations"]) == 8
    assert -4.0 <= r["u"] <= -0.5
    assert r["ncc"] == max(v for _, v in r["evaluations"])
    z, _ = plan.mbir_solve(ym, "l1", r["lam"], 30, delta=delta)
    assert abs(plan.ncc(z, ref) - r["ncc"]) <= 1e-12
    # a coarse scan run one candidate at a time and as one batched solve
    import dataclasses
    flush("[tune] coarse scan: sequential vs batched")
    rs = tune_lambda(plan, ym, ref, "l1", lam_max, delta, iters=30, u_range=(-4.0, -0.5), search_iters=2,
                     coarse=8)
    rb = tune_lambda(plan, ym, ref, "l1", lam_max, delta, iters=30, u_range=(-4.0, -0.5), search_iters=2,
                     coarse=8, batched_plan=P.Plan(dataclasses.replace(pg, batch=8), mask))
    for (ua, va), (ub, vb) in zip(rs["evaluations"][:8], rb["evaluations"][:8]):
        assert ua == ub and abs(va - vb) <= 1e-5
    assert rs["u"] == rb["u"]
    torch.cuda.synchronize()
