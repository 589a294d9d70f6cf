"""Parity of the HIP operator, adjoint and gradient with the FP64 oracle
(relative L2 <= 1e-5), the FP32 adjoint identity, determinism and edge cases."""
import zlib

import numpy as np
import pytest

import oracle as O
from gpu_util import both_geoms, flush, rand_image, rand_meas, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

OP_TOL = 1e-5

CASES = {
    # several lateral tiles, ragged last tile (n_x = 60 rows of depth 200)
    "bscan_200x60_k300_b2": dict(n_depth=200, n_x=60, n_k=300, batch=2, disp_b=1e-6),
    "bscan_512x64": dict(n_depth=512, n_x=64, n_k=512),
    "bscan_odd_75x45_k90_focus": dict(n_depth=75, n_x=45, n_k=90, z_focus=20.0),
    "bscan_j4_128x30": dict(n_depth=128, n_x=30, n_k=128, kb_width=4),
    "bscan_j8_128x42_k256": dict(n_depth=128, n_x=42, n_k=256, kb_width=8),
    "bscan_sigma25_96x24": dict(n_depth=96, n_x=24, n_k=100, oversamp=2.5),
    # sample spacing below one grid cell: the adjoint gathers cell by cell
    "bscan_sigma15_128x32": dict(n_depth=128, n_x=32, n_k=128, oversamp=1.5),
    # more samples than grid cells in a column: several phases of the gather
    "bscan_k3n_64x24": dict(n_depth=64, n_x=24, n_k=192),
    "ascan_single_256": dict(n_depth=256, n_x=1, n_k=256),
    "evanescent_64x32": dict(n_depth=64, n_x=32, n_k=64, k_min=0.3, k_max=0.9, dx=0.5),
    "volume_64x16x12_b2": dict(n_depth=64, n_x=16, n_y=12, lateral_dims=2, n_k=96, batch=2),
    "volume_128x8x8": dict(n_depth=128, n_x=8, n_y=8, lateral_dims=2, n_k=128),
    "wide_2000x64": dict(n_depth=64, n_x=2000, n_k=64),
    # K = 4032 = 2^6 3^2 7 and N_x = 3528 = 2^3 3^2 7^2: radix-7 transforms with
    # more radix-3 butterflies per stage than threads (two per thread)
    "radix7_k4032_2016x8": dict(n_depth=2016, n_x=8, n_k=2016),
    "radix7_nx3528_16x3528": dict(n_depth=16, n_x=3528, n_k=16),
    # 4096 columns: the adjoint runs narrower workgroups
    "many_columns_64x1024_b4": dict(n_depth=64, n_x=1024, n_k=64, batch=4),
    # largest grid coordinates the 16-bit base cells take (t up to ~3.07e4 of the 3.2e4 limit,
    # wrapping the 128-cell grid ~240 times): an explicit depth pitch of 90 um
    "max_t_dz90_64x8": dict(n_depth=64, n_x=8, n_k=64, dz=90.0),
    # a volume one A-scan wide in y (a length-1 transform along y)
    "volume_ny1_64x16x1": dict(n_depth=64, n_x=16, n_y=1, lateral_dims=2, n_k=64),
    # odd n_x and n_y: no Nyquist column; only q_x = 0 pairs within the half spectrum
    "volume_odd_32x9x7": dict(n_depth=32, n_x=9, n_y=7, lateral_dims=2, n_k=48),
}


def _mask(rng, og, kind):
    shp = (og.n_y if og.lateral_dims == 2 else 1, og.n_x, og.n_k)
    if kind == "ones":
        return None
    return (rng.random(shp) < 0.55).astype(np.uint8)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("mask_kind", ["ones", "random"])
def test_forward_adjoint_grad_match_oracle(name, mask_kind):
    import paper_2108_01438_amd as P
    flush(f"[operator] {name} mask={mask_kind}")
    og, pg = both_geoms(**CASES[name])
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    mask = _mask(rng, og, mask_kind)
    plan = P.Plan(pg, mask)
    x32, x64 = rand_image(rng, O.img_shape(og))
    r32, r64 = rand_meas(rng, O.meas_shape(og))
    y_or = O.forward(x64, og, mask)
    y = to_host(plan.forward(to_dev(x32)))
    assert rel(y, y_or) <= OP_TOL
    a_or = O.adjoint(r64, og, mask)
    a = to_host(plan.adjoint(to_dev(r32)))
    assert rel(a, a_or) <= OP_TOL
    g_or, res = O.grad(x64, r64, og, mask)
    g, hr = plan.grad(to_dev(x32), to_dev(r32))
    assert rel(to_host(g), g_or) <= OP_TOL
    assert abs(float(hr.item()) - 0.5 * float(np.sum(res * res))) <= 1e-5 * 0.5 * float(np.sum(res * res))


@pytest.mark.parametrize("name", ["bscan_200x60_k300_b2", "volume_64x16x12_b2", "bscan_odd_75x45_k90_focus",
                                  "evanescent_64x32", "volume_odd_32x9x7", "volume_ny1_64x16x1"])
def test_full_mask_seam(name):
    """With every pixel observed (eq. (7), s = 1) a volume's gradient takes
    the residual seam in the lateral-frequency domain (a B-scan's keeps its
    one-pass seam); a mask array of all ones must give bitwise the plan
    without a mask, and one unobserved pixel the general seam, both within
    the operator tolerance of the oracle (value and 1/2 ||r||^2)."""
    import paper_2108_01438_amd as P
    flush(f"[full-mask seam] {name}")
    og, pg = both_geoms(**CASES[name])
    rng = np.random.default_rng(zlib.crc32(name.encode()) + 1)
    x32, x64 = rand_image(rng, O.img_shape(og))
    r32, r64 = rand_meas(rng, O.meas_shape(og))
    shp = (og.n_y if og.lateral_dims == 2 else 1, og.n_x, og.n_k)
    ones = np.ones(shp, dtype=np.uint8)
    one_off = ones.copy()
    one_off[0, og.n_x // 2, og.n_k // 3] = 0
    out = {}
    for kind, mask in (("none", None), ("ones", ones), ("one_off", one_off)):
        plan = P.Plan(pg, mask)
        g, hr = plan.grad(to_dev(x32), to_dev(r32))
        out[kind] = (to_host(g), float(hr.item()))
        plan.close()
        g_or, res = O.grad(x64, r64, og, None if mask is None else mask)
        assert rel(out[kind][0], g_or) <= OP_TOL, kind
        hr_or = 0.5 * float(np.sum(res * res))
        assert abs(out[kind][1] - hr_or) <= 1e-5 * hr_or, kind
    assert np.array_equal(out["none"][0], out["ones"][0]) and out["none"][1] == out["ones"][1]


@pytest.mark.parametrize("name", ["bscan_512x64", "volume_64x16x12_b2", "bscan_200x60_k300_b2"])
def test_adjoint_identity_fp32(name):
    """<Phi x, r> = Re<x, Phi^H r> with FP64 inner products of FP32 results."""
    import paper_2108_01438_amd as P
    flush(f"[adjoint identity] {name}")
    og, pg = both_geoms(**CASES[name])
    rng = np.random.default_rng(7)
    plan = P.Plan(pg)
    x32, _ = rand_image(rng, O.img_shape(og))
    r32, _ = rand_meas(rng, O.meas_shape(og))
    y = to_host(plan.forward(to_dev(x32))).astype(np.float64)
    a = to_host(plan.adjoint(to_dev(r32))).astype(np.complex128)
    lhs = float(np.sum(y * r32.astype(np.float64)))
    rhs = float(np.real(np.vdot(x32.astype(np.complex128), a)))
    scale = np.linalg.norm(y) * np.linalg.norm(r32)
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_determinism_bitwise():
    import paper_2108_01438_amd as P
    flush("[determinism] adjoint and grad repeat bitwise")
    og, pg = both_geoms(**CASES["bscan_200x60_k300_b2"])
    rng = np.random.default_rng(9)
    plan = P.Plan(pg, _mask(rng, og, "random"))
    x32, _ = rand_image(rng, O.img_shape(og))
    r32, _ = rand_meas(rng, O.meas_shape(og))
    xd, rd = to_dev(x32), to_dev(r32)
    a1 = to_host(plan.adjoint(rd))
    a2 = to_host(plan.adjoint(rd))
    g1, h1 = plan.grad(xd, rd)
    g1 = to_host(g1)
    h1 = float(h1.item())
    g2, h2 = plan.grad(xd, rd)
    assert np.array_equal(a1.view(np.uint32), a2.view(np.uint32))
    assert np.array_equal(g1.view(np.uint32), to_host(g2).view(np.uint32))
    assert h1 == float(h2.item())


def test_full_size_bscan_2048x1000():
    """The full-size B-scan workload (2048 spectral pixels x 1000 A-scans, 50%
    random mask): forward, adjoint and gradient against the oracle."""
    import paper_2108_01438_amd as P
    import synth
    flush("[full size] bscan 2048x1000")
    pr = synth.preset("bscan_2048x1000_tv")
    og, pg = both_geoms(**pr["geom"])
    rng = np.random.default_rng(1)
    mask = synth.mask_random_exact(rng, (1, og.n_x), og.n_k, og.n_k // 2)
    plan = P.Plan(pg, mask)
    x32, x64 = rand_image(rng, O.img_shape(og))
    r32, r64 = rand_meas(rng, O.meas_shape(og))
    assert rel(to_host(plan.forward(to_dev(x32))), O.forward(x64, og, mask)) <= OP_TOL
    assert rel(to_host(plan.adjoint(to_dev(r32))), O.adjoint(r64, og, mask)) <= OP_TOL


def test_batch_items_are_independent():
    import paper_2108_01438_amd as P
    flush("[batch] items independent")
    kw = dict(CASES["bscan_200x60_k300_b2"])
    og, pg = both_geoms(**kw)
    _, pg1 = both_geoms(**dict(kw, batch=1))
    rng = np.random.default_rng(3)
    plan = P.Plan(pg)
    plan1 = P.Plan(pg1)
    x32, _ = rand_image(rng, O.img_shape(og))
    y = to_host(plan.forward(to_dev(x32)))
    y1 = to_host(plan1.forward(to_dev(x32[1:2].copy())))
    assert np.array_equal(y[1:2].view(np.uint32), y1.view(np.uint32))


def test_nonfinite_inputs_stay_local():
    """A NaN in one batch item does not leak into another."""
    import paper_2108_01438_amd as P
    flush("[edge] NaN isolation")
    og, pg = both_geoms(**CASES["bscan_200x60_k300_b2"])
    rng = np.random.default_rng(4)
    plan = P.Plan(pg)
    x32, _ = rand_image(rng, O.img_shape(og))
    x32[0, 0, 3, 5] = np.nan
    y = to_host(plan.forward(to_dev(x32)))
    assert np.isnan(y[0]).any()
    assert np.isfinite(y[1]).all()
