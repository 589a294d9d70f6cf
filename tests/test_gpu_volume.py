"""The 2048 x 256 x 256 volume workload (2-D lateral FFT, 3-level 3-D Haar):
properties that hold at any size, checked at full size; the full-size solves
(noisy and noise-free) against the FP64 oracle's stored reference; oracle
parity of the same path on a smaller volume."""
import os
import sys

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import both_geoms, flush, rand_image, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

FULL = synth.preset("volume_2048x256x256_haar")["geom"]


def test_full_volume_separable_inputs_match_oracle_bscans():
    """An image constant along y gives, on every y-plane, the B-scan result of
    its x-profile (only q_y = 0 survives the lateral transform); likewise
    along x.  Checked at the full 2048 x 256 x 256 size against the oracle's
    2048 x 256 B-scan."""
    import torch
    import paper_2108_01438_amd as P
    flush("[volume] full-size separable inputs")
    g = P.Geometry.from_dict(FULL)
    plan = P.Plan(g)
    ob = O.Geometry(**dict(FULL, lateral_dims=1, n_y=1))
    rng = np.random.default_rng(31)
    b32, b64 = rand_image(rng, (1, 1, 256, 2048))
    yb = O.forward(b64, ob)[0, 0]                       # (256, 2048)
    x = torch.from_numpy(b32[0, 0]).cuda()
    vol = x[None, None, :, :].expand(1, 256, 256, 2048).contiguous()     # constant along y
    y = plan.forward(vol)
    for ly in (0, 77, 255):
        assert rel(to_host(y[0, ly]), yb) <= 1e-5
    vol = x[None, :, None, :].expand(1, 256, 256, 2048).contiguous()     # constant along x
    y = plan.forward(vol)
    for lx in (0, 130, 255):
        assert rel(to_host(y[0, :, lx]), yb) <= 1e-5


def test_full_volume_adjoint_identity():
    import torch
    import paper_2108_01438_amd as P
    flush("[volume] full-size adjoint identity")
    g = P.Geometry.from_dict(FULL)
    plan = P.Plan(g)
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn(g.img_shape, dtype=torch.complex64, device="cuda", generator=gen)
    r = torch.randn(g.meas_shape, dtype=torch.float32, device="cuda", generator=gen)
    y = plan.forward(x)
    a = plan.adjoint(r)
    lhs = float((y.double() * r.double()).sum().item())
    rhs = float((torch.view_as_real(x).double() * torch.view_as_real(a).double()).sum().item())
    scale = float(y.double().norm().item() * r.double().norm().item())
    assert abs(lhs - rhs) <= 1e-6 * scale


def _volume_specimen(rng, shape, n_scat, field_rms):
    x = synth.scatterers(rng, shape, n_scat)
    x[0] += synth.smooth_field_coarse(rng, shape[1:], 16, field_rms)
    return x.astype(np.complex64)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def volume_reference():
    """The oracle's stored reference of the full-size volume solve and the
    oracle's own float32 measurements of the same seeded specimen (the oracle's
    forward operator at full size on the host's threads)."""
    import importlib.util
    path = os.path.join(GOLDEN, "volume_2048x256x256_haar50.npz")
    if not os.path.exists(path):
        pytest.skip("the oracle's volume reference has not been written (make_volume_haar_reference.py)")
    ref = np.load(path)
    spec = importlib.util.spec_from_file_location("make_vol_ref", os.path.join(GOLDEN, "make_volume_haar_reference.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    flush("[volume] oracle measurements of the full-size specimen (host threads)")
    prev = O.set_workers(min(16, os.cpu_count() or 1))
    try:
        pr, g, x, noise = m.inputs()
        yn, yc = m.measurements(pr, g, x, noise)
    finally:
        O.set_workers(prev)
    return m, pr, ref, {"noisy_": yn, "clean_": yc}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("tag", ["noisy_", "clean_"])
def test_full_volume_haar_reconstruction_matches_oracle(volume_reference, tag):
    """50 FISTA iterations with the 3-level Haar prox on the full 2048 x 256 x
    256 volume, with 1% noise and noise-free, against the FP64 oracle's stored
    reference: z^50 at 2^16 seeded voxels, the norms of its 64 x 16 x 16
    blocks, a whole-volume CountSketch (the relative L2 error over every
    voxel, estimated) and its norm within 1e-4; the objective history within
    1e-5."""
    import paper_2108_01438_amd as P
    sys.path.insert(0, GOLDEN)
    import refstats
    m, pr, ref, ys = volume_reference
    y32 = ys[tag]
    ynorm = float(np.linalg.norm(y32.reshape(-1).astype(np.float64)))
    assert abs(ynorm - float(ref[tag + "ynorm"])) <= 1e-12 * ynorm
    plan = P.Plan(P.Geometry.from_dict(pr["geom"]))
    flush(f"[volume] {tag[:-1]}: 50 Haar iterations on the GPU")
    z, info = plan.mbir_solve(to_dev(y32), "haar", float(ref[tag + "lam"]), int(ref["iters"]),
                              delta=float(ref["delta"]), haar_levels=3, objective=True)
    z = to_host(z)
    plan.close()
    err = refstats.compare(z[0], ref, tag, tuple(int(b) for b in ref["block"]))
    print(f"[volume] {tag[:-1]} errors vs the oracle: {err}")
    for k in ("samples", "blocks", "whole_sketch", "norm"):
        assert err[k] <= 1e-4, (k, err[k])
    np.testing.assert_allclose(info["objective"], ref[tag + "hist"], rtol=1e-5)


def test_smaller_volume_haar_fista_matches_oracle():
    import paper_2108_01438_amd as P
    flush("[volume] 256 x 64 x 64 Haar FISTA vs oracle")
    kw = dict(FULL, n_depth=256, n_k=256, n_x=64, n_y=64)
    og, pg = both_geoms(**kw)
    rng = np.random.default_rng(7)
    x = _volume_specimen(rng, O.img_shape(og), 60, 0.04)
    y = synth.noisy(O.forward(x.astype(np.complex128), og), synth.standard_normal(rng, O.meas_shape(og)),
                    None, 0.01).astype(np.float32)
    y64 = y.astype(np.float64)
    lam = 0.01 * O.lambda_max(y64, og)
    delta = O.step_size(O.lipschitz(og, None, iters=10))
    zo, ho = O.fista(y64, og, None, O.PEN_HAAR, lam, delta, 12, haar_levels=3)
    plan = P.Plan(pg)
    z, info = plan.mbir_solve(to_dev(y), "haar", lam, 12, delta=delta, objective=True)
    err = rel(to_host(z), zo)
    print(f"[volume] 256x64x64 Haar rel err {err:.3e}")
    assert err <= 1e-4
    np.testing.assert_allclose(info["objective"], ho, rtol=1e-5)
