"""The 2048 x 256 x 256 volume workload (2-D lateral FFT, 3-level 3-D Haar):
properties that hold at any size, checked at full size, and oracle parity of
the same path on a smaller volume."""
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


@pytest.fixture(scope="module")
def full_specimen():
    """5000 scatterers in a smooth random background at 5% of the mean
    scatterer amplitude, at the full volume size (complex64)."""
    flush("[volume] generating the full-size specimen")
    pr = synth.preset("volume_2048x256x256_haar")
    rng = np.random.default_rng(2)
    shape = (1, FULL["n_y"], FULL["n_x"], FULL["n_depth"])
    return _volume_specimen(rng, shape, pr["scatterers"], pr["field"] * 0.75)


@pytest.mark.parametrize("noise", [0.01, 0.0])
def test_full_volume_haar_solve(noise, full_specimen):
    """50 FISTA iterations with the 3-level Haar prox on the full volume: the
    objective falls, and without noise the data residual falls far."""
    import torch
    import paper_2108_01438_amd as P
    flush(f"[volume] full-size Haar solve, noise={noise}")
    pr = synth.preset("volume_2048x256x256_haar")
    g = P.Geometry.from_dict(FULL)
    plan = P.Plan(g)
    xt = torch.from_numpy(full_specimen).cuda()
    y = plan.forward(xt)
    if noise > 0:
        y = y + noise * float(y.abs().max().item()) * torch.randn_like(y)
    lam = pr["lam"] * float(plan.adjoint(y).abs().max().item())
    z, info = plan.mbir_solve(y, "haar", lam, pr["iters"], delta=0.0, power_iters=50, objective=True)
    h = info["objective"]
    assert np.all(np.isfinite(h)) and h[-1] < 0.5 * h[0]
    if noise == 0:
        r = plan.forward(z) - y
        assert float(r.norm().item()) / float(y.norm().item()) < 0.1
    z2, _ = plan.mbir_solve(y, "haar", lam, 3, delta=info["delta"])
    z3, _ = plan.mbir_solve(y, "haar", lam, 3, delta=info["delta"])
    assert torch.equal(z2, z3)


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
