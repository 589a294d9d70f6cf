"""The serving loop on the GPU: every result in a concurrent mix is bitwise the
result of the same request solved alone, and one of them matches the oracle."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import flush, rel

pytestmark = pytest.mark.gpu


def _requests():
    import torch
    import paper_2108_01438_amd as P
    from paper_2108_01438_amd.serve import Request
    specs = [
        (dict(n_depth=128, n_x=64, n_k=128), "l1", 0.01, 30, False),
        (dict(n_depth=256, n_x=40, n_k=256), "tv", 0.005, 25, True),
        (dict(n_depth=96, n_x=48, n_k=96), "haar", 0.01, 20, False),
        (dict(n_depth=64, n_x=16, n_y=16, lateral_dims=2, n_k=64), "haar", 0.01, 15, False),
        (dict(n_depth=32, n_x=16, n_y=8, lateral_dims=2, n_k=32), "tv", 0.005, 10, False),
        (dict(n_depth=128, n_x=64, n_k=128), "l1", 0.02, 30, False),   # same geometry: plan reuse
        (dict(n_depth=256, n_x=40, n_k=256), "tv", 0.005, 25, True),
        (dict(n_depth=512, n_x=64, n_k=512), "l1", 0.01, 20, False),
    ]
    reqs = []
    for i, (geo, pen, lf, iters, masked) in enumerate(specs):
        rng = np.random.default_rng(4_000_000 + i)
        g = P.Geometry(**geo)
        mask = None
        if masked:
            mask = synth.mask_random_exact(rng, (g.n_y, g.n_x), g.n_k, g.n_k // 2)
        x = synth.scatterers(rng, g.img_shape, 12).astype(np.complex64)
        plan = P.Plan(g, mask)
        y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
        y = synth.noisy(y, synth.standard_normal(rng, y.shape), mask, 0.01).astype(np.float32)
        lam = lf * float(plan.adjoint(torch.from_numpy(y).cuda()).abs().max().item())
        delta = 1.0 / (1.05 * plan.lipschitz(50))
        plan.close()
        reqs.append(Request(geom=g, y=y, penalty=pen, lam=lam, iters=iters, mask=mask, delta=delta))
    return reqs


def test_mix_equals_alone_and_oracle():
    from paper_2108_01438_amd.serve import HipExecutor, Server, run_sequential
    flush("[serve] building requests")
    reqs = _requests()
    flush("[serve] alone")
    alone, _ = run_sequential(HipExecutor(slots=1), reqs)
    flush("[serve] mix")
    # a budget of ~2.5 of the largest requests: idle pooled plans are released
    # (without a device-wide wait) while other requests run
    from paper_2108_01438_amd.serve import request_footprint
    import paper_2108_01438_amd as P
    budget = int(2.5 * max(request_footprint(P, r) for r in reqs))
    srv = Server(HipExecutor(slots=4), mem_budget=budget, slots=4)
    futs = [srv.submit(r) for r in reqs]
    mix = [f.result(timeout=60) for f in futs]
    srv.close()
    for a, m in zip(alone, mix):
        assert np.array_equal(a.view(np.uint32), m.view(np.uint32))
    st = srv.latency_stats()
    assert st["n"] == len(reqs)
    # request 1 (masked TV B-scan) against the oracle
    r = reqs[1]
    og = O.Geometry(**{k: getattr(r.geom, k) for k in r.geom.__dataclass_fields__})
    zo, _ = O.fista(r.y.astype(np.float64), og, r.mask, O.PEN_TV, r.lam, r.delta, r.iters, tv_inner=10)
    assert rel(mix[1], zo) <= 1e-4


def test_released_plan_memory_is_reused_correctly():
    """oct_plan_release frees an idle plan without a device-wide wait; its
    memory serves the next plan, whose results are those of a fresh plan."""
    import torch
    import paper_2108_01438_amd as P
    g = P.Geometry(n_depth=256, n_x=64, n_k=256)
    gen = torch.Generator(device="cuda").manual_seed(3)
    x = torch.randn(g.img_shape, dtype=torch.complex64, device="cuda", generator=gen)
    a = P.Plan(g)
    ya = a.forward(x)
    torch.cuda.synchronize()
    a.release()
    for _ in range(3):
        b = P.Plan(g)
        yb = b.forward(x)
        z, _ = b.mbir_solve(yb, "tv", 0.1, 5, delta=1e-4)
        torch.cuda.synchronize()
        assert torch.equal(ya, yb)
        b.release()
