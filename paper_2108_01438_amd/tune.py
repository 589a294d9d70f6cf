"""Regularisation-weight search of Sec. 3.2: lambda is chosen to maximise the
NCC of eq. (17) against a reference image by a golden-section line search.

The search runs over u = log10(lambda / lambda_max), lambda_max = ||Phi^H(s y)||_inf
(the weight above which the l1 solution is zero).  Every evaluation is one
FISTA solve and one NCC on the device (oct_mbir_solve, oct_ncc); independent
searches (other masks, penalties or specimens) can run concurrently on
separate plans and streams.  The coarse scan that brackets the search can run
as one batched solve: a plan with one batch item per candidate, the
measurement replicated over the batch and one weight per item (the solve's
per-item weights), then one allocation-free NCC per item.
"""
from __future__ import annotations

import math
from typing import Callable, List, Tuple

INV_PHI = (math.sqrt(5.0) - 1.0) / 2.0


def golden_section_max(f: Callable[[float], float], lo: float, hi: float, iters: int
                       ) -> Tuple[float, float, List[Tuple[float, float]]]:
    """Maximise a unimodal f on [lo, hi] with `iters` interval reductions by
    the golden ratio (iters + 2 evaluations).  Returns (u_best, f_best,
    [(u, f(u)) in evaluation order]); u_best is the best evaluated point."""
    hist: List[Tuple[float, float]] = []

    def ev(u: float) -> float:
        v = float(f(u))
        hist.append((u, v))
        return v

    a, b = float(lo), float(hi)
    c, d = b - INV_PHI * (b - a), a + INV_PHI * (b - a)
    fc, fd = ev(c), ev(d)
    for _ in range(iters):
        if fc >= fd:      # maximum in [a, d]
            b, d, fd = d, c, fc
            c = b - INV_PHI * (b - a)
            fc = ev(c)
        else:             # maximum in [c, b]
            a, c, fc = c, d, fd
            d = a + INV_PHI * (b - a)
            fd = ev(d)
    u_best, f_best = max(hist, key=lambda t: t[1])
    return u_best, f_best, hist


def scan_lambda_batched(plan_b, y, ref, penalty: str, lam_max: float, delta: float, us, iters: int = 100,
                        tv_inner: int = 10, haar_levels: int = 3, stream=None):
    """NCC(z^iters(lambda), ref) for lambda = lam_max 10^u, every u in `us`, from
    one batched solve.  plan_b: the search's geometry and mask with batch =
    len(us); y, ref: one measurement and one reference (batch 1).  Returns
    ([(u, ncc)], z) with z the batch of solutions."""
    import torch
    from . import ncc_noalloc
    B = plan_b.geom.batch
    if len(us) != B:
        raise ValueError("the plan's batch must equal the number of candidates")
    yb = y.expand((B,) + tuple(y.shape[1:])).contiguous()
    lams = [lam_max * 10.0 ** u for u in us]
    z, _ = plan_b.mbir_solve(yb, penalty, lams, iters, delta=delta, tv_inner=tv_inner, haar_levels=haar_levels,
                             stream=stream)
    r = torch.empty(B, dtype=torch.float64, device=y.device)
    for b in range(B):
        ncc_noalloc(z[b], ref[0], r[b], stream=stream)
    if stream is not None:
        stream.synchronize()
    return list(zip([float(u) for u in us], r.cpu().tolist())), z


def tune_lambda(plan, y, ref, penalty: str, lam_max: float, delta: float, iters: int = 100,
                u_range=(-3.5, -0.5), search_iters: int = 10, coarse: int = 0, tv_inner: int = 10,
                haar_levels: int = 3, stream=None, batched_plan=None):
    """Golden-section search of lambda = lam_max 10^u maximising NCC(z^iters, ref).
    With coarse > 1 the search is first bracketed by a scan of `coarse`
    equispaced u (the NCC need not be unimodal over a wide range) and the
    golden-section search then runs between the best scan point's neighbours;
    with batched_plan (batch = coarse, same geometry and mask) the scan is one
    batched solve.  Returns dict(lam, u, ncc, z, evaluations)."""
    import torch
    z = torch.empty_like(ref)

    def score(u: float) -> float:
        plan.mbir_solve(y, penalty, lam_max * 10.0 ** u, iters, delta=delta, tv_inner=tv_inner,
                        haar_levels=haar_levels, x_out=z, stream=stream)
        return plan.ncc(z, ref, stream=stream)

    lo, hi = float(u_range[0]), float(u_range[1])
    scan: List[Tuple[float, float]] = []
    if coarse > 1:
        us = [lo + (hi - lo) * i / (coarse - 1) for i in range(coarse)]
        if batched_plan is not None:
            scan, _ = scan_lambda_batched(batched_plan, y, ref, penalty, lam_max, delta, us, iters, tv_inner,
                                          haar_levels, stream)
        else:
            scan = [(u, score(u)) for u in us]
        i = max(range(coarse), key=lambda j: scan[j][1])
        lo, hi = us[max(i - 1, 0)], us[min(i + 1, coarse - 1)]
    u, r, hist = golden_section_max(score, lo, hi, search_iters)
    hist = scan + hist
    u, r = max(hist, key=lambda t: t[1])
    plan.mbir_solve(y, penalty, lam_max * 10.0 ** u, iters, delta=delta, tv_inner=tv_inner,
                    haar_levels=haar_levels, x_out=z, stream=stream)
    return dict(lam=lam_max * 10.0 ** u, u=u, ncc=r, z=z, evaluations=hist)


__all__ = ["golden_section_max", "scan_lambda_batched", "tune_lambda"]
