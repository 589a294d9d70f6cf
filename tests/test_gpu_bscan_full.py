"""Full-size B-scan (2048 spectral px x 1000 A-scans, 50% random mask, TV,
100 FISTA iterations) against the FP64 oracle's stored reference
(tests/golden/bscan_2048x1000_tv100.npz, written by the script beside it):
z^100 at 2^18 seeded pixels, on the whole image border, the norms of its
40 x 64 tiles and a whole-image CountSketch (an estimate of the relative L2
error over every pixel) within 1e-4; the objective history within 1e-5."""
import importlib.util
import os
import sys

import numpy as np
import pytest

from gpu_util import flush, to_dev, to_host

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def _ref_module():
    spec = importlib.util.spec_from_file_location(
        "make_ref", os.path.join(HERE, "golden", "make_bscan_tv_reference.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_full_bscan_tv_reconstruction_matches_oracle():
    import paper_2108_01438_amd as P
    import refstats
    ref = np.load(os.path.join(HERE, "golden", "bscan_2048x1000_tv100.npz"))
    m = _ref_module()
    flush("[full B-scan] oracle inputs")
    pr, og, x_true, mask, noise = m.inputs()
    y32 = m.measurements(pr, og, x_true, mask, noise)
    assert abs(np.linalg.norm(y32.astype(np.float64)) - float(ref["ynorm"])) <= 1e-12 * float(ref["ynorm"])
    plan = P.Plan(P.Geometry.from_dict(pr["geom"]), mask)
    flush("[full B-scan] 100 TV iterations on the GPU")
    z, info = plan.mbir_solve(to_dev(y32), "tv", float(ref["lam"]), pr["iters"], delta=float(ref["delta"]),
                              tv_inner=10, objective=True)
    z = to_host(z)
    err = refstats.compare(z[0, 0], ref, "", tuple(ref["block"]))
    bd = m.border(z.astype(np.complex128))
    err["border"] = float(np.linalg.norm(bd - ref["border"]) / np.linalg.norm(ref["border"]))
    print(f"[full B-scan] errors vs the oracle: {err}")
    for k in ("samples", "blocks", "whole_sketch", "norm", "border"):
        assert err[k] <= 1e-4, (k, err[k])
    np.testing.assert_allclose(info["objective"], ref["hist"], rtol=1e-5)
    # the GPU's own power iteration agrees with the oracle's L
    L = plan.lipschitz(50, seed=0)
    assert abs(L - float(ref["L"])) <= 1e-5 * float(ref["L"])

