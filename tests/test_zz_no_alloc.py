"""The allocation-free NCC entry point (oct_ncc_noalloc) against oct_ncc:
same result on two calls in a row, the second on a smaller input; repeated
calls are bitwise equal; bad sizes are rejected before any device work."""
import ctypes

import numpy as np
import pytest

from gpu_util import flush, to_dev

pytestmark = pytest.mark.gpu


def _pair(rng, shape):
    import torch
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    z = (x + 0.3 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))).astype(np.complex64)
    return to_dev(x), to_dev(z), torch.empty((), dtype=torch.float64, device="cuda")


def test_ncc_noalloc_matches_ncc_on_two_calls_second_smaller():
    import torch
    import paper_2108_01438_amd as P
    rng = np.random.default_rng(71)
    cases = [P.Geometry(n_depth=2048, n_x=1000, n_k=2048),      # 2.05 M pixels: 1024 partial blocks
             P.Geometry(n_depth=96, n_x=24, n_k=96)]            # 2304 pixels: 9 partial blocks
    for g in cases:
        flush(f"[noalloc] NCC on {g.img_shape}")
        x, z, r = _pair(rng, g.img_shape)
        plan = P.Plan(g)
        want = plan.ncc(x, z)
        P.ncc_noalloc(x, z, r)
        torch.cuda.synchronize()
        got = float(r.item())
        assert abs(got - want) <= 1e-13 * abs(want), (got, want)
        again = torch.empty_like(r)
        P.ncc_noalloc(x, z, again)
        assert torch.equal(r, again)
        plan.close()


def test_ncc_noalloc_constant_magnitude_is_nan():
    import torch
    import paper_2108_01438_amd as P
    x = torch.ones((4, 64), dtype=torch.complex64, device="cuda")
    z = torch.randn((4, 64), dtype=torch.complex64, device="cuda")
    r = torch.empty((), dtype=torch.float64, device="cuda")
    P.ncc_noalloc(x, z, r)
    assert np.isnan(float(r.item()))


def test_ncc_noalloc_rejects_bad_sizes():
    import torch
    import paper_2108_01438_amd as P
    x = torch.ones(8, dtype=torch.complex64, device="cuda")
    r = torch.empty((), dtype=torch.float64, device="cuda")
    lib = P._lib
    p = ctypes.c_void_p(x.data_ptr())
    for n in (0, -1, (1 << 40) + 1):
        st = lib.oct_ncc_noalloc(p, p, ctypes.c_int64(n), ctypes.c_void_p(r.data_ptr()), None)
        assert st == P.OCT_E_INVALID and "n must be" in P.last_error()
    assert lib.oct_ncc_noalloc(None, p, ctypes.c_int64(8), ctypes.c_void_p(r.data_ptr()), None) == P.OCT_E_INVALID
