"""The C-ABI library loads, exports what include/oct.h declares, and rejects
bad arguments before touching the device (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "oct.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(oct_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["oct_plan_create", "oct_plan_destroy", "oct_forward", "oct_adjoint", "oct_grad", "oct_prox",
              "oct_mbir_solve", "oct_lipschitz", "oct_last_error", "oct_plan_footprint_bytes", "oct_direct",
              "oct_adjoint_paper", "oct_dtcwt_filter",
              "oct_ncc"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2108_01438_amd as P
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(oct_\w+)", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(P.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n)


def _g(**kw):
    import paper_2108_01438_amd as P
    base = dict(n_depth=64, n_x=8, n_k=64)
    base.update(kw)
    return P.Geometry(**base)


@pytest.mark.parametrize("kw,status", [
    (dict(n_depth=0), 1), (dict(n_k=1), 1), (dict(batch=0), 1), (dict(kb_width=5), 1),
    (dict(lateral_dims=1, n_y=3), 1), (dict(k_min=3.0, k_max=2.0), 1), (dict(oversamp=1.7, n_depth=63), 1),
    (dict(n_x=11), 4), (dict(n_depth=8192), 4), (dict(lateral_dims=2, n_y=13), 4),
    # maximum sizes: more spectrometer pixels than the column kernels take, and grid coordinates
    # t = K dz k / pi beyond the adjoint's 16-bit base cells (dz = 100 um: ~3.4e4 cells)
    (dict(n_k=9000), 4), (dict(dz=100.0), 4),
])
def test_plan_create_rejects_bad_geometry(kw, status):
    import paper_2108_01438_amd as P
    with pytest.raises(P.OctError) as e:
        P.Plan(_g(**kw))
    assert e.value.status == status
    assert len(P.last_error()) > 0


def test_footprint_scales_with_size_and_penalty():
    import paper_2108_01438_amd as P
    a = P.footprint_bytes(_g())
    b = P.footprint_bytes(_g(n_x=64))
    c = P.footprint_bytes(_g(n_x=64), P.PEN_TV)
    assert 0 < a < b < c
    n = 64 * 64
    assert b >= n * 8 * 4                # workspace + two iterates
    assert P.footprint_bytes(_g(n_depth=0)) == 0


def test_mask_shape_checked_on_host():
    import numpy as np
    import paper_2108_01438_amd as P
    with pytest.raises(ValueError):
        P.Plan(_g(), mask=np.ones((1, 8, 63), dtype=np.uint8))


def test_dtcwt_filters_designed_by_the_library_match_the_oracle():
    """The library designs the DT-CWT filters on the host, independently of the
    oracle (its own halfband solve, Weierstrass root finder and spectral
    factor); both give the same taps, up to the FP32 rounding of the library's."""
    import paper_2108_01438_amd as P
    import oracle as O
    F = O.dtcwt_filters()
    ref = [F["first"][0], F["first"][1], F["later"][0], F["later"][1]]
    for which in range(4):
        got = P.dtcwt_filter(which)
        assert got.shape == ref[which].shape
        np.testing.assert_allclose(got, ref[which], atol=1e-7)
    with pytest.raises(P.OctError):
        P.dtcwt_filter(4)


def _shift_orthonormal(h, tol):
    for k in range(0, len(h) // 2):
        s = float(np.dot(h[: len(h) - 2 * k], h[2 * k:]))
        assert abs(s - (1.0 if k == 0 else 0.0)) <= tol, (k, s)


def _highpass_moments(h, K, tol):
    n = np.arange(len(h))
    for p in range(K):
        assert abs(float(np.sum((-1.0) ** n * n ** p * h))) <= tol * max(1, len(h) ** p), p


def test_dtcwt_filters_of_the_library_satisfy_their_design_properties():
    """The DT-CWT filters the library designs on the host, checked against the
    mathematics of the design rather than against the oracle's own design:
    lowpass sum sqrt(2), orthonormal to even shifts, K = 3 vanishing moments;
    the first level is the published 6-tap Daubechies filter (tree b one sample
    later); the later-level pair has equal magnitude responses and tree b lags
    tree a by half a sample at low frequencies (Selesnick's common-factor
    design with a maximally flat delay)."""
    import paper_2108_01438_amd as P
    a1, b1, a2, b2 = (P.dtcwt_filter(w) for w in range(4))
    for h in (a1, b1, a2, b2):
        assert abs(h.sum() - np.sqrt(2.0)) <= 1e-6
        _shift_orthonormal(h, 1e-6)
        _highpass_moments(h, 3, 1e-5)
    d6 = np.array([0.3326705529500825, 0.8068915093110924, 0.4598775021184914,
                   -0.1350110200102546, -0.0854412738820267, 0.0352262918857095])   # Daubechies 1988
    core = a1[np.abs(a1) > 1e-9]
    assert min(np.max(np.abs(core - d6)), np.max(np.abs(core[::-1] - d6))) <= 2e-6
    assert np.allclose(b1[1:], a1[:-1], atol=0) and b1[0] == 0.0
    w = np.linspace(0.0, np.pi, 257)
    E = np.exp(-1j * np.outer(w, np.arange(len(a2))))
    Ha, Hb = E @ a2, E @ b2
    assert np.max(np.abs(np.abs(Ha) - np.abs(Hb))) <= 1e-6
    low = w <= np.pi / 2
    dphi = np.unwrap(np.angle(Hb[low])) - np.unwrap(np.angle(Ha[low]))
    dphi -= dphi[0]
    assert np.max(np.abs(dphi + 0.5 * w[low])) <= 0.02 or np.max(np.abs(dphi - 0.5 * w[low])) <= 0.02
