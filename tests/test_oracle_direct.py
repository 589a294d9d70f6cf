"""Pins of the oracle's direct reconstructions (Sec. 3.1, Figure 1) and the
interpolated-ISAM baseline: the axial transform is the paper's zero-pad and
2N-point inverse DFT, A-scans are independent, interpolation reproduces linear
spectra, and ISAM refocuses an out-of-focus point where the axial transform
does not."""
import numpy as np
import pytest

import oracle as O
import synth


def _g(**kw):
    base = dict(synth.OPTICS)
    base.update(dict(lateral_dims=1, n_y=1, batch=1))
    base.update(kw)
    return O.Geometry(**base)


@pytest.mark.parametrize("dispersion", [False, True])
def test_direct_axial_is_zero_pad_inverse_dft(dispersion):
    g = _g(n_depth=64, n_x=1, n_k=96, disp_a=2e-3, disp_b=1e-5)
    d = O.derived(g)
    rng = np.random.default_rng(0)
    y = rng.standard_normal(O.meas_shape(g))
    x = O.direct_axial(y, g, dispersion=dispersion, exact=True)[0, 0, 0]
    spec = y.reshape(-1).astype(np.complex128)
    if dispersion:
        spec = spec * np.exp(-1j * O.omega(g))
    two_n = 2 * g.n_depth
    padded = np.zeros(two_n, dtype=np.complex128)
    padded[: g.n_k] = spec
    ref = np.fft.ifft(padded) * two_n                       # e^{+j 2 pi m n / 2N}
    ref = ref[: g.n_depth] * np.exp(1j * 2.0 * g.k_min * np.arange(g.n_depth) * d.dz)
    assert np.max(np.abs(x - ref)) <= 1e-10 * np.max(np.abs(ref))
    # the KB form of the same transform, within the interpolation error
    xk = O.direct_axial(y, g, dispersion=dispersion)[0, 0, 0]
    assert np.linalg.norm(xk - ref) <= 2e-5 * np.linalg.norm(ref)


def test_direct_axial_treats_a_scans_independently():
    g = _g(n_depth=48, n_x=6, n_k=64)
    rng = np.random.default_rng(1)
    y = rng.standard_normal(O.meas_shape(g))
    mask = (rng.random((1, 6, 64)) < 0.6).astype(np.uint8)
    x = O.direct_axial(y, g, mask)
    g1 = g.with_(n_x=1)
    for l in range(6):
        x1 = O.direct_axial(y[:, :, l:l + 1], g1, mask[:, l:l + 1])
        assert np.allclose(x[:, :, l:l + 1], x1, rtol=0, atol=1e-12 * np.max(np.abs(x)))


def test_interp_fill_properties():
    g = _g(n_depth=32, n_x=5, n_k=40)
    rng = np.random.default_rng(2)
    y = rng.standard_normal(O.meas_shape(g))
    ones = np.ones((1, 5, 40), dtype=np.uint8)
    assert np.array_equal(O.interp_fill(y, g, ones), y)
    # a spectrum linear in the pixel index is recovered wherever it is bracketed
    lin = np.broadcast_to(1.5 - 0.25 * np.arange(40), O.meas_shape(g)).copy()
    m = (rng.random((1, 5, 40)) < 0.5).astype(np.uint8)
    m[..., 0] = 1
    m[..., -1] = 1
    assert np.allclose(O.interp_fill(lin, g, m), lin, atol=1e-13)
    # outside the observed band the nearest observed value is held
    part = synth.mask_partial((1, 5), 40)
    f = O.interp_fill(y, g, part)
    lo, hi = 10, 29
    assert np.array_equal(f[..., :lo], np.broadcast_to(y[..., lo:lo + 1], f[..., :lo].shape))
    assert np.array_equal(f[..., hi + 1:], np.broadcast_to(y[..., hi:hi + 1], f[..., hi + 1:].shape))
    # brute force on one A-scan: nearest observed neighbours on each side
    row, mr = y[0, 0, 2], m[0, 2]
    obs = [i for i in range(40) if mr[i]]
    fm = O.interp_fill(y, g, m)
    for i in range(40):
        left = max([o for o in obs if o <= i])
        right = min([o for o in obs if o >= i])
        want = row[left] if right == left else row[left] + (row[right] - row[left]) * (i - left) / (right - left)
        assert fm[0, 0, 2, i] == pytest.approx(want, abs=1e-13)
    # an A-scan with nothing observed stays zero
    none = m.copy()
    none[0, 3] = 0
    assert not np.any(O.interp_fill(y, g, none)[0, 0, 3])


def test_interp_isam_with_full_mask_is_isam():
    g = _g(n_depth=40, n_x=8, n_k=48)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(O.meas_shape(g))
    ones = np.ones((1, 8, 48), dtype=np.uint8)
    assert np.allclose(O.interp_isam(y, g, ones), O.direct_isam(y, g), atol=1e-12)


def test_isam_refocuses_an_out_of_focus_point():
    """A point 100 samples (~110 um, ~7 Rayleigh ranges of a 2 um waist) below
    the focus: the ISAM image puts its peak row's energy into the point's
    column and its neighbours, where the axial transform leaves the defocus
    blur spread over many columns."""
    g = _g(n_depth=256, n_x=64, n_k=256, beam_waist=2.0)
    x = np.zeros(O.img_shape(g), dtype=np.complex128)
    n0, l0 = O.derived(g).n_c + 100, 32
    x[0, 0, l0, n0] = 1.0
    y = O.forward(x, g)

    def lateral_concentration(img):
        a = np.abs(img[0, 0])
        row = a[:, n0 - 3: n0 + 4].max(axis=1)
        return float(np.sum(row[l0 - 1: l0 + 2] ** 2) / np.sum(row ** 2))

    c_isam = lateral_concentration(O.direct_isam(y, g))
    c_axial = lateral_concentration(O.direct_axial(y, g))
    assert c_isam > 0.99
    assert c_axial < 0.6
