"""Pins of the oracle's dual-tree complex wavelet transform (Sec. 2.2): the
filter design against closed forms and its defining properties, the transform
against Parseval, perfect reconstruction, analyticity and shift invariance,
and its shrinkage step."""
import math

import numpy as np
import pytest

import oracle as O


def cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def test_daubechies_special_case_closed_form():
    """L = 0, K = 2 is the 4-tap Daubechies filter (1+r3, 3+r3, 3-r3, 1-r3)/(4 r2)."""
    h, g = O.maxflat_halfband_factor(2, 0)
    r3, r2 = math.sqrt(3.0), math.sqrt(2.0)
    ref = np.array([1 + r3, 3 + r3, 3 - r3, 1 - r3]) / (4 * r2)
    np.testing.assert_allclose(h, ref, atol=1e-13)
    np.testing.assert_allclose(g, ref, atol=1e-13)


@pytest.mark.parametrize("K,L", [(3, 0), (2, 2), (3, 3)])
def test_design_orthonormal_with_vanishing_moments(K, L):
    h, g = O.maxflat_halfband_factor(K, L)
    for f in (h, g):
        n = len(f)
        assert abs(np.sum(f) - math.sqrt(2.0)) < 1e-12
        for k in range(n // 2):
            c = np.dot(f[:n - 2 * k], f[2 * k:])
            assert abs(c - (1.0 if k == 0 else 0.0)) < 1e-11, (k, c)
        hi = np.array([(-1) ** i * f[n - 1 - i] for i in range(n)])
        for m in range(K):
            mom = np.sum(np.arange(n) ** m * hi)
            assert abs(mom) < 1e-9 * np.sum(np.abs(np.arange(n) ** m * hi)), (m, mom)


@pytest.mark.parametrize("L", [2, 3])
def test_design_half_sample_delay(L):
    """G/H is the allpass z^-L D(1/z)/D(z): unit modulus and a maximally flat
    delay of half a sample at low frequency."""
    h, g = O.maxflat_halfband_factor(3, L)
    w = np.linspace(1e-3, 0.2, 50)
    e = np.exp(-1j * w)
    H = np.polyval(h[::-1], e)
    G = np.polyval(g[::-1], e)
    ratio = G / H
    np.testing.assert_allclose(np.abs(ratio), 1.0, atol=1e-9)
    phase = np.unwrap(np.angle(ratio))
    assert np.max(np.abs(phase + 0.5 * w)) < 1e-6


def _equiv_wavelet(first, later, level):
    def up(f, m):
        o = np.zeros((len(f) - 1) * m + 1)
        o[::m] = f
        return o

    def qmf(f):
        n = len(f)
        return np.array([(-1) ** i * f[n - 1 - i] for i in range(n)])
    e = first
    for j in range(2, level):
        e = np.convolve(e, up(later, 2 ** (j - 1)))
    return np.convolve(e, up(qmf(later), 2 ** (level - 1)))


@pytest.mark.parametrize("level", [2, 3, 4])
def test_complex_wavelet_is_nearly_analytic(level):
    """The tree-b wavelet is close to the Hilbert transform of the tree-a one:
    psi_a + j psi_b has almost no energy at negative frequencies.  Negative
    control: pairing tree a with itself one sample later (no half-sample
    delay at the later levels) leaves a large share there."""
    F = O.dtcwt_filters()
    (fa, fb), (ha, hb) = F["first"], F["later"]

    def neg_share(pa, pb):
        c = np.zeros(8192, dtype=complex)
        c[:len(pa)] += pa
        c[:len(pb)] += 1j * pb
        S = np.abs(np.fft.fft(c)) ** 2
        return min(S[4097:].sum(), S[1:4096].sum()) / S.sum()
    assert neg_share(_equiv_wavelet(fa, ha, level), _equiv_wavelet(fb, hb, level)) < 1e-3
    assert neg_share(_equiv_wavelet(fa, ha, level), _equiv_wavelet(fb, ha, level)) > 2e-2


@pytest.mark.parametrize("shape,levels", [((1, 1, 40, 64), 3), ((2, 1, 24, 16), 2), ((1, 1, 8, 8), 1)])
def test_dtcwt_parseval_and_perfect_reconstruction(shape, levels):
    rng = np.random.default_rng(3)
    x = cn(rng, shape)
    det, lows = O.dtcwt_forward(x, (3, 2), levels)
    e = sum(np.sum(np.abs(u) ** 2 + np.abs(w) ** 2) for per in det for pair in per for u, w in pair)
    e += sum(np.sum(np.abs(v) ** 2) for v in lows.values())
    assert abs(e / np.sum(np.abs(x) ** 2) - 1.0) < 1e-12
    np.testing.assert_allclose(O.dtcwt_inverse(det, lows, (3, 2), levels), x, atol=1e-12)


def test_dtcwt_shift_invariance_against_a_single_tree():
    """Band energies of the DT-CWT barely move under a one-sample shift of the
    image; those of the single-tree Haar DWT move a lot."""
    n = 64
    zz, xx = np.meshgrid(np.arange(n), np.arange(32), indexing="xy")
    img = np.exp(-((zz - 30.3) ** 2) / 8.0 - ((xx - 15.2) ** 2) / 8.0)[None, None].astype(complex)

    def dt_energy(a):
        det, _ = O.dtcwt_forward(a, (3, 2), 3)
        return np.array([sum(np.sum(np.abs(u) ** 2 + np.abs(w) ** 2) for pair in det[2] for u, w in pair)])

    def haar_energy(a):
        c = O.haar_forward(a, (3, 2), 3)
        m = O.haar_detail_mask(c.shape, (3, 2), 3)
        lev3 = np.zeros_like(m)
        lev3[..., : 32 // 4, : n // 4] = True
        return np.array([np.sum(np.abs(c[m & lev3]) ** 2)])
    var_dt = np.std([dt_energy(np.roll(img, s, axis=3))[0] for s in range(8)])
    var_h = np.std([haar_energy(np.roll(img, s, axis=3))[0] for s in range(8)])
    mean_dt = np.mean([dt_energy(np.roll(img, s, axis=3))[0] for s in range(8)])
    mean_h = np.mean([haar_energy(np.roll(img, s, axis=3))[0] for s in range(8)])
    print("relative spread of level-3 band energy: DT-CWT", var_dt / mean_dt, "Haar", var_h / mean_h)
    assert var_dt / mean_dt < 0.25 * (var_h / mean_h)


def test_prox_dtcwt_limits_and_nonexpansive():
    rng = np.random.default_rng(4)
    v = cn(rng, (1, 1, 32, 48))
    axes = (3, 2)
    np.testing.assert_allclose(O.prox_dtcwt(v, 0.0, axes, 3), v, atol=1e-12)
    det, lows = O.dtcwt_forward(v, axes, 3)
    zero = [[((0 * u1, 0 * v1), (0 * u2, 0 * v2)) for (u1, v1), (u2, v2) in per] for per in det]
    np.testing.assert_allclose(O.prox_dtcwt(v, 1e6, axes, 3), O.dtcwt_inverse(zero, lows, axes, 3), atol=1e-12)
    w = v + 0.1 * cn(rng, v.shape)
    a, b = O.prox_dtcwt(v, 0.3, axes, 3), O.prox_dtcwt(w, 0.3, axes, 3)
    assert np.linalg.norm(a - b) <= np.linalg.norm(v - w) * (1 + 1e-12)
    assert O.dtcwt_value(a, axes, 3) < O.dtcwt_value(v, axes, 3)


def test_fista_dtcwt_reduces_objective():
    g = O.Geometry(n_depth=32, n_x=16, n_k=32)
    rng = np.random.default_rng(5)
    xt = np.zeros(O.img_shape(g), dtype=complex)
    xt[0, 0, 4, 10] = 1.0
    xt[0, 0, 9, 20] = 0.5j
    y = O.forward(xt, g) + 0.01 * rng.standard_normal(O.meas_shape(g))
    delta = O.step_size(O.lipschitz(g, None, iters=100))
    lam = 0.02 * O.lambda_max(y, g)

    def F(z):
        return O.data_loss(z, y, g) + lam * O.dtcwt_value(z, (3, 2), 2)
    z5, _ = O.fista(y, g, None, O.PEN_DTCWT, lam, delta, 5, haar_levels=2)
    z60, hist = O.fista(y, g, None, O.PEN_DTCWT, lam, delta, 60, haar_levels=2)
    assert F(z60) < F(z5) < F(np.zeros_like(z5))


def test_oriented_subbands_occupy_one_quadrant():
    """Each of the six complex subbands of the 2-D transform is a complex
    wavelet whose spectrum lies almost entirely in one quadrant of the 2-D
    frequency plane (the orientation selectivity the tree combination buys; a
    sign slip in the combination spreads it over two quadrants)."""
    shape, levels, lev = (1, 1, 64, 64), 3, 1
    x = np.zeros(shape, dtype=complex)
    det, lows = O.dtcwt_forward(x, (3, 2), levels)
    for band in range(3):
        for which in range(2):
            resp = []
            for comp in range(2):
                d = [[((np.zeros_like(u1), np.zeros_like(v1)), (np.zeros_like(u2), np.zeros_like(v2)))
                      for (u1, v1), (u2, v2) in per] for per in det]
                pair = list(d[lev][band][which])
                c = np.zeros_like(pair[comp])
                c[0, 0, c.shape[2] // 2, c.shape[3] // 2] = 1.0
                pair[comp] = c
                d[lev][band] = tuple(tuple(pair) if k == which else d[lev][band][k] for k in range(2))
                resp.append(O.dtcwt_inverse(d, {t: np.zeros_like(v) for t, v in lows.items()}, (3, 2), levels))
            psi = resp[0] + 1j * resp[1]
            S = np.abs(np.fft.fft2(psi[0, 0])) ** 2
            h = S.shape[0] // 2, S.shape[1] // 2
            quads = [S[:h[0], :h[1]].sum(), S[:h[0], h[1]:].sum(), S[h[0]:, :h[1]].sum(), S[h[0]:, h[1]:].sum()]
            q = np.array(quads) / sum(quads)
            print(band, which, np.round(q, 4))
            # the high-pass direction is analytic: one half plane holds all but a trace
            half = max(q[0] + q[1], q[2] + q[3], q[0] + q[2], q[1] + q[3])
            assert half > 0.999, (band, which, q)
            # diagonal bands are analytic in both directions: one quadrant
            if band == 2:
                assert q.max() > 0.99, (band, which, q)


@pytest.mark.parametrize("d", [2, 3])
def test_combination_is_orthogonal(d):
    C = O.dtcwt_combination(d)
    np.testing.assert_allclose(C @ C.T, np.eye(2 ** d), atol=1e-15)


@pytest.mark.parametrize("shape,levels", [((1, 8, 8, 16), 2), ((2, 4, 8, 8), 1), ((1, 16, 8, 32), 3)])
def test_dtcwt_3d_parseval_and_perfect_reconstruction(shape, levels):
    rng = np.random.default_rng(6)
    x = cn(rng, shape)
    axes = (3, 2, 1)
    det, lows = O.dtcwt_forward(x, axes, levels)
    assert len(det[0]) == 7 and len(det[0][0]) == 4          # 28 oriented subbands per level
    e = sum(np.sum(np.abs(u) ** 2 + np.abs(w) ** 2) for per in det for pairs in per for u, w in pairs)
    e += sum(np.sum(np.abs(v) ** 2) for v in lows.values())
    assert abs(e / np.sum(np.abs(x) ** 2) - 1.0) < 1e-12
    np.testing.assert_allclose(O.dtcwt_inverse(det, lows, axes, levels), x, atol=1e-12)
    np.testing.assert_allclose(O.prox_dtcwt(x, 0.0, axes, levels), x, atol=1e-12)


def test_dtcwt_3d_diagonal_subbands_occupy_one_octant():
    """The four complex subbands of the all-high-pass band of the 3-D transform
    each lie almost entirely in one octant of the frequency space, four
    different ones (a sign slip in the combination spreads them over two)."""
    shape, levels, lev, band = (1, 32, 32, 32), 3, 1, 6
    x = np.zeros(shape, dtype=complex)
    det, lows = O.dtcwt_forward(x, (3, 2, 1), levels)
    zero_lows = {t: np.zeros_like(v) for t, v in lows.items()}
    best = []
    for which in range(4):
        resp = []
        for comp in range(2):
            d = [[[(np.zeros_like(u), np.zeros_like(w)) for u, w in pairs] for pairs in per] for per in det]
            c = np.zeros_like(det[lev][band][which][comp])
            c[0, c.shape[1] // 2, c.shape[2] // 2, c.shape[3] // 2] = 1.0
            pair = list(d[lev][band][which])
            pair[comp] = c
            d[lev][band][which] = tuple(pair)
            resp.append(O.dtcwt_inverse(d, zero_lows, (3, 2, 1), levels))
        psi = (resp[0] + 1j * resp[1])[0]
        S = np.abs(np.fft.fftn(psi)) ** 2
        h = [n // 2 for n in S.shape]
        oct_e = [S[a * h[0]:(a + 1) * h[0], b * h[1]:(b + 1) * h[1], c_ * h[2]:(c_ + 1) * h[2]].sum()
                 for a in range(2) for b in range(2) for c_ in range(2)]
        q = np.array(oct_e) / sum(oct_e)
        assert q.max() > 0.99, (which, np.round(q, 3))
        best.append(int(np.argmax(q)))
    assert len(set(best)) == 4
