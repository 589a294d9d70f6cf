"""Pins of the oracle's system operator against what the paper and the
mathematics fix (no GPU).  Each test names the part it pins."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import i0

import oracle as O


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def cn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# --- Kaiser-Bessel transform pair (deapodisation) ---------------------------
@pytest.mark.parametrize("J,sigma", [(4, 2.0), (6, 2.0), (8, 2.0), (6, 1.5)])
def test_kb_fourier_pair_against_quadrature(J, sigma):
    """Closed-form FT of both KB windows equals numerical quadrature."""
    b = O.kb_beta_default(J, sigma)
    for f in [0.0, 0.05, 0.13, 0.25, 0.4, 0.49]:
        q0 = integrate.quad(lambda u: float(O.kb_kernel(u, J, b)) * math.cos(2 * math.pi * f * u),
                            -J / 2, J / 2, epsabs=1e-15, epsrel=1e-13, limit=400)[0]
        qs = integrate.quad(lambda u: float(O.kb_kernel_standard(u, J, b)) * math.cos(2 * math.pi * f * u),
                            -J / 2, J / 2, epsabs=1e-15, epsrel=1e-13, limit=400)[0]
        assert abs(float(O.kb_deapod(f, J, b)) - q0) <= 1e-12 * abs(q0) + 1e-14
        assert abs(float(O.kb_deapod_standard(f, J, b)) - qs) <= 1e-12 * abs(qs)


def test_kb_shape_and_edge():
    """Beatty closed form for J=6, sigma=2; zero-edge window is 1 at 0, 0 at J/2."""
    b = O.kb_beta_default(6, 2.0)
    assert abs(b - math.pi * math.sqrt(9.0 * 1.5 ** 2 - 0.8)) < 1e-14
    assert abs(b - 13.855) < 1e-3
    assert O.kb_kernel(0.0, 6, b) == pytest.approx(1.0, abs=1e-15)
    assert float(O.kb_kernel(3.0, 6, b)) == 0.0
    assert float(O.kb_kernel(3.2, 6, b)) == 0.0
    assert float(O.kb_kernel_standard(3.0, 6, b)) == pytest.approx(1.0)   # I0(0) = 1
    assert float(O.kb_kernel_standard(0.0, 6, b)) == pytest.approx(float(i0(b)))


# --- NUFFT against the brute-force non-uniform DFT --------------------------
def _nudft(cols, g, q2):
    d = O.derived(g)
    beta, _, prop = O.beta_t(g, q2)
    n = np.arange(g.n_depth)
    out = np.zeros((cols.shape[0], g.n_k), dtype=complex)
    for c in range(cols.shape[0]):
        for m in range(g.n_k):
            if prop[c, m]:
                out[c, m] = np.sum(cols[c] * np.exp(-1j * beta[c, m] * d.dz * (n - d.n_c)))
    return out


@pytest.mark.parametrize("nz", [16, 32, 64])
def test_nufft_against_nudft(nz):
    rng = np.random.default_rng(nz)
    g = O.Geometry(n_depth=nz, n_x=4, n_k=nz)
    q2 = rng.uniform(0.0, 2.4, size=5)
    cols = cn(rng, (5, nz))
    H = O.filter_H(g, q2)
    ref = _nudft(cols, g, q2)
    errs = []
    for J in (4, 6, 8):
        gj = g.with_(kb_width=J)
        got = O.nufft_cols_forward(cols, q2, gj) / H
        errs.append(rel(got, ref))
    assert errs[1] <= 1e-5
    assert errs[0] > errs[1] > errs[2]
    # exact mode is the brute-force sum
    assert rel(O.nufft_cols_forward(cols, q2, g, exact=True) / H, ref) < 1e-13


def test_nufft_uncentred_negative_control():
    """Dropping the centring of the NUFFT index gives an O(0.1) error: the
    brute-force comparison above would catch that mistake."""
    rng = np.random.default_rng(3)
    g = O.Geometry(n_depth=64, n_x=4, n_k=64)
    q2 = rng.uniform(0.0, 2.4, size=4)
    cols = cn(rng, (4, 64))
    ref = _nudft(cols, g, q2)
    bad = O.nufft_cols_forward(cols, q2, g, centered=False) / O.filter_H(g, q2)
    assert rel(bad, ref) > 0.05


# --- adjoint identity ---------------------------------------------------------
GEOMS = [
    O.Geometry(n_depth=32, n_x=8, n_k=32),
    O.Geometry(n_depth=32, n_x=6, n_k=40, disp_b=2e-5, z_focus=10.0),
    O.Geometry(n_depth=16, n_x=4, n_y=4, lateral_dims=2, n_k=24, batch=2),
    O.Geometry(n_depth=24, n_x=5, n_k=48, kb_width=4, beam_waist=0.0),
    O.Geometry(n_depth=32, n_x=8, n_k=64),                         # paper sizing M = 2N
    O.Geometry(n_depth=16, n_x=8, n_k=16, k_min=0.3, k_max=0.9, dx=0.5),   # evanescent bins
    O.Geometry(n_depth=20, n_x=3, n_k=20, oversamp=2.5, kb_width=8),
]


@pytest.mark.parametrize("gi", range(len(GEOMS)))
def test_adjoint_identity(gi):
    g = GEOMS[gi]
    rng = np.random.default_rng(100 + gi)
    x = cn(rng, O.img_shape(g))
    r = rng.standard_normal(O.meas_shape(g))
    mask = (rng.random(O.meas_shape(g)[1:]) < 0.6).astype(np.uint8)
    for exact in (False, True):
        lhs = float(np.sum(O.forward(x, g, mask, exact=exact) * r))
        rhs = float(np.real(np.vdot(x, O.adjoint(r, g, mask, exact=exact))))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1e-300) * 10 + 1e-13 * np.linalg.norm(x) * np.linalg.norm(r)


def test_evanescent_components_vanish():
    g = GEOMS[5]
    q2 = O.q_squared(g).ravel()
    _, _, prop = O.beta_t(g, q2)
    assert (~prop).any() and prop.any()
    H = O.filter_H(g, q2)
    assert np.all(H[~prop] == 0)


# --- dense matrix: adjoint = transpose, L = sigma_max^2 -----------------------
def _dense(g, mask):
    n = int(np.prod(O.img_shape(g)))
    cols = []
    for j in range(n):
        e = np.zeros(n, dtype=complex)
        e[j] = 1.0
        cols.append(O.forward(e.reshape(O.img_shape(g)), g, mask).ravel())
    for j in range(n):
        e = np.zeros(n, dtype=complex)
        e[j] = 1j
        cols.append(O.forward(e.reshape(O.img_shape(g)), g, mask).ravel())
    return np.array(cols).T        # (M, 2N)


def test_dense_matrix_transpose_and_lipschitz():
    g = O.Geometry(n_depth=8, n_x=4, n_k=12)
    rng = np.random.default_rng(7)
    mask = (rng.random((1, 4, 12)) < 0.7).astype(np.uint8)
    A = _dense(g, mask)
    n = A.shape[1] // 2
    M = A.shape[0]
    for i in range(M):
        e = np.zeros(M)
        e[i] = 1.0
        a = O.adjoint(e.reshape(O.meas_shape(g)), g, mask).ravel()
        got = np.concatenate([a.real, a.imag])
        assert np.max(np.abs(got - A[i])) < 1e-13 * max(1.0, np.max(np.abs(A)))
    L = np.linalg.svd(A, compute_uv=False)[0] ** 2
    Lhat = O.lipschitz(g, mask, iters=2000)
    assert abs(Lhat - L) / L < 1e-9
    L50 = O.lipschitz(g, mask, iters=50)
    assert L50 <= L * (1 + 1e-12)


def test_paper_power_iteration_is_the_spectral_radius():
    """With backward="paper" the power iteration tends to the spectral radius of
    the real-linear map Phi* Phi (dense 2N x 2N matrix, eigenvalues by LAPACK),
    which on a masked B-scan exceeds the exact L = sigma_max(Phi)^2."""
    g = O.Geometry(n_depth=8, n_x=4, n_k=12)
    rng = np.random.default_rng(7)
    mask = (rng.random((1, 4, 12)) < 0.7).astype(np.uint8)
    n = int(np.prod(O.img_shape(g)))
    cols = []
    for j in range(2 * n):
        e = np.zeros(n, dtype=complex)
        e[j % n] = 1.0 if j < n else 1j
        w = O.paper_backward(O.forward(e.reshape(O.img_shape(g)), g, mask), g, mask).ravel()
        cols.append(np.concatenate([w.real, w.imag]))
    rho = float(np.max(np.abs(np.linalg.eigvals(np.array(cols).T))))
    Lp = O.lipschitz(g, mask, iters=2000, backward="paper")
    assert abs(Lp - rho) / rho < 1e-9
    assert rho > 1.2 * O.lipschitz(g, mask, iters=2000)


# --- the paper's literal D Q chain at a single A-scan --------------------------
@pytest.mark.parametrize("nz,mk", [(32, 32), (32, 64), (64, 48)])
def test_single_ascan_equals_literal_DQ_chain(nz, mk):
    """At q = 0 (one A-scan) Phi x = Re{e^{j Omega} D Q (x e^{-j 2 k_min z})} for
    the first M_k bins of the 2N_z-point DFT (eq. (7)-(9))."""
    g = O.Geometry(n_depth=nz, n_x=1, n_k=mk, disp_a=3e-3, disp_b=1e-5)
    rng = np.random.default_rng(nz + mk)
    x = cn(rng, nz)
    d = O.derived(g)
    zn = np.arange(nz) * d.dz
    pad = np.concatenate([x * np.exp(-2j * g.k_min * zn), np.zeros(nz)])
    D = np.fft.fft(pad)
    lit = np.real(np.exp(1j * O.omega(g)) * D[:mk])
    got = O.forward(x.reshape(1, 1, 1, nz), g, exact=True).ravel()
    assert rel(got, lit) < 1e-12
    kb = O.forward(x.reshape(1, 1, 1, nz), g).ravel()
    assert rel(kb, lit) < 2e-5


def test_paper_backward_relation():
    """Without dispersion and with M_k = 2 N_z the paper's Hilbert backward
    operator equals the exact adjoint times 1 (DC depth bin) and 2 (others)."""
    g = O.Geometry(n_depth=32, n_x=1, n_k=64, disp_a=0.0)
    M = g.n_k
    E = np.eye(M)
    A = np.array([O.adjoint(E[i].reshape(1, 1, 1, M), g, exact=True).ravel() for i in range(M)])
    P = np.array([O.paper_backward_nx1(E[i], g) for i in range(M)])
    c = np.array([np.vdot(A[:, n], P[:, n]) / np.vdot(A[:, n], A[:, n]) for n in range(g.n_depth)])
    expect = np.full(g.n_depth, 2.0)
    expect[0] = 1.0
    assert np.max(np.abs(c - expect)) < 1e-12
    for n in range(g.n_depth):
        assert np.linalg.norm(P[:, n] - c[n] * A[:, n]) < 1e-11


# --- the paper's literal K, Q, D chain (model 1) -------------------------------
def test_literal_chain_equals_the_direct_model_at_one_ascan():
    """At q = 0 (one A-scan) beta = 2k is linear in k, so the spectrum sampled at
    the even pixels and trigonometrically interpolated by D Q is exact: the
    literal chain equals the direct model at every pixel (exact NUDFT mode,
    with 2nd and 3rd order dispersion)."""
    rng = np.random.default_rng(31)
    g = O.Geometry(n_depth=32, n_x=1, n_k=64, disp_a=3e-3, disp_b=1e-5, model=1)
    x = cn(rng, O.img_shape(g))
    lit = O.forward(x, g, exact=True)
    direct = O.forward(x, g.with_(model=0), exact=True)
    assert rel(lit, direct) < 1e-12


def test_literal_chain_even_pixels_are_the_direct_model():
    """For any lateral frequency the even detector pixels of the literal chain
    carry K's samples unchanged, so they equal the direct model there; the odd
    pixels (interpolated) differ when q != 0."""
    rng = np.random.default_rng(32)
    g = O.Geometry(n_depth=64, n_x=24, n_k=128, model=1)
    x = cn(rng, O.img_shape(g))
    lit = O.forward(x, g)
    direct = O.forward(x, g.with_(model=0))
    assert rel(lit[..., ::2], direct[..., ::2]) < 1e-12
    assert rel(lit[..., 1::2], direct[..., 1::2]) > 1e-3


@pytest.mark.parametrize("kw", [dict(n_depth=32, n_x=12, n_k=64), dict(n_depth=16, n_x=6, n_y=5, lateral_dims=2, n_k=32)])
def test_literal_chain_adjoint_identity(kw):
    rng = np.random.default_rng(33)
    g = O.Geometry(model=1, **kw)
    mask = (rng.random(O.meas_shape(g)[1:]) < 0.6).astype(np.uint8)
    x = cn(rng, O.img_shape(g))
    r = rng.standard_normal(O.meas_shape(g))
    a = np.sum(O.forward(x, g, mask) * r)
    b = np.real(np.vdot(x, O.adjoint(r, g, mask)))
    assert abs(a - b) <= 1e-12 * abs(a)


def test_literal_chain_needs_mk_twice_nz():
    g = O.Geometry(n_depth=32, n_x=4, n_k=48, model=1)
    with pytest.raises(ValueError):
        O.forward(np.zeros(O.img_shape(g), complex), g)


# --- lateral structure ---------------------------------------------------------
def test_lateral_shift_equivariance():
    g = O.Geometry(n_depth=32, n_x=8, n_k=32)
    rng = np.random.default_rng(11)
    x = cn(rng, O.img_shape(g))
    y = O.forward(x, g)
    ys = O.forward(np.roll(x, 3, axis=2), g)
    assert rel(ys, np.roll(y, 3, axis=2)) < 1e-12


def test_volume_shift_equivariance_both_axes():
    g = O.Geometry(n_depth=16, n_x=4, n_y=6, lateral_dims=2, n_k=16)
    rng = np.random.default_rng(12)
    x = cn(rng, O.img_shape(g))
    y = O.forward(x, g)
    ys = O.forward(np.roll(np.roll(x, 1, axis=1), 2, axis=2), g)
    assert rel(ys, np.roll(np.roll(y, 1, axis=1), 2, axis=2)) < 1e-12


def _gaussian_beam_field(g, d_um, l0):
    """Paraxial Gaussian-beam closed form of a point scatterer at depth z_f + d:
    V(m, l) = e^{j theta_m} dx / (2 sqrt(pi a)) exp(-x^2 / (4 a)),
    a = w0^2/8 - j d/(4 k_m), theta_m = -2 k_m z_f + Omega_m - 2 k_m d,
    x = (l - l0) dx, periodised over the lateral field of view."""
    d = O.derived(g)
    k = O.k_grid(g)
    a = g.beam_waist ** 2 / 8.0 - 1j * d_um / (4.0 * k)
    theta = -2.0 * k * d.z_f + O.omega(g) - 2.0 * k * d_um
    out = np.zeros((g.n_x, g.n_k), dtype=complex)
    for l in range(g.n_x):
        for wrap in (-2, -1, 0, 1, 2):
            xx = (l - l0 + wrap * g.n_x) * g.dx
            out[l] += g.dx / (2.0 * np.sqrt(np.pi * a)) * np.exp(-xx * xx / (4.0 * a))
    return np.real(np.exp(1j * theta)[None, :] * out)


@pytest.mark.parametrize("dn", [0, 12, -12])
def test_point_scatterer_gaussian_beam(dn):
    """In focus the lateral PSF is the Gaussian of waist w0; out of focus it
    follows the paraxial Gaussian-beam law with the defocus sign of eq. (5)."""
    g = O.Geometry(n_depth=64, n_x=64, n_k=64)
    d = O.derived(g)
    x = np.zeros(O.img_shape(g), dtype=complex)
    l0 = 20
    x[0, 0, l0, d.n_c + dn] = 1.0
    y = O.forward(x, g, exact=True)[0, 0]
    ref = _gaussian_beam_field(g, dn * d.dz, l0)
    assert np.max(np.abs(y - ref)) < 3e-3 * np.max(np.abs(ref))


# --- gradient -------------------------------------------------------------------
def test_gradient_central_differences():
    g = O.Geometry(n_depth=16, n_x=4, n_k=20)
    rng = np.random.default_rng(5)
    x = cn(rng, O.img_shape(g))
    y = rng.standard_normal(O.meas_shape(g))
    mask = (rng.random(O.meas_shape(g)[1:]) < 0.5).astype(np.uint8)
    gr, _ = O.grad(x, y, g, mask)
    f0 = O.data_loss(x, y, g, mask)
    h = 1e-6
    for _ in range(10):
        dvec = cn(rng, x.shape)
        fp = O.data_loss(x + h * dvec, y, g, mask)
        fm = O.data_loss(x - h * dvec, y, g, mask)
        fd = (fp - fm) / (2 * h)
        an = float(np.real(np.vdot(gr, dvec)))
        # the loss is quadratic: central differences are exact up to rounding,
        # which is about eps * f0 / h = 2.2e-10 f0
        assert abs(fd - an) <= 1e-9 * (f0 + abs(an))


def test_paper_backward_general_form_matches_the_literal_chain():
    """The general backward operator (conjugate analytic signal, then the
    adjoint of the complex model) equals the literal K^H D^H Q^T chain of the
    single-A-scan form, with and without dispersion (exact NUDFT mode)."""
    rng = np.random.default_rng(12)
    for disp in (0.0, 3e-3):
        g = O.Geometry(n_depth=32, n_x=1, n_k=64, disp_a=disp)
        r = rng.standard_normal(O.meas_shape(g))
        p = O.paper_backward(r, g, exact=True).ravel()
        lit = O.paper_backward_nx1(r.ravel(), g)
        assert np.max(np.abs(p - lit)) <= 1e-11 * np.max(np.abs(lit))


def test_paper_backward_b_scan_properties():
    """On a masked B-scan the backward operator is linear, sees only observed
    samples, and differs from the exact adjoint (it is not Phi's transpose)."""
    g = O.Geometry(n_depth=40, n_x=12, n_k=56)
    rng = np.random.default_rng(13)
    mask = (rng.random((1, 12, 56)) < 0.6).astype(np.uint8)
    a, b = rng.standard_normal(O.meas_shape(g)), rng.standard_normal(O.meas_shape(g))
    pa, pb = O.paper_backward(a, g, mask), O.paper_backward(b, g, mask)
    assert np.allclose(O.paper_backward(2.0 * a - b, g, mask), 2.0 * pa - pb, atol=1e-12)
    assert np.allclose(O.paper_backward(a + (1 - mask[None]) * b, g, mask), pa, atol=1e-12)
    ex = O.adjoint(a, g, mask)
    assert np.linalg.norm(pa - ex) > 0.1 * np.linalg.norm(ex)
