"""Plain FP64 CPU oracle of the ISAM system operator, its adjoint, the proximal
steps and FISTA, for model-based iterative reconstruction (MBIR) of
spectral-domain OCT (Mason et al., "Model-based iterative reconstruction for
spectral-domain optical coherence tomography").

TEST INFRASTRUCTURE.  This module is the oracle: only the test suite, the smoke
check and the benchmark's CPU-baseline leg may import it.  The HIP library never
calls it and it never calls the HIP library.  It is written for a reader who
checks it against the paper by eye: NumPy / SciPy in complex128 / float64, no
blocking, fusion or reordering beyond what the paper's definitions state.

What the paper fixes and what is a reading (every reading is also listed in the
design notes of the repository):

* Objective, fidelity and gradient: Sec. 2.1, eq. (1)-(3).
* Phi = diag(s) Re{ diag(e^{j Omega}) D Q K x }: Sec. 2.1, eq. (4)-(9).
  Reading: the N_z depth samples have pitch dz = pi / (2 N_z dk), so that
  D Q (zero-pad to 2N, 2N-point DFT) evaluated at the spectrometer wavenumbers
  k_m equals a sum over depth with phase e^{-j 2 k_m z_n}; the ISAM resampling
  of eq. (5) and the D Q chain then collapse into one non-uniform transform
  evaluated at beta_m(q) = sqrt(4 k_m^2 - q^2) for each lateral frequency q.
  At q = 0 this is literally the paper's D Q (pinned in the tests).
* The NUFFT with Kaiser-Bessel interpolation (Sec. 2.1, citing Fessler and
  Sutton): J-tap interpolation from a sigma-times oversampled FFT grid,
  centred at n_c = floor(N_z/2).  Reading: a zero-edge KB kernel
  psi0(u) = (I0(b sqrt(1-(2u/J)^2)) - 1) / (I0(b) - 1) with the Beatty et al.
  shape b = pi sqrt(J^2/sigma^2 (sigma-1/2)^2 - 0.8), and deapodisation by its
  continuous Fourier transform (closed form below, pinned against quadrature).
* Filter (Sec. 2.1, eq. (5), not given by the paper): beam(q) = e^{-q^2 w0^2/8},
  focus phase e^{-j 2 k z_f} e^{j beta (z_f - n_c dz)}, dispersion e^{j Omega},
  zero for evanescent components (4 k^2 <= q^2).
* Omega (eq. (9)) in pixel units: Omega_m = a (m-m_c)^2 + b (m-m_c)^3,
  m_c = (M_k-1)/2.
* The adjoint is the exact transpose of Phi under <a,b> = Re(a^H b); the
  paper's Hilbert-transform backward operator (eq. (10)-(11)) is provided
  separately (``paper_backward``, and its literal single-A-scan chain
  ``paper_backward_nx1``), with a FISTA and a power iteration that use it.
* Regularisers (Sec. 2.2, eq. (12)-(14)): l1 (Psi = I), isotropic TV (complex,
  Neumann forward differences, FGP inner solver with a fixed inner count and a
  warm-started dual), 3-level orthonormal Haar on the detail bands, and the
  2-D DT-CWT (B-scans) with filters designed by Selesnick's common-factor
  method, since the paper does not give its filter banks.  The constraint set
  C of eq. (16) is read as a per-pixel modulus bound (l1 and TV).
* Operator models: 0, the NUFFT evaluated at every detector wavenumber; 1, the
  paper's literal K, Q, D chain (M_k = 2 N_z).
* FISTA (Sec. 2.3, eq. (15)-(16)) with x^1 = x0, z^0 = x^1, t^1 = 1; returns
  z^K.  Step 1/(1.05 L) with L from a 50-step power iteration on Phi^H Phi
  whose start vector comes from the SplitMix64 counter generator.

Array layouts (match the library's): images (B, N_y, N_x, N_z) complex,
measurements (B, N_y, N_x, M_k) real, mask (N_y, N_x, M_k) shared by the batch.
A B-scan has N_y = 1.
"""
from __future__ import annotations

from dataclasses import dataclass, replace
import itertools
import math

import numpy as np
import scipy.fft as sfft
from scipy.special import i0

__all__ = [
    "Geometry", "kb_beta_default", "kb_kernel", "kb_kernel_standard",
    "kb_deapod", "kb_deapod_standard", "derived", "q_squared", "k_grid",
    "omega", "beta_t", "filter_H", "nufft_cols_forward", "nufft_cols_adjoint",
    "literal_cols_forward", "literal_cols_adjoint", "columns_forward", "columns_adjoint",
    "img_shape", "meas_shape", "forward", "adjoint", "grad", "data_loss", "project_box", "prox_l1", "tv_grad", "tv_div",
    "tv_dual_gap",
    "prox_tv", "tv_value", "haar_forward", "haar_inverse", "haar_detail_mask",
    "prox_haar", "haar_value", "penalty_value", "splitmix64", "counter_uniform",
    "power_start", "lipschitz", "step_size", "fista_momenta", "fista",
    "lambda_max", "set_workers", "get_workers", "paper_backward_nx1", "paper_backward", "adjoint_complex", "ncc", "direct_axial", "direct_isam", "interp_fill",
    "interp_isam", "PEN_L1", "PEN_TV", "PEN_HAAR", "PEN_DTCWT",
    "maxflat_halfband_factor", "dtcwt_filters", "dtcwt_combination", "dtcwt_forward", "dtcwt_inverse", "prox_dtcwt", "dtcwt_value",
]

PEN_L1, PEN_TV, PEN_HAAR, PEN_DTCWT = 0, 1, 2, 3


# ----------------------------------------------------------------------------
# Geometry (Sec. 2.1; Sec. 3.1 for the optics)
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class Geometry:
    """Problem statement of Sec. 2.1: image x in C^N (N_z depth x N_x [x N_y]
    lateral), measurements y in R^M (M_k spectral pixels per A-scan)."""
    n_depth: int
    n_x: int
    n_k: int
    n_y: int = 1
    lateral_dims: int = 1
    batch: int = 1
    k_min: float = 2.0 * math.pi / 0.9     # rad/um
    k_max: float = 2.0 * math.pi / 0.75    # rad/um
    dx: float = 2.0                        # um
    dy: float = 2.0                        # um
    dz: float = 0.0                        # <= 0: pi / (2 N_z dk)
    z_focus: float = -1.0                  # < 0: n_c dz
    beam_waist: float = 5.0                # w0 (1/e^2 intensity radius); <= 0: no beam filter
    disp_a: float = 1e-3                   # rad / px^2
    disp_b: float = 0.0                    # rad / px^3
    kb_width: int = 6                      # J
    oversamp: float = 2.0                  # sigma
    kb_beta: float = 0.0                   # <= 0: Beatty closed form
    model: int = 0                         # 0: NUFFT at every detector wavenumber; 1: literal K, Q, D chain

    def with_(self, **kw) -> "Geometry":
        return replace(self, **kw)


def kb_beta_default(J: int, sigma: float) -> float:
    """KB shape parameter of Beatty, Nishimura and Pauly (2005)."""
    return math.pi * math.sqrt(J * J / (sigma * sigma) * (sigma - 0.5) ** 2 - 0.8)


@dataclass(frozen=True)
class Derived:
    dk: float
    dz: float
    n_c: int
    K: int
    z_f: float
    kb_b: float
    J: int


def derived(g: Geometry) -> Derived:
    dk = (g.k_max - g.k_min) / (g.n_k - 1)
    dz = g.dz if g.dz > 0 else math.pi / (2.0 * g.n_depth * dk)
    n_c = g.n_depth // 2
    Kf = g.oversamp * g.n_depth
    K = int(round(Kf))
    if abs(K - Kf) > 1e-9:
        raise ValueError("sigma * N_z must be an integer")
    z_f = g.z_focus if g.z_focus >= 0 else n_c * dz
    b = g.kb_beta if g.kb_beta > 0 else kb_beta_default(g.kb_width, g.oversamp)
    return Derived(dk=dk, dz=dz, n_c=n_c, K=K, z_f=z_f, kb_b=b, J=g.kb_width)


def k_grid(g: Geometry) -> np.ndarray:
    """Detected wavenumbers, linear in k with inclusive endpoints."""
    return np.linspace(g.k_min, g.k_max, g.n_k)


def omega(g: Geometry) -> np.ndarray:
    """Dispersion phase of eq. (9), in spectral-pixel units about the band centre."""
    m = np.arange(g.n_k, dtype=np.float64)
    u = m - (g.n_k - 1) / 2.0
    return g.disp_a * u * u + g.disp_b * u * u * u


def q_squared(g: Geometry) -> np.ndarray:
    """|q|^2 of every lateral frequency, shape (N_y, N_x); q = 2 pi fftfreq(N, pitch)."""
    qx = 2.0 * np.pi * np.fft.fftfreq(g.n_x, d=g.dx)
    if g.lateral_dims == 2:
        qy = 2.0 * np.pi * np.fft.fftfreq(g.n_y, d=g.dy)
    else:
        qy = np.zeros(1)
    return qy[:, None] ** 2 + qx[None, :] ** 2


# ----------------------------------------------------------------------------
# Kaiser-Bessel interpolation kernel and its Fourier transform (Sec. 2.1)
# ----------------------------------------------------------------------------
def kb_kernel_standard(u, J: int, b: float):
    """Standard KB window I0(b sqrt(1 - (2u/J)^2)) on |u| <= J/2."""
    u = np.asarray(u, dtype=np.float64)
    s = 1.0 - (2.0 * u / J) ** 2
    out = np.where(s >= 0.0, i0(b * np.sqrt(np.clip(s, 0.0, None))), 0.0)
    return out


def kb_kernel(u, J: int, b: float):
    """Zero-edge KB window psi0(u) = (I0(b sqrt(1-(2u/J)^2)) - 1) / (I0(b) - 1),
    |u| <= J/2, zero outside.  It vanishes at the window edge."""
    u = np.asarray(u, dtype=np.float64)
    s = 1.0 - (2.0 * u / J) ** 2
    val = (i0(b * np.sqrt(np.clip(s, 0.0, None))) - 1.0) / (i0(b) - 1.0)
    return np.where(s >= 0.0, val, 0.0)


def _sinhc_term(w, J: int, b: float):
    """J sinh(sqrt(b^2 - w^2)) / sqrt(b^2 - w^2), continued as J sin(.)/(.) for w > b."""
    w = np.asarray(w, dtype=np.float64)
    a2 = b * b - w * w
    out = np.empty_like(w)
    pos = a2 > 0
    a = np.sqrt(np.abs(a2))
    with np.errstate(invalid="ignore", divide="ignore"):
        out[pos] = J * np.sinh(a[pos]) / a[pos]
        neg = a2 < 0
        out[neg] = J * np.sin(a[neg]) / a[neg]
    out[a2 == 0] = J
    return out


def kb_deapod_standard(f, J: int, b: float):
    """Continuous FT int psi(u) e^{-j 2 pi f u} du of the standard KB window."""
    w = np.pi * J * np.asarray(f, dtype=np.float64)
    return _sinhc_term(w, J, b)


def kb_deapod(f, J: int, b: float):
    """Continuous FT of the zero-edge window: [J sinh(a)/a - J sin(w)/w] / (I0(b)-1),
    a = sqrt(b^2 - w^2), w = pi J f."""
    w = np.pi * J * np.asarray(f, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        box = np.where(w == 0.0, float(J), J * np.sin(w) / np.where(w == 0.0, 1.0, w))
    return (_sinhc_term(w, J, b) - box) / (i0(b) - 1.0)


# ----------------------------------------------------------------------------
# ISAM resampling coordinates and filter (Sec. 2.1, eq. (5), (9))
# ----------------------------------------------------------------------------
def beta_t(g: Geometry, q2: np.ndarray):
    """beta_m(q) = sqrt(4 k_m^2 - q^2) and its oversampled-grid coordinate
    t_m(q) = K beta dz / (2 pi).  Shapes (C, M_k); evanescent entries are NaN."""
    d = derived(g)
    k = k_grid(g)
    arg = 4.0 * k[None, :] ** 2 - np.asarray(q2, dtype=np.float64)[:, None]
    prop = arg > 0.0
    beta = np.where(prop, np.sqrt(np.where(prop, arg, 1.0)), np.nan)
    t = d.K * beta * d.dz / (2.0 * np.pi)
    return beta, t, prop


def filter_H(g: Geometry, q2: np.ndarray) -> np.ndarray:
    """Filter of eq. (5) with the focus, beam and dispersion phases (shape (C, M_k))."""
    d = derived(g)
    k = k_grid(g)
    beta, _, prop = beta_t(g, q2)
    q2 = np.asarray(q2, dtype=np.float64)
    if g.beam_waist > 0:
        beam = np.exp(-q2 * g.beam_waist ** 2 / 8.0)
    else:
        beam = np.ones_like(q2)
    phase = -2.0 * k[None, :] * d.z_f + omega(g)[None, :] \
        + np.where(prop, beta, 0.0) * (d.z_f - d.n_c * d.dz)
    H = beam[:, None] * np.exp(1j * phase)
    return np.where(prop, H, 0.0)


# ----------------------------------------------------------------------------
# Per-column NUFFT (type 2) and its exact adjoint (Sec. 2.1, eq. (5)-(6))
# ----------------------------------------------------------------------------
def _taps(t: np.ndarray, J: int):
    """Integer tap cells floor(t) - J/2 + 1 + j, j = 0..J-1 (shape (..., J))."""
    base = np.floor(t) - J // 2 + 1
    return base[..., None] + np.arange(J)


def nufft_cols_forward(cols: np.ndarray, q2: np.ndarray, g: Geometry,
                       exact: bool = False, centered: bool = True) -> np.ndarray:
    """U[c, m] ~= sum_n cols[c, n] e^{-j beta_m(q_c) dz (n - n_c)}, then W = H U.

    KB mode: deapodise, place n' = n - n_c at n' mod K of a zero K-grid,
    K-point FFT, J-tap zero-edge KB interpolation at t_m(q).  Exact mode: the
    plain non-uniform DFT (brute force).  ``centered=False`` drops the centring
    (used only as a negative control in the tests)."""
    d = derived(g)
    nz = g.n_depth
    nc = d.n_c if centered else 0
    beta, t, prop = beta_t(g, q2)
    n = np.arange(nz)
    if exact:
        ph = np.exp(-1j * np.where(prop, beta, 0.0)[:, :, None] * d.dz * (n - nc)[None, None, :])
        U = np.einsum("cmn,cn->cm", ph, cols)
    else:
        nprime = n - nc
        grid = np.zeros((cols.shape[0], d.K), dtype=np.complex128)
        grid[:, nprime % d.K] = cols / kb_deapod(nprime / d.K, d.J, d.kb_b)[None, :]
        G = sfft.fft(grid, axis=1)
        tt = np.where(prop, t, 0.0)
        cells = _taps(tt, d.J)                               # (C, M, J)
        w = kb_kernel(tt[..., None] - cells, d.J, d.kb_b)    # (C, M, J)
        idx = (cells.astype(np.int64)) % d.K
        Gc = np.take_along_axis(G[:, None, :], idx.reshape(cols.shape[0], 1, -1), axis=2)
        Gc = Gc.reshape(idx.shape)
        U = np.sum(w * Gc, axis=2)
    return filter_H(g, q2) * U


def _even_geometry(g: Geometry) -> Geometry:
    """The N even detector wavenumbers k_{2j} = k_min + 2 j dk, j < N, with the
    depth pitch, focus and window of g and no dispersion phase."""
    d = derived(g)
    n = g.n_depth
    return g.with_(n_k=n, k_max=g.k_min + 2.0 * (n - 1) * d.dk, dz=d.dz, z_focus=d.z_f,
                   disp_a=0.0, disp_b=0.0, model=0)


def _check_literal(g: Geometry):
    if g.n_k != 2 * g.n_depth:
        raise ValueError("the literal chain has M_k = 2 N_z (Q pads N to 2N, D is 2N x 2N)")


def literal_cols_forward(cols: np.ndarray, q2: np.ndarray, g: Geometry, exact: bool = False) -> np.ndarray:
    """The paper's literal chain per lateral frequency, eq. (4)-(9):
    K: the filtered spectrum f^ . x^(q, beta) sampled at the N wavenumbers of
    the even detector pixels (the same KB NUFFT, or the plain NUDFT in exact
    mode), u = K x its N-point inverse DFT; Q pads u with N zeros; D is the
    2N-point DFT; then the dispersion phase e^{j Omega} of all 2N pixels.
    Reading: with D Q reproducing the K samples at the even pixels, K samples
    the N even wavenumbers; the odd pixels are the trigonometric interpolation
    that D Q implies (exact at q = 0, where beta = 2k is linear in k)."""
    _check_literal(g)
    n = g.n_depth
    uh = nufft_cols_forward(cols, q2, _even_geometry(g), exact=exact)      # (C, N)
    u = sfft.ifft(uh, axis=1)
    pad = np.zeros((cols.shape[0], 2 * n), dtype=np.complex128)
    pad[:, :n] = u
    return np.exp(1j * omega(g))[None, :] * sfft.fft(pad, axis=1)


def literal_cols_adjoint(rows: np.ndarray, q2: np.ndarray, g: Geometry, exact: bool = False) -> np.ndarray:
    """Exact adjoint of ``literal_cols_forward``: e^{-j Omega}, D^H (2N ifft x 2N),
    Q^T (first N), the adjoint of the N-point inverse DFT (fft / N), then the
    adjoint NUFFT at the even wavenumbers."""
    _check_literal(g)
    n = g.n_depth
    w = np.exp(-1j * omega(g))[None, :] * np.asarray(rows, dtype=np.complex128)
    u = (sfft.ifft(w, axis=1) * (2 * n))[:, :n]
    uh = sfft.fft(u, axis=1) / n
    return nufft_cols_adjoint(uh, q2, _even_geometry(g), exact=exact)


def columns_forward(cols, q2, g: Geometry, exact: bool = False):
    """Per-lateral-frequency part of the model: the direct NUFFT at every
    detector wavenumber (model 0) or the literal chain (model 1)."""
    if g.model == 1:
        return literal_cols_forward(cols, q2, g, exact=exact)
    return nufft_cols_forward(cols, q2, g, exact=exact)


def columns_adjoint(rows, q2, g: Geometry, exact: bool = False):
    if g.model == 1:
        return literal_cols_adjoint(rows, q2, g, exact=exact)
    return nufft_cols_adjoint(rows, q2, g, exact=exact)


def nufft_cols_adjoint(rows: np.ndarray, q2: np.ndarray, g: Geometry,
                       exact: bool = False) -> np.ndarray:
    """Exact adjoint of ``nufft_cols_forward``: (C, M_k) -> (C, N_z)."""
    d = derived(g)
    nz = g.n_depth
    beta, t, prop = beta_t(g, q2)
    Uh = np.conj(filter_H(g, q2)) * rows
    n = np.arange(nz)
    if exact:
        ph = np.exp(1j * np.where(prop, beta, 0.0)[:, :, None] * d.dz * (n - d.n_c)[None, None, :])
        return np.einsum("cmn,cm->cn", ph, Uh)
    C = rows.shape[0]
    tt = np.where(prop, t, 0.0)
    cells = _taps(tt, d.J)
    w = kb_kernel(tt[..., None] - cells, d.J, d.kb_b) * prop[..., None]
    idx = (cells.astype(np.int64)) % d.K + (np.arange(C) * d.K)[:, None, None]
    contrib = w * Uh[..., None]
    flat = idx.reshape(-1)
    Gh = (np.bincount(flat, weights=contrib.real.reshape(-1), minlength=C * d.K)
          + 1j * np.bincount(flat, weights=contrib.imag.reshape(-1), minlength=C * d.K))
    Gh = Gh.reshape(C, d.K)
    gh = sfft.ifft(Gh, axis=1) * d.K          # unnormalised e^{+j} transform
    nprime = n - d.n_c
    return gh[:, nprime % d.K] / kb_deapod(nprime / d.K, d.J, d.kb_b)[None, :]


# ----------------------------------------------------------------------------
# Phi, its adjoint and the data-fidelity gradient (Sec. 2.1, eq. (2), (3), (7))
# ----------------------------------------------------------------------------
def _lat_axes(g: Geometry):
    return (1, 2) if g.lateral_dims == 2 else (2,)


def _n_lat(g: Geometry) -> int:
    return g.n_x * (g.n_y if g.lateral_dims == 2 else 1)


def img_shape(g: Geometry):
    return (g.batch, g.n_y if g.lateral_dims == 2 else 1, g.n_x, g.n_depth)


def meas_shape(g: Geometry):
    return (g.batch, g.n_y if g.lateral_dims == 2 else 1, g.n_x, g.n_k)


def _chunks(total: int, per: int):
    for s in range(0, total, per):
        yield s, min(total, s + per)


# Host threads for the large workloads.  With n > 1 the independent column
# chunks of forward / adjoint run concurrently (each chunk is the same code on
# its own slice, so the result is bitwise the one-thread result) and the
# lateral transforms use scipy.fft's own workers.  Default: one thread.
_WORKERS = 1


def set_workers(n: int) -> int:
    """Set the host threads of forward / adjoint; returns the previous value."""
    global _WORKERS
    prev = _WORKERS
    _WORKERS = max(1, int(n))
    return prev


def get_workers() -> int:
    return _WORKERS


def _for_chunks(total: int, per: int, body):
    """body(a, b) for every chunk [a, b) of range(total): in order on one
    thread, or spread over _WORKERS threads (bodies write disjoint slices)."""
    spans = list(_chunks(total, per))
    if _WORKERS <= 1 or len(spans) <= 1:
        for a, b in spans:
            body(a, b)
        return
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=_WORKERS) as ex:
        for f in [ex.submit(body, a, b) for a, b in spans]:
            f.result()


def forward(x: np.ndarray, g: Geometry, mask=None, exact: bool = False,
            chunk: int = 256) -> np.ndarray:
    """y = diag(s) Re{ ifft_lat( H . NUFFT_q( fft_lat(x) ) ) }  (eq. (7))."""
    x = np.asarray(x, dtype=np.complex128).reshape(img_shape(g))
    X1 = sfft.fftn(x, axes=_lat_axes(g), workers=_WORKERS)
    cols = X1.reshape(-1, g.n_depth)
    q2 = np.broadcast_to(q_squared(g)[None], img_shape(g)[:3]).reshape(-1)
    W = np.empty((cols.shape[0], g.n_k), dtype=np.complex128)

    def body(a, b):
        W[a:b] = columns_forward(cols[a:b], q2[a:b], g, exact=exact)
    _for_chunks(cols.shape[0], chunk, body)
    V = sfft.ifftn(W.reshape(meas_shape(g)), axes=_lat_axes(g), workers=_WORKERS)
    y = V.real
    if mask is not None:
        y = y * np.asarray(mask, dtype=np.float64)[None]
    return y


def adjoint(r: np.ndarray, g: Geometry, mask=None, exact: bool = False,
            chunk: int = 256) -> np.ndarray:
    """Exact adjoint of ``forward`` under <a,b> = Re(a^H b) on C^N, dot on R^M."""
    r = np.asarray(r, dtype=np.float64).reshape(meas_shape(g))
    if mask is not None:
        r = r * np.asarray(mask, dtype=np.float64)[None]
    return adjoint_complex(r.astype(np.complex128), g, exact=exact, chunk=chunk)


def adjoint_complex(R: np.ndarray, g: Geometry, exact: bool = False, chunk: int = 256) -> np.ndarray:
    """Adjoint of the model before its real part, K^H (D Q)^H diag(e^{-j Omega}),
    applied to complex spectra R (shape of the measurement)."""
    R = np.asarray(R, dtype=np.complex128).reshape(meas_shape(g))
    Rh = sfft.fftn(R, axes=_lat_axes(g), workers=_WORKERS) / _n_lat(g)
    rows = Rh.reshape(-1, g.n_k)
    q2 = np.broadcast_to(q_squared(g)[None], img_shape(g)[:3]).reshape(-1)
    X = np.empty((rows.shape[0], g.n_depth), dtype=np.complex128)

    def body(a, b):
        X[a:b] = columns_adjoint(rows[a:b], q2[a:b], g, exact=exact)
    _for_chunks(rows.shape[0], chunk, body)
    return sfft.ifftn(X.reshape(img_shape(g)), axes=_lat_axes(g), workers=_WORKERS) * _n_lat(g)


def grad(x: np.ndarray, y: np.ndarray, g: Geometry, mask=None, exact: bool = False):
    """Gradient of eq. (3): Phi^H (Phi x - y); returns (gradient, residual)."""
    y = np.asarray(y, dtype=np.float64).reshape(meas_shape(g))
    if mask is not None:
        y = y * np.asarray(mask, dtype=np.float64)[None]
    res = forward(x, g, mask, exact=exact) - y
    return adjoint(res, g, mask, exact=exact), res


def data_loss(x, y, g: Geometry, mask=None) -> float:
    """Data fidelity of eq. (2): 1/2 ||Phi x - y||^2 over the observed samples."""
    y = np.asarray(y, dtype=np.float64).reshape(meas_shape(g))
    if mask is not None:
        y = y * np.asarray(mask, dtype=np.float64)[None]
    res = forward(x, g, mask) - y
    return 0.5 * float(np.sum(res * res))


# ----------------------------------------------------------------------------
# Proximal operators (Sec. 2.2, eq. (12)-(14); Sec. 2.3, eq. (16))
# ----------------------------------------------------------------------------
def project_box(x: np.ndarray, bound=None) -> np.ndarray:
    """Projection onto the constraint set C of eq. (16).  Reading: for a complex
    image the box is a bound on each pixel's modulus, C = {x : |x_i| <= bound}
    (a disc per pixel); bound None means C = C^N."""
    x = np.asarray(x, dtype=np.complex128)
    if bound is None:
        return x.copy()
    mag = np.abs(x)
    return np.where(mag > bound, x * (bound / np.where(mag > 0, mag, 1.0)), x)


def prox_l1(v: np.ndarray, tau: float, bound=None) -> np.ndarray:
    """argmin_{x in C} 1/2 ||x - v||^2 + tau sum |x_i| for complex x (Psi = I,
    eq. (13), (16)): shrink each modulus by tau, zero when |v_i| <= tau.  With
    the modulus bound the problem stays separable and radial: the modulus is
    clip(|v_i| - tau, 0, bound), i.e. the projection of the unconstrained
    result."""
    v = np.asarray(v, dtype=np.complex128)
    mag = np.abs(v)
    scale = np.where(mag > tau, 1.0 - tau / np.where(mag > 0, mag, 1.0), 0.0)
    return project_box(v * scale, bound)


def _img_axes(g: Geometry):
    """Image axes the regularisers act on, in the (B, N_y, N_x, N_z) layout."""
    return (3, 2, 1) if g.lateral_dims == 2 else (3, 2)


def tv_grad(x: np.ndarray, axes) -> np.ndarray:
    """Forward differences along each axis, zero at the last index (Neumann)."""
    out = np.zeros((len(axes),) + x.shape, dtype=x.dtype)
    for c, ax in enumerate(axes):
        hi = [slice(None)] * x.ndim
        lo = [slice(None)] * x.ndim
        hi[ax] = slice(1, None)
        lo[ax] = slice(0, -1)
        out[c][tuple(lo)] = x[tuple(hi)] - x[tuple(lo)]
    return out


def tv_div(p: np.ndarray, axes) -> np.ndarray:
    """div = -(tv_grad)^T:  (div p)_i = p_i [i < N-1] - p_{i-1} [i > 0] per axis."""
    out = np.zeros(p.shape[1:], dtype=p.dtype)
    for c, ax in enumerate(axes):
        pc = p[c]
        n = pc.shape[ax]
        lo = [slice(None)] * pc.ndim
        lo[ax] = slice(0, n - 1)
        out[tuple(lo)] += pc[tuple(lo)]
        src = [slice(None)] * pc.ndim
        dst = [slice(None)] * pc.ndim
        src[ax] = slice(0, n - 1)
        dst[ax] = slice(1, n)
        out[tuple(dst)] -= pc[tuple(src)]
    return out


def tv_value(x: np.ndarray, axes) -> float:
    """Isotropic TV of eq. (14): sum_i sqrt(sum_c |(grad_c x)_i|^2)."""
    d = tv_grad(np.asarray(x, dtype=np.complex128), axes)
    return float(np.sum(np.sqrt(np.sum(np.abs(d) ** 2, axis=0))))


def prox_tv(v: np.ndarray, tau: float, axes, n_inner: int, p0=None, bound=None):
    """Isotropic complex TV prox by the fast gradient projection (FGP) method of
    Beck and Teboulle (2009) on the dual: x = v + tau div p,
    p <- Proj_{|p_i| <= 1}( r + 1/(4 d tau) grad(v + tau div r) ), with FISTA
    momentum on p restarted each call; p0 warm-starts the dual (its entries
    without a forward neighbour, which carry no edge, are taken as zero).
    With a constraint set C (eq. (16), modulus bound) their constrained form:
    the primal point is P_C(v + tau div p) inside every step and at the end.
    Returns (x, p)."""
    v = np.asarray(v, dtype=np.complex128)
    nd = len(axes)
    p = np.zeros((nd,) + v.shape, dtype=np.complex128) if p0 is None else np.array(p0, dtype=np.complex128)
    # the dual lives on the grid edges of the forward differences: component
    # c has no entry at the last index along axis c
    for c, ax in enumerate(axes):
        last = [slice(None)] * v.ndim
        last[ax] = -1
        p[c][tuple(last)] = 0.0
    if tau <= 0:
        return project_box(v, bound), p
    step = 1.0 / (4.0 * nd * tau)
    r = p.copy()
    t = 1.0
    for _ in range(n_inner):
        d = project_box(v + tau * tv_div(r, axes), bound)
        pn = r + step * tv_grad(d, axes)
        mag = np.sqrt(np.sum(np.abs(pn) ** 2, axis=0))
        pn = pn / np.maximum(1.0, mag)[None]
        tn = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        r = pn + ((t - 1.0) / tn) * (pn - p)
        p = pn
        t = tn
    return project_box(v + tau * tv_div(p, axes), bound), p


def tv_dual_gap(x: np.ndarray, p: np.ndarray, v: np.ndarray, tau: float, axes, bound=None) -> float:
    """Duality gap of min_{x in C} 1/2 ||x - v||^2 + tau TV(x) at the primal x and
    the dual p: with w = v + tau div p the dual value is
    1/2 ||w - P_C w||^2 - 1/2 ||w||^2 + 1/2 ||v||^2 (the inner minimum over
    x in C of the Lagrangian), the primal 1/2 ||x - v||^2 + tau TV(x)."""
    v = np.asarray(v, dtype=np.complex128)
    w = v + tau * tv_div(p, axes)
    dual = 0.5 * np.sum(np.abs(w - project_box(w, bound)) ** 2) - 0.5 * np.sum(np.abs(w) ** 2) \
        + 0.5 * np.sum(np.abs(v) ** 2)
    primal = 0.5 * np.sum(np.abs(x - v) ** 2) + tau * tv_value(x, axes)
    return float(primal - dual)


def _haar_axes_sizes(x: np.ndarray, axes):
    return [x.shape[a] for a in axes]


def haar_forward(x: np.ndarray, axes, levels: int) -> np.ndarray:
    """Orthonormal Haar Mallat pyramid over ``axes``: at each level split the
    current low band along every axis into (x_even + x_odd)/sqrt2 (first half)
    and (x_even - x_odd)/sqrt2 (second half); recurse on the all-low corner."""
    c = np.array(x, dtype=np.complex128)
    sizes = _haar_axes_sizes(c, axes)
    for lev in range(levels):
        region = [slice(None)] * c.ndim
        for a, s in zip(axes, sizes):
            region[a] = slice(0, s >> lev)
        sub = c[tuple(region)]
        for a in axes:
            ev = np.take(sub, np.arange(0, sub.shape[a], 2), axis=a)
            od = np.take(sub, np.arange(1, sub.shape[a], 2), axis=a)
            sub = np.concatenate([(ev + od) / math.sqrt(2.0), (ev - od) / math.sqrt(2.0)], axis=a)
        c[tuple(region)] = sub
    return c


def haar_inverse(c: np.ndarray, axes, levels: int) -> np.ndarray:
    """Inverse (= transpose) of ``haar_forward``."""
    x = np.array(c, dtype=np.complex128)
    sizes = _haar_axes_sizes(x, axes)
    for lev in reversed(range(levels)):
        region = [slice(None)] * x.ndim
        for a, s in zip(axes, sizes):
            region[a] = slice(0, s >> lev)
        sub = x[tuple(region)]
        for a in reversed(axes):
            h = sub.shape[a] // 2
            lo = np.take(sub, np.arange(0, h), axis=a)
            hi = np.take(sub, np.arange(h, 2 * h), axis=a)
            ev = (lo + hi) / math.sqrt(2.0)
            od = (lo - hi) / math.sqrt(2.0)
            out = np.empty_like(sub)
            idx_e = [slice(None)] * sub.ndim
            idx_o = [slice(None)] * sub.ndim
            idx_e[a] = slice(0, 2 * h, 2)
            idx_o[a] = slice(1, 2 * h, 2)
            out[tuple(idx_e)] = ev
            out[tuple(idx_o)] = od
            sub = out
        x[tuple(region)] = sub
    return x


def haar_detail_mask(shape, axes, levels: int) -> np.ndarray:
    """True on detail coefficients, False on the coarsest all-low band."""
    m = np.ones(shape, dtype=bool)
    region = [slice(None)] * len(shape)
    for a in axes:
        region[a] = slice(0, shape[a] >> levels)
    m[tuple(region)] = False
    return m


def prox_haar(v: np.ndarray, tau: float, axes, levels: int) -> np.ndarray:
    """prox of tau ||W_d x||_1 for the orthonormal Haar W: W^T soft_tau(W v) on
    the detail bands, the coarsest approximation band untouched."""
    c = haar_forward(v, axes, levels)
    dm = haar_detail_mask(c.shape, axes, levels)
    c = np.where(dm, prox_l1(c, tau), c)
    return haar_inverse(c, axes, levels)


def haar_value(x: np.ndarray, axes, levels: int) -> float:
    c = haar_forward(x, axes, levels)
    return float(np.sum(np.abs(c[haar_detail_mask(c.shape, axes, levels)])))


# ----------------------------------------------------------------------------
# Dual-tree complex wavelet transform (Sec. 2.2, the DT-CWT of Selesnick,
# Baraniuk and Kingsbury), 2-D, for B-scans
# ----------------------------------------------------------------------------
def maxflat_halfband_factor(K: int, L: int):
    """Orthonormal lowpass pair (h, g) of Selesnick's common-factor design of
    approximate Hilbert-transform pairs of wavelet bases: h = F D, g = F D~
    with D the degree-L maximally flat (Thiran) allpass denominator for a
    half-sample delay, D~(z) = z^-L D(1/z), and F = Q (1 + 1/z)^K chosen so that
    P = H(z) H(1/z) = (z + 2 + 1/z)^K D(z) D(1/z) R(z) is halfband (p(0) = 1,
    p(2n) = 0): a linear system for the symmetric R, whose minimum-phase
    spectral factor is Q.  Then g(n) is approximately h(n - 1/2).  L = 0 gives
    the Daubechies orthonormal filter with K vanishing moments.  Normalised to
    sum sqrt(2)."""
    d = np.array([(-1) ** n * math.comb(L, n)
                  * np.prod([(0.5 - L + k) / (1.5 + k) for k in range(n)]) for n in range(L + 1)])
    s = np.convolve(d, d[::-1])                         # D(z) D(1/z)
    b = np.array([1.0])
    for _ in range(K):
        b = np.convolve(b, [1.0, 2.0, 1.0])            # (z + 2 + 1/z)^K
    q0 = np.convolve(b, s)
    M = K + L - 1                                       # R(z) = sum_{|i| <= M} r_|i| z^-i
    nP = K + L + M
    cols = []
    for i in range(M + 1):
        r = np.zeros(2 * M + 1)
        r[M + i] = 1.0
        r[M - i] = 1.0
        cols.append(np.convolve(q0, r))
    A = np.array(cols).T
    rows = [nP + 2 * n for n in range((nP + 1) // 2)]
    rhs = np.zeros(len(rows))
    rhs[0] = 1.0
    coef = np.linalg.solve(A[rows], rhs)
    R = np.zeros(2 * M + 1)
    R[M] = coef[0]
    for i in range(1, M + 1):
        R[M + i] = R[M - i] = coef[i]
    roots = np.roots(R) if M > 0 else np.array([])
    f = np.real(np.poly(roots[np.abs(roots) < 1.0])) if M > 0 else np.array([1.0])
    for _ in range(K):
        f = np.convolve(f, [1.0, 1.0])
    h = np.convolve(f, d)
    g = np.convolve(f, d[::-1])
    sc = math.sqrt(2.0) / np.sum(h)
    return h * sc, g * sc


def dtcwt_filters():
    """Lowpass analysis filters of the two trees.  First level: the 6-tap
    Daubechies filter (tree a) and the same filter one sample later (tree b).
    Later levels: the 12-tap common-factor pair (K = 3, L = 3) of
    ``maxflat_halfband_factor``.  Every filter is padded to even length."""
    d1, _ = maxflat_halfband_factor(3, 0)
    first_a = np.concatenate([d1, [0.0, 0.0]])
    first_b = np.concatenate([[0.0], d1, [0.0]])
    ha, hb = maxflat_halfband_factor(3, 3)
    return {"first": (first_a, first_b), "later": (ha, hb)}


def _qmf(h):
    """Highpass of an orthonormal even-length lowpass: (-1)^k h(L-1-k)."""
    n = len(h)
    return np.array([(-1) ** k * h[n - 1 - k] for k in range(n)])


def _afb(x, h0, axis):
    """One periodic analysis step along ``axis``: lo[i] = sum_k h0[k] x[2i + k],
    hi[i] = sum_k h1[k] x[2i + k] (indices mod n)."""
    x = np.moveaxis(np.asarray(x), axis, -1)
    n = x.shape[-1]
    h1 = _qmf(h0)
    idx = (2 * np.arange(n // 2)[:, None] + np.arange(len(h0))[None, :]) % n
    seg = x[..., idx]                                   # (..., n/2, L)
    lo = np.tensordot(seg, h0, axes=([-1], [0]))
    hi = np.tensordot(seg, h1, axes=([-1], [0]))
    return np.moveaxis(lo, -1, axis), np.moveaxis(hi, -1, axis)


def _sfb(lo, hi, h0, axis):
    """Transpose (= inverse, the analysis being orthogonal) of ``_afb``."""
    lo = np.moveaxis(np.asarray(lo), axis, -1)
    hi = np.moveaxis(np.asarray(hi), axis, -1)
    m = lo.shape[-1]
    n = 2 * m
    h1 = _qmf(h0)
    out = np.zeros(lo.shape[:-1] + (n,), dtype=np.result_type(lo, hi, np.float64))
    for k in range(len(h0)):
        idx = (2 * np.arange(m) + k) % n
        np.add.at(out, (..., idx), h0[k] * lo + h1[k] * hi)
    return np.moveaxis(out, -1, axis)


def _dt_trees(d: int):
    """The 2^d trees: one filter tree (a or b) per image axis, in axis order."""
    return list(itertools.product("ab", repeat=d))


def dtcwt_combination(d: int) -> np.ndarray:
    """Orthogonal map from the 2^d tree values of one detail coefficient to the
    real and imaginary parts (rows u_0, v_0, u_1, v_1, ...) of its complex
    coefficients.  The 1-D complex wavelet is tree a + j tree b; a d-D complex
    wavelet is the product over the axes of it or of its conjugate (the first
    axis never conjugated), expanded into tree products.  2-D:
    u = (aa - s bb)/sqrt2, v = (s ab + ba)/sqrt2 for s = +1 and (with the sign
    of v flipped) s = -1.  3-D, for s_x, s_y = +-1:
    u = (aaa - s_x s_y abb - s_x bba - s_y bab)/2,
    v = (s_x aba + s_y aab + baa - s_x s_y bbb)/2 (trees named depth, x, y)."""
    idx = {"".join(t): i for i, t in enumerate(_dt_trees(d))}
    rows = []
    if d == 2:
        r = 1.0 / math.sqrt(2.0)
        for u, v in (({"aa": 1, "bb": -1}, {"ab": 1, "ba": 1}), ({"aa": 1, "bb": 1}, {"ab": 1, "ba": -1})):
            for part in (u, v):
                row = np.zeros(4)
                for k, c in part.items():
                    row[idx[k]] = c * r
                rows.append(row)
    elif d == 3:
        for sx, sy in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
            u = {"aaa": 1, "abb": -sx * sy, "bba": -sx, "bab": -sy}
            v = {"aba": sx, "aab": sy, "baa": 1, "bbb": -sx * sy}
            for part in (u, v):
                row = np.zeros(8)
                for k, c in part.items():
                    row[idx[k]] = 0.5 * c
                rows.append(row)
    else:
        raise ValueError("the DT-CWT here is 2-D or 3-D")
    return np.array(rows)


def _tree_forward(x, axes, levels, tree, F):
    """Separable orthonormal DWT of one tree (filters of tree tree[i] along
    axes[i]): per level, analysis along every axis in order; band b of a
    level has bit i (most significant first) set when it is high-pass along
    axes[i].  Returns ([details of each level: bands 1..2^d - 1], low band)."""
    pick = {"a": 0, "b": 1}
    low = x
    bands = []
    for lev in range(levels):
        key = "first" if lev == 0 else "later"
        parts = [low]
        for ax, t in zip(axes, tree):
            f = F[key][pick[t]]
            nxt = []
            for part in parts:
                lo, hi = _afb(part, f, ax)
                nxt += [lo, hi]
            parts = nxt
        bands.append(parts[1:])
        low = parts[0]
    return bands, low


def _tree_inverse(bands, low, axes, levels, tree, F):
    pick = {"a": 0, "b": 1}
    for lev in reversed(range(levels)):
        key = "first" if lev == 0 else "later"
        parts = [low] + list(bands[lev])
        for ax, t in reversed(list(zip(axes, tree))):
            f = F[key][pick[t]]
            parts = [_sfb(parts[2 * i], parts[2 * i + 1], f, ax) for i in range(len(parts) // 2)]
        low = parts[0]
    return low


def dtcwt_forward(x, axes, levels: int):
    """DT-CWT of x over axes (depth, lateral) or (depth, x, y): the 2^d
    separable trees, each scaled by 2^(-d/2), and per level and detail band
    the orthogonal combination of ``dtcwt_combination`` into the complex
    coefficients (u_k, v_k): 6 oriented subbands in 2-D, 28 in 3-D.  For a
    complex image the trees act on it linearly and a coefficient is the pair
    (u, v) of complex numbers.  Returns (details [level][band] = [(u_k, v_k)],
    lows {tree: band})."""
    F = dtcwt_filters()
    d = len(axes)
    x = np.asarray(x, dtype=np.complex128)
    trees = _dt_trees(d)
    sc = 2.0 ** (-d / 2.0)
    tr = {t: _tree_forward(sc * x, axes, levels, t, F) for t in trees}
    C = dtcwt_combination(d)
    details = []
    for lev in range(levels):
        per = []
        for b in range(2 ** d - 1):
            stack = np.stack([tr[t][0][lev][b] for t in trees])
            coef = np.tensordot(C, stack, axes=([1], [0]))
            per.append([(coef[2 * k], coef[2 * k + 1]) for k in range(len(trees) // 2)])
        details.append(per)
    lows = {t: tr[t][1] for t in trees}
    return details, lows


def dtcwt_inverse(details, lows, axes, levels: int):
    """Adjoint of ``dtcwt_forward`` (its inverse: the transform is a Parseval frame)."""
    F = dtcwt_filters()
    d = len(axes)
    trees = _dt_trees(d)
    sc = 2.0 ** (-d / 2.0)
    C = dtcwt_combination(d)
    per_tree = {t: [] for t in trees}
    for lev in range(levels):
        bands = {t: [] for t in trees}
        for b in range(2 ** d - 1):
            coef = np.stack([c for pair in details[lev][b] for c in pair])
            stack = np.tensordot(C.T, coef, axes=([1], [0]))
            for i, t in enumerate(trees):
                bands[t].append(stack[i])
        for t in trees:
            per_tree[t].append(bands[t])
    out = 0.0
    for t in trees:
        out = out + sc * _tree_inverse(per_tree[t], lows[t], axes, levels, t, F)
    return out


def _dtcwt_axes(x, axes):
    if len(axes) not in (2, 3):
        raise ValueError("the DT-CWT here is 2-D or 3-D")
    return axes


def prox_dtcwt(v, tau: float, axes, levels: int):
    """W^T soft(W v) for the DT-CWT W: every complex coefficient (u, v) of the
    detail bands shrinks its modulus sqrt(|u|^2 + |v|^2) by tau, the low bands
    are kept.  (W is a Parseval frame, not a basis: this is the usual
    shrinkage step for the DT-CWT penalty, exact for an orthonormal W.)"""
    axes = _dtcwt_axes(v, axes)
    details, lows = dtcwt_forward(v, axes, levels)
    out = []
    for per in details:
        pb = []
        for pairs in per:
            q = []
            for u, w in pairs:
                mag = np.sqrt(np.abs(u) ** 2 + np.abs(w) ** 2)
                sc = np.where(mag > tau, 1.0 - tau / np.where(mag > 0, mag, 1.0), 0.0)
                q.append((u * sc, w * sc))
            pb.append(q)
        out.append(pb)
    return dtcwt_inverse(out, lows, axes, levels)


def dtcwt_value(x, axes, levels: int) -> float:
    """||W x||_1 over the detail bands: the sum of the coefficient moduli."""
    details, _ = dtcwt_forward(x, _dtcwt_axes(x, axes), levels)
    return float(sum(np.sum(np.sqrt(np.abs(u) ** 2 + np.abs(w) ** 2))
                     for per in details for pairs in per for u, w in pairs))


def penalty_value(x: np.ndarray, g: Geometry, pen: int, haar_levels: int = 3) -> float:
    """R(x) of eq. (12) for the regularisers (haar_levels also sets the DT-CWT levels)."""
    x = np.asarray(x, dtype=np.complex128).reshape(img_shape(g))
    if pen == PEN_L1:
        return float(np.sum(np.abs(x)))
    if pen == PEN_TV:
        return tv_value(x, _img_axes(g))
    if pen == PEN_HAAR:
        return haar_value(x, _img_axes(g), haar_levels)
    if pen == PEN_DTCWT:
        return dtcwt_value(x, _img_axes(g), haar_levels)
    raise ValueError("unknown penalty")


# ----------------------------------------------------------------------------
# Step size, counter-based start vector (Sec. 2.3)
# ----------------------------------------------------------------------------
_SM_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_SM_M1 = np.uint64(0xBF58476D1CE4E5B9)
_SM_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter: np.ndarray, seed: int) -> np.ndarray:
    """SplitMix64 (Steele, Lea and Flood, 2014) as a counter-based generator:
    state = seed + (counter + 1) * golden gamma, then the published mixer."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(counter, dtype=np.uint64) + np.uint64(1)) * _SM_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _SM_M1
        z = (z ^ (z >> np.uint64(27))) * _SM_M2
        return z ^ (z >> np.uint64(31))


def counter_uniform(counter: np.ndarray, seed: int) -> np.ndarray:
    """Uniform on [-1, 1): top 53 bits of SplitMix64 scaled by 2^-52, minus 1."""
    bits = splitmix64(counter, seed) >> np.uint64(11)
    return bits.astype(np.float64) * (2.0 ** -52) - 1.0


def power_start(g: Geometry, seed: int = 0) -> np.ndarray:
    """Start vector of the power iteration: element e (flattened image index)
    has real part u(2e) and imaginary part u(2e+1)."""
    n = int(np.prod(img_shape(g)))
    e = np.arange(n, dtype=np.uint64)
    re = counter_uniform(2 * e, seed)
    im = counter_uniform(2 * e + 1, seed)
    return (re + 1j * im).reshape(img_shape(g))


def lipschitz(g: Geometry, mask=None, iters: int = 50, seed: int = 0, start=None,
              backward: str = "exact") -> float:
    """Power iteration on Phi^H Phi: x_0 = s/||s||, w = Phi^H Phi x_{i-1},
    L_i = ||w||, x_i = w / L_i; returns L_iters.  backward="paper" iterates
    the operator the paper's gradient uses, Phi* Phi with Phi* of eq. (10)-(11)
    (not self-adjoint: L_iters then tends to its spectral radius), so that the
    step size of Sec. 2.3 bounds the steps actually taken."""
    x = power_start(g, seed) if start is None else np.asarray(start, dtype=np.complex128)
    x = x / np.linalg.norm(x)
    L = 0.0
    for _ in range(iters):
        if backward == "paper":
            w = paper_backward(forward(x, g, mask), g, mask)
        else:
            w = adjoint(forward(x, g, mask), g, mask)
        L = float(np.linalg.norm(w))
        if L == 0.0:
            # the operator annihilated a random start: Phi = 0 on this mask (no
            # observed sample), so the norm is 0 and every later iterate is 0
            return 0.0
        x = w / L
    return L


def step_size(L: float) -> float:
    """delta = 1 / (1.05 L): 'appropriately small' (Sec. 2.3) with a margin for
    the power iteration's underestimate of L.  L = 0 (nothing observed) makes
    the data term constant, so every delta > 0 is admissible: delta = 1."""
    return 1.0 / (1.05 * L) if L > 0.0 else 1.0


# ----------------------------------------------------------------------------
# FISTA (Sec. 2.3, eq. (15)-(16))
# ----------------------------------------------------------------------------
def fista_momenta(iters: int) -> np.ndarray:
    """mu_k = (t_k - 1) / t_{k+1} with t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2."""
    mu = np.empty(iters)
    t = 1.0
    for k in range(iters):
        tn = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        mu[k] = (t - 1.0) / tn
        t = tn
    return mu


def fista(y, g: Geometry, mask, pen: int, lam: float, delta: float, iters: int,
          tv_inner: int = 10, haar_levels: int = 3, x0=None, backward: str = "exact", bound=None):
    """FISTA of eq. (15): z^k = prox_{lam delta R}(x^k - delta grad D(x^k)),
    t update, x^{k+1} = z^k + (t^k - 1)/t^{k+1} (z^k - z^{k-1}).
    backward="paper" takes the gradient with the paper's backward operator
    (eq. (10)-(11)) in place of the exact adjoint.  bound: the modulus bound of
    the constraint set C in the prox of eq. (16) (l1 and TV; None = C^N).
    Returns (z^K, history) with history[k] = 1/2 ||Phi x^k - y||^2 + lam R(z^k)."""
    x = np.zeros(img_shape(g), dtype=np.complex128) if x0 is None \
        else np.array(x0, dtype=np.complex128).reshape(img_shape(g))
    z_prev = x.copy()
    mu = fista_momenta(iters)
    tau = lam * delta
    p = None
    axes = _img_axes(g)
    hist = np.empty(iters)
    for k in range(iters):
        if backward == "paper":
            yy = np.asarray(y, dtype=np.float64).reshape(meas_shape(g))
            if mask is not None:
                yy = yy * np.asarray(mask, dtype=np.float64)[None]
            res = forward(x, g, mask) - yy
            gr = paper_backward(res, g, mask)
        else:
            gr, res = grad(x, y, g, mask)
        v = x - delta * gr
        if pen == PEN_L1:
            z = prox_l1(v, tau, bound)
        elif pen == PEN_TV:
            z, p = prox_tv(v, tau, axes, tv_inner, p0=p, bound=bound)
        elif pen == PEN_HAAR:
            if bound is not None:
                raise ValueError("the constrained Haar prox has no closed form")
            z = prox_haar(v, tau, axes, haar_levels)
        elif pen == PEN_DTCWT:
            if bound is not None:
                raise ValueError("the constrained DT-CWT step has no closed form")
            z = prox_dtcwt(v, tau, axes, haar_levels)
        else:
            raise ValueError("unknown penalty")
        hist[k] = 0.5 * float(np.sum(res * res)) + lam * penalty_value(z, g, pen, haar_levels)
        x = z + mu[k] * (z - z_prev)
        z_prev = z
    return z_prev, hist


def paper_backward(r: np.ndarray, g: Geometry, mask=None, exact: bool = False) -> np.ndarray:
    """The paper's backward operator, eq. (10)-(11): K^H D^H Q^T diag(e^{-j Omega})
    A(s . y) with A(z) = Re z - j H(z), the conjugate analytic signal; the
    Hilbert transform runs along the spectral axis of every A-scan (reading:
    the discrete analytic signal, FFT with the negative frequencies removed and
    the positive ones doubled)."""
    from scipy.signal import hilbert
    r = np.asarray(r, dtype=np.float64).reshape(meas_shape(g))
    if mask is not None:
        r = r * np.asarray(mask, dtype=np.float64)[None]
    return adjoint_complex(np.conj(hilbert(r, axis=-1)), g, exact=exact)


def lambda_max(y, g: Geometry, mask=None) -> float:
    """||Phi^H (s y)||_inf: the l1 weight above which x = 0 is optimal."""
    return float(np.max(np.abs(adjoint(y, g, mask))))


# ----------------------------------------------------------------------------
# The paper's own backward operator (eq. (10)-(11)), N_x = 1, exact NUDFT
# ----------------------------------------------------------------------------
def paper_backward_nx1(r: np.ndarray, g: Geometry) -> np.ndarray:
    """Phi*(y) = K^H D^H Q^T diag(e^{-j Omega}) A(s y), A(z) = Re z - j Hilbert(z),
    for a single A-scan (q = 0, beam = 1) with M_k = 2 N_z, so that D is the
    2N-point DFT.  K^H at q = 0 undoes the e^{-j 2 k_min z_n} modulation."""
    from scipy.signal import hilbert
    assert g.n_x == 1 and g.lateral_dims == 1 and g.n_k == 2 * g.n_depth
    d = derived(g)
    r = np.asarray(r, dtype=np.float64).reshape(-1)
    a = np.conj(hilbert(r))                     # Re r - j H(r)
    a = a * np.exp(-1j * omega(g))
    back = np.fft.ifft(a) * a.size              # D^H: unnormalised e^{+j}
    xq = back[: g.n_depth]                      # Q^T
    zn = np.arange(g.n_depth) * d.dz
    return xq * np.exp(1j * 2.0 * g.k_min * zn)


# ----------------------------------------------------------------------------
# Direct reconstructions (Sec. 3.1, Figure 1) and the interpolated-ISAM
# baseline of the sub-sampling study (Sec. 3.1)
# ----------------------------------------------------------------------------
def direct_axial(y, g: Geometry, mask=None, dispersion: bool = True, exact: bool = False,
                 chunk: int = 256) -> np.ndarray:
    """Per-A-scan depth transform without the ISAM resampling ("IFFT", and with
    dispersion=True "dispersion corrected" in Figure 1).

    Reading: every A-scan is taken as the lateral-frequency-zero column of the
    model (beta = 2k, no beam term, no lateral transforms), and the
    reconstruction is the adjoint of that axial model applied to s . y; with
    dispersion=False the dispersion phase Omega is left out.  In the exact mode
    this is sum_m s_m y_m e^{-j Omega_m} e^{+j 2 k_m z_n}: the paper's zero-pad
    and 2N-point inverse DFT of the (dispersion-compensated) spectrum."""
    y = np.asarray(y, dtype=np.float64).reshape(meas_shape(g))
    if mask is not None:
        y = y * np.asarray(mask, dtype=np.float64)[None]
    ga = g.with_(beam_waist=0.0) if dispersion else g.with_(beam_waist=0.0, disp_a=0.0, disp_b=0.0)
    rows = y.reshape(-1, g.n_k).astype(np.complex128)
    X = np.empty((rows.shape[0], g.n_depth), dtype=np.complex128)
    zero = np.zeros(rows.shape[0])
    for a, b in _chunks(rows.shape[0], chunk):
        X[a:b] = nufft_cols_adjoint(rows[a:b], zero[a:b], ga, exact=exact)
    return X.reshape(img_shape(g))


def direct_isam(y, g: Geometry, mask=None) -> np.ndarray:
    """ISAM reconstruction of Figure 1 (dispersion compensation and the ISAM
    resampling): the adjoint of the full model applied to s . y."""
    return adjoint(y, g, mask)


def interp_fill(y, g: Geometry, mask) -> np.ndarray:
    """Fill the unobserved spectral samples of every A-scan by linear
    interpolation in k from its observed samples (k is linear in the pixel
    index); outside the first and last observed sample the nearest observed
    value is held; an A-scan with no observed sample stays zero."""
    y = np.asarray(y, dtype=np.float64).reshape(meas_shape(g))
    m = np.broadcast_to(np.asarray(mask, dtype=bool)[None], y.shape)
    rows, mrow = y.reshape(-1, g.n_k), m.reshape(-1, g.n_k)
    out = np.zeros_like(rows)
    grid = np.arange(g.n_k, dtype=np.float64)
    for i in range(rows.shape[0]):
        obs = np.nonzero(mrow[i])[0]
        if obs.size:
            out[i] = np.interp(grid, obs.astype(np.float64), rows[i, obs])
    return out.reshape(y.shape)


def interp_isam(y, g: Geometry, mask) -> np.ndarray:
    """Baseline of the sub-sampling study: direct ISAM on the linearly
    interpolated measurements."""
    return adjoint(interp_fill(y, g, mask), g, None)


# ----------------------------------------------------------------------------
# Evaluation metric (Sec. 3.2, eq. (17))
# ----------------------------------------------------------------------------
def ncc(x, z) -> float:
    """Normalised cross-correlation of magnitudes against ground truth z."""
    a = np.abs(np.asarray(x)).ravel()
    b = np.abs(np.asarray(z)).ravel()
    a = a - a.mean()
    b = b - b.mean()
    return float(np.sum(a * b) / (np.sqrt(np.sum(a * a)) * np.sqrt(np.sum(b * b))))
