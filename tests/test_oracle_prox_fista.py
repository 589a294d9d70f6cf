"""Pins of the oracle's proximal operators, FISTA, power iteration, counter
generator and NCC against closed forms and optimality conditions (no GPU)."""
import math

import numpy as np
import pytest

import oracle as O


def cn(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# --- l1 prox (eq. (13)) -----------------------------------------------------------
def test_prox_l1_closed_form():
    v = np.array([3 + 4j, 0.5 - 0.5j, 1.0 + 0j, 0j, -2j])
    z = O.prox_l1(v, 1.0)
    assert z[0] == pytest.approx(2.4 + 3.2j, abs=1e-15)
    assert z[1] == 0 and z[2] == 0 and z[3] == 0        # |v| <= tau (tie -> 0)
    assert z[4] == pytest.approx(-1j, abs=1e-15)


def test_prox_l1_subgradient_optimality():
    rng = np.random.default_rng(1)
    v = cn(rng, 1000)
    tau = 0.9
    z = O.prox_l1(v, tau)
    on = z != 0
    # (v - z)/tau is a subgradient of sum|z|: z/|z| on the support, |.| <= 1 off it
    np.testing.assert_allclose((v[on] - z[on]) / tau, z[on] / np.abs(z[on]), atol=1e-14)
    assert np.all(np.abs(v[~on]) / tau <= 1 + 1e-15)


# --- TV prox (eq. (14)) -----------------------------------------------------------
def test_tv_value_matches_eq14_loops():
    rng = np.random.default_rng(2)
    x = cn(rng, (1, 1, 5, 4))            # (B, N_y, N_x=5 lateral, N_z=4 depth)
    tot = 0.0
    a = x[0, 0].T                        # a[i, j]: i depth, j lateral
    for i in range(a.shape[0]):
        for j in range(a.shape[1]):
            di = a[i + 1, j] - a[i, j] if i + 1 < a.shape[0] else 0.0
            dj = a[i, j + 1] - a[i, j] if j + 1 < a.shape[1] else 0.0
            tot += math.sqrt(abs(di) ** 2 + abs(dj) ** 2)
    assert O.tv_value(x, (3, 2)) == pytest.approx(tot, rel=1e-14)


@pytest.mark.parametrize("axes,shape", [((3, 2), (1, 1, 6, 5)), ((3, 2, 1), (2, 3, 4, 5))])
def test_div_is_negative_adjoint_of_grad(axes, shape):
    rng = np.random.default_rng(3)
    x = cn(rng, shape)
    p = cn(rng, (len(axes),) + shape)
    lhs = np.real(np.vdot(p, O.tv_grad(x, axes)))
    rhs = -np.real(np.vdot(O.tv_div(p, axes), x))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("along", ["depth", "lateral"])
def test_prox_tv_two_pixel_closed_form(along):
    """Two pixels: if |v1 - v2| <= 2 tau both become the mean, otherwise the
    difference shrinks by 2 tau along (v1 - v2)/|v1 - v2|."""
    shape = (1, 1, 1, 2) if along == "depth" else (1, 1, 2, 1)
    for v1, v2, tau in [(1 + 1j, 0.2 - 0.3j, 0.3), (1 + 1j, 0.8 + 0.9j, 0.3), (2.0, -1j, 0.05)]:
        v = np.array([v1, v2]).reshape(shape)
        x, _ = O.prox_tv(v, tau, (3, 2), n_inner=3000)
        x = x.ravel()
        dv = v1 - v2
        if abs(dv) <= 2 * tau:
            e = np.array([(v1 + v2) / 2, (v1 + v2) / 2])
        else:
            u = dv / abs(dv)
            e = np.array([v1 - tau * u, v2 + tau * u])
        np.testing.assert_allclose(x, e, atol=1e-9)


def test_prox_tv_constant_fixed_point_and_mean():
    rng = np.random.default_rng(4)
    c = np.full((1, 1, 7, 9), 0.3 - 0.7j)
    x, _ = O.prox_tv(c, 0.5, (3, 2), n_inner=10)
    np.testing.assert_allclose(x, c, atol=1e-15)
    v = cn(rng, (1, 1, 7, 9))
    x, _ = O.prox_tv(v, 0.4, (3, 2), n_inner=10)
    assert abs(np.sum(x) - np.sum(v)) < 1e-12 * np.sum(np.abs(v))


@pytest.mark.parametrize("axes,shape", [((3, 2), (1, 1, 8, 10)), ((3, 2, 1), (1, 4, 5, 6))])
def test_prox_tv_duality_gap_vanishes(axes, shape):
    """Primal P(x) = 1/2||x - v||^2 + tau TV(x) and dual D(p) = 1/2||v||^2 -
    1/2||v + tau div p||^2 (|p_i| <= 1) bracket the optimum; the gap of the
    FGP pair falls towards zero as the inner count grows."""
    rng = np.random.default_rng(5)
    v = cn(rng, shape)
    tau = 0.35
    gaps = []
    for n_inner in (10, 100, 2000):
        x, p = O.prox_tv(v, tau, axes, n_inner=n_inner)
        assert np.max(np.sqrt(np.sum(np.abs(p) ** 2, axis=0))) <= 1 + 1e-12
        P = 0.5 * np.sum(np.abs(x - v) ** 2) + tau * O.tv_value(x, axes)
        D = 0.5 * np.sum(np.abs(v) ** 2) - 0.5 * np.sum(np.abs(v + tau * O.tv_div(p, axes)) ** 2)
        gaps.append(P - D)
    assert gaps[0] >= -1e-12 and gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] < 1e-6 * np.sum(np.abs(v) ** 2)


def test_prox_tv_dual_lives_on_edges():
    """Dual entries with no forward neighbour never matter: junk there in the
    warm start gives the same prox and comes back zero."""
    rng = np.random.default_rng(61)
    v = cn(rng, (1, 1, 9, 7))
    p0 = cn(rng, (2, 1, 1, 9, 7)) * 0.3
    clean = p0.copy()
    clean[0][..., -1] = 0.0           # depth component at the last depth index
    clean[1][..., -1, :] = 0.0        # lateral component at the last lateral index
    x1, p1 = O.prox_tv(v, 0.3, (3, 2), 6, p0=p0)
    x2, p2 = O.prox_tv(v, 0.3, (3, 2), 6, p0=clean)
    np.testing.assert_array_equal(x1, x2)
    assert np.all(p1[0][..., -1] == 0) and np.all(p1[1][..., -1, :] == 0)


def test_prox_tv_warm_start_continues():
    """Ten inner steps from the dual of ten earlier steps are closer to the
    exact prox than ten from zero."""
    rng = np.random.default_rng(6)
    v = cn(rng, (1, 1, 12, 12))
    tau = 0.5
    xe, _ = O.prox_tv(v, tau, (3, 2), n_inner=4000)
    x1, p1 = O.prox_tv(v, tau, (3, 2), n_inner=10)
    x2, _ = O.prox_tv(v, tau, (3, 2), n_inner=10, p0=p1)
    assert np.linalg.norm(x2 - xe) < np.linalg.norm(x1 - xe)


# --- constraint set C of eq. (16): modulus bound -------------------------------------
def test_prox_l1_with_bound_brute_force():
    """argmin over the disc |x| <= c of 1/2 |x - v|^2 + tau |x|, by a polar grid
    search (modulus step 4e-4, angle step 1e-3 rad), against the closed form."""
    rng = np.random.default_rng(70)
    tau, c = 0.3, 0.8
    rho = np.linspace(0.0, c, 2001)
    th = np.linspace(-math.pi, math.pi, 6284)
    X = rho[:, None] * np.exp(1j * th[None, :])
    for v in list(cn(rng, 6) * 1.5) + [0.2 + 0.1j, 0.9 + 0.0j, 1.1j]:
        f = 0.5 * np.abs(X - v) ** 2 + tau * np.abs(X)
        i = np.unravel_index(np.argmin(f), f.shape)
        z = O.prox_l1(np.array([v]), tau, bound=c)[0]
        assert abs(z - X[i]) < 2e-3, (v, z, X[i])
        assert abs(z) <= c * (1 + 1e-15)
    # no bound, and a bound the result never reaches, are the same map
    v = cn(rng, 50)
    np.testing.assert_array_equal(O.prox_l1(v, tau), O.prox_l1(v, tau, bound=100.0))


@pytest.mark.parametrize("axes,shape", [((3, 2), (1, 1, 12, 16)), ((3, 2, 1), (1, 4, 5, 6))])
def test_prox_tv_with_bound_duality_gap_vanishes(axes, shape):
    """Constrained TV prox (FGP with P_C in every step): the duality gap of
    min_{|x_i| <= c} 1/2||x - v||^2 + tau TV(x) falls to rounding, the result is
    feasible, and projecting the unconstrained prox afterwards is not optimal
    (its gap stays large).  An inactive bound changes nothing."""
    rng = np.random.default_rng(71)
    v = cn(rng, shape) * 1.5
    tau, c = 0.3, 0.4
    gaps = []
    for n_inner in (10, 100, 3000):
        x, p = O.prox_tv(v, tau, axes, n_inner, bound=c)
        assert np.max(np.abs(x)) <= c * (1 + 1e-12)
        gaps.append(O.tv_dual_gap(x, p, v, tau, axes, bound=c))
    assert gaps[0] > gaps[1] > max(gaps[2], 0.0) - 1e-12
    assert abs(gaps[2]) < 1e-9 * np.sum(np.abs(v) ** 2)
    xu, pu = O.prox_tv(v, tau, axes, 3000)
    assert O.tv_dual_gap(O.project_box(xu, c), pu, v, tau, axes, bound=c) > 1e3 * abs(gaps[2]) + 1e-3
    big = 10.0 * np.max(np.abs(v))
    xb, pb = O.prox_tv(v, tau, axes, 20, bound=big)
    x0, p0 = O.prox_tv(v, tau, axes, 20)
    np.testing.assert_array_equal(xb, x0)


def test_fista_l1_with_bound_kkt():
    """Long-run constrained l1 FISTA on the dense problem: feasible, and the KKT
    conditions of min_{|x_i| <= c} D(x) + lam ||x||_1 hold: |g_i| <= lam at
    zeros, g_i = -lam z_i/|z_i| strictly inside the disc, and on its edge -g_i
    points along z_i with modulus >= lam."""
    g, mask, A, y = _dense_problem()
    L = np.linalg.svd(A, compute_uv=False)[0] ** 2
    delta = 1 / (1.05 * L)
    lam, c = 0.05, 0.5
    zs, _ = O.fista(y, g, mask, O.PEN_L1, lam, delta, 20000, bound=c)
    gr, _ = O.grad(zs, y, g, mask)
    mag = np.abs(zs)
    assert np.all(mag <= c * (1 + 1e-12))
    zero = mag < 1e-9
    edge = mag > c * (1 - 1e-9)
    inner = ~zero & ~edge
    assert edge.any()
    assert np.all(np.abs(gr[zero]) <= lam * (1 + 1e-6))
    np.testing.assert_allclose(gr[inner], -lam * zs[inner] / mag[inner], atol=1e-6 * lam)
    u = zs[edge] / mag[edge]
    proj = np.real(np.conj(u) * -gr[edge])           # component of -g along z
    perp = np.abs(-gr[edge] - proj * u)
    assert np.all(proj >= lam * (1 - 1e-6)) and np.all(perp <= 1e-6 * lam)


# --- Haar prox ----------------------------------------------------------------------
def test_haar_single_level_hand_example():
    a = np.array([[1.0, 2.0], [3.0, 5.0]])          # a[l, n]
    x = a.reshape(1, 1, 2, 2).astype(complex)
    c = O.haar_forward(x, (3, 2), 1)[0, 0]
    x00, x01, x10, x11 = 1.0, 2.0, 3.0, 5.0
    np.testing.assert_allclose(c, [[(x00 + x01 + x10 + x11) / 2, (x00 - x01 + x10 - x11) / 2],
                                   [(x00 + x01 - x10 - x11) / 2, (x00 - x01 - x10 + x11) / 2]],
                               atol=1e-15)


@pytest.mark.parametrize("axes,shape", [((3, 2), (1, 1, 8, 8)), ((3, 2, 1), (1, 8, 8, 8))])
def test_haar_orthonormal(axes, shape):
    n = int(np.prod(shape))
    W = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        W[:, j] = O.haar_forward(e.reshape(shape), axes, 3).real.ravel()
    np.testing.assert_allclose(W.T @ W, np.eye(n), atol=1e-14)
    rng = np.random.default_rng(8)
    x = cn(rng, shape)
    np.testing.assert_allclose(O.haar_inverse(O.haar_forward(x, axes, 3), axes, 3), x, atol=1e-14)


@pytest.mark.parametrize("axes,shape,blk", [((3, 2), (2, 1, 16, 24), (1, 1, 8, 8)),
                                            ((3, 2, 1), (1, 16, 8, 16), (1, 8, 8, 8))])
def test_haar_prox_limits(axes, shape, blk):
    """tau = 0 is the identity; a huge tau zeroes every detail band, leaving the
    mean of each 8 x 8 (x 8) block."""
    rng = np.random.default_rng(9)
    v = cn(rng, shape)
    np.testing.assert_allclose(O.prox_haar(v, 0.0, axes, 3), v, atol=1e-13)
    z = O.prox_haar(v, 1e9, axes, 3)
    r = v.reshape(shape[0], shape[1] // blk[1], blk[1], shape[2] // blk[2], blk[2],
                  shape[3] // blk[3], blk[3])
    means = r.mean(axis=(2, 4, 6), keepdims=True)
    expect = np.broadcast_to(means, r.shape).reshape(shape)
    np.testing.assert_allclose(z, expect, atol=1e-12)


def test_haar_prox_is_soft_threshold_in_coefficients():
    rng = np.random.default_rng(10)
    axes = (3, 2)
    v = cn(rng, (1, 1, 8, 16))
    tau = 0.4
    z = O.prox_haar(v, tau, axes, 3)
    cz = O.haar_forward(z, axes, 3)
    cv = O.haar_forward(v, axes, 3)
    dm = O.haar_detail_mask(cv.shape, axes, 3)
    np.testing.assert_allclose(cz[~dm], cv[~dm], atol=1e-13)
    mag = np.abs(cv[dm])
    expect = np.where(mag > tau, cv[dm] * (1 - tau / mag), 0)
    np.testing.assert_allclose(cz[dm], expect, atol=1e-13)


# --- FISTA (eq. (15)) --------------------------------------------------------------
def test_fista_momenta():
    mu = O.fista_momenta(50)
    assert mu[0] == 0.0
    t = [1.0]
    for _ in range(51):
        t.append((1 + math.sqrt(1 + 4 * t[-1] ** 2)) / 2)
    assert t[1] == pytest.approx((1 + math.sqrt(5)) / 2, abs=1e-15)
    for k in range(1, 51):
        assert t[k - 1] >= (k + 1) / 2 - 1e-12 or k == 1
    np.testing.assert_allclose(mu, [(t[k] - 1) / t[k + 1] for k in range(50)], atol=1e-15)


def _dense_problem():
    g = O.Geometry(n_depth=8, n_x=4, n_k=12)
    rng = np.random.default_rng(11)
    mask = (rng.random((1, 4, 12)) < 0.8).astype(np.uint8)
    n = int(np.prod(O.img_shape(g)))
    cols = []
    for unit in (1.0, 1j):
        for j in range(n):
            e = np.zeros(n, dtype=complex)
            e[j] = unit
            cols.append(O.forward(e.reshape(O.img_shape(g)), g, mask).ravel())
    A = np.array(cols).T
    xt = np.zeros(O.img_shape(g), dtype=complex)
    xt[0, 0, 1, 3] = 1 + 0.5j
    xt[0, 0, 3, 6] = -0.7j
    y = O.forward(xt, g, mask) + 0.01 * rng.standard_normal(O.meas_shape(g)) * mask
    return g, mask, A, y


def _dense_fista(A, y, shape, prox, delta, iters):
    n = A.shape[1] // 2
    x = np.zeros(n, dtype=complex)
    zp = x.copy()
    mu = O.fista_momenta(iters)
    for k in range(iters):
        xr = np.concatenate([x.real, x.imag])
        gr = A.T @ (A @ xr - y.ravel())
        gc = gr[:n] + 1j * gr[n:]
        z = prox((x - delta * gc).reshape(shape)).ravel()
        x = z + mu[k] * (z - zp)
        zp = z
    return zp.reshape(shape)


@pytest.mark.parametrize("pen", [O.PEN_L1, O.PEN_HAAR])
def test_fista_equals_dense_matrix_fista(pen):
    g, mask, A, y = _dense_problem()
    L = np.linalg.svd(A, compute_uv=False)[0] ** 2
    delta = 1 / (1.05 * L)
    lam = 0.05
    shape = O.img_shape(g)
    if pen == O.PEN_L1:
        prox = lambda v: O.prox_l1(v, lam * delta)       # noqa: E731
    else:
        g = g.with_(n_x=8, n_depth=8)
        rng = np.random.default_rng(12)
        mask = (rng.random((1, 8, 12)) < 0.8).astype(np.uint8)
        n = int(np.prod(O.img_shape(g)))
        A = np.array([O.forward((np.eye(n)[j] * u).reshape(O.img_shape(g)), g, mask).ravel()
                      for u in (1.0, 1j) for j in range(n)]).T
        y = (A @ rng.standard_normal(2 * n)).reshape(O.meas_shape(g))
        L = np.linalg.svd(A, compute_uv=False)[0] ** 2
        delta = 1 / (1.05 * L)
        shape = O.img_shape(g)
        prox = lambda v: O.prox_haar(v, lam * delta, (3, 2), 3)   # noqa: E731
    z, _ = O.fista(y, g, mask, pen, lam, delta, 30)
    zd = _dense_fista(A, y, shape, prox, delta, 30)
    assert np.max(np.abs(z - zd)) < 1e-12 * max(1.0, np.max(np.abs(zd)))


@pytest.mark.parametrize("pen", [O.PEN_L1, O.PEN_TV, O.PEN_HAAR])
def test_zero_weight_fista_is_the_dense_least_squares_iteration(pen):
    """lambda = 0: every penalty's prox is the identity, so the oracle's FISTA
    is the dense-matrix iteration on 1/2 ||A x - y||^2 with no prox at all."""
    g, mask, A, y = _dense_problem()
    g = g.with_(n_x=8)
    rng = np.random.default_rng(13)
    mask = (rng.random((1, 8, 12)) < 0.8).astype(np.uint8)
    n = int(np.prod(O.img_shape(g)))
    A = np.array([O.forward((np.eye(n)[j] * u).reshape(O.img_shape(g)), g, mask).ravel()
                  for u in (1.0, 1j) for j in range(n)]).T
    y = (A @ rng.standard_normal(2 * n)).reshape(O.meas_shape(g))
    delta = 1 / (1.05 * np.linalg.svd(A, compute_uv=False)[0] ** 2)
    z, _ = O.fista(y, g, mask, pen, 0.0, delta, 30, haar_levels=3)
    zd = _dense_fista(A, y, O.img_shape(g), lambda v: v, delta, 30)
    assert np.max(np.abs(z - zd)) < 1e-12 * max(1.0, np.max(np.abs(zd)))


def test_fista_l1_kkt_and_rate():
    """Long-run l1 FISTA satisfies the KKT conditions (|g_i| <= lam off the
    support, g_i = -lam z_i/|z_i| on it) and the O(1/k^2) bound of Beck and
    Teboulle: F(z_k) - F* <= 2 ||x0 - x*||^2 / (delta (k+1)^2)."""
    g, mask, A, y = _dense_problem()
    L = np.linalg.svd(A, compute_uv=False)[0] ** 2
    delta = 1 / (1.05 * L)
    lam = 0.05
    zs, _ = O.fista(y, g, mask, O.PEN_L1, lam, delta, 20000)
    gr, _ = O.grad(zs, y, g, mask)
    on = np.abs(zs) > 1e-9
    assert np.all(np.abs(gr[~on]) <= lam * (1 + 1e-6))
    np.testing.assert_allclose(gr[on], -lam * zs[on] / np.abs(zs[on]), atol=1e-6 * lam)

    def F(z):
        return O.data_loss(z, y, g, mask) + lam * np.sum(np.abs(z))
    Fs = F(zs)
    for k in (5, 20, 80):
        zk, hist = O.fista(y, g, mask, O.PEN_L1, lam, delta, k)
        assert F(zk) - Fs <= 2 * np.sum(np.abs(zs) ** 2) / (delta * (k + 1) ** 2) + 1e-12
        # history[k-1] = 1/2||Phi x^k - y||^2 + lam R(z^k)
        assert hist[-1] >= lam * np.sum(np.abs(zk)) - 1e-12


def _tv_fixed_point_error(g, mask, y, z, lam, delta):
    """How far z is from a minimiser of 1/2||Phi z - y||^2 + lam TV(z)
    (eq. (2), (14)): (1) the fixed-point residual of the FISTA map with the TV
    prox solved to 5000 inner steps, and (2) the KKT residual with the dual
    certificate p of that prox: grad D(z) = lam div p, |p_i| <= 1 and
    <p, grad z> = TV(z) (so that -div p is a subgradient of TV at z)."""
    axes = (3, 2)
    gr, _ = O.grad(z, y, g, mask)
    zp, p = O.prox_tv(z - delta * gr, lam * delta, axes, 5000)
    fp = np.linalg.norm(zp - z) / np.linalg.norm(z)
    kkt = np.linalg.norm(gr - lam * O.tv_div(p, axes)) / np.linalg.norm(gr)
    pmax = float(np.sqrt(np.sum(np.abs(p) ** 2, axis=0)).max())
    tv = O.tv_value(z, axes)
    gap = (tv - float(np.real(np.sum(np.conj(p) * O.tv_grad(z, axes))))) / tv
    return fp, kkt, pmax, gap


def test_fista_tv_converges_to_the_tv_minimiser():
    """Long-run FISTA-TV (10 warm-started inner steps) on the dense problem
    reaches the minimiser of eq. (2) + lambda TV (eq. (14)): a fixed point of
    the map with an exactly solved prox, and a KKT point with a feasible dual
    certificate."""
    g, mask, A, y = _dense_problem()
    L = np.linalg.svd(A, compute_uv=False)[0] ** 2
    delta = 1 / (1.05 * L)
    lam = 0.02
    z, _ = O.fista(y, g, mask, O.PEN_TV, lam, delta, 3000, tv_inner=10)
    fp, kkt, pmax, gap = _tv_fixed_point_error(g, mask, y, z, lam, delta)
    assert fp < 1e-8 and kkt < 1e-6
    assert pmax <= 1 + 1e-12 and abs(gap) < 1e-9


@pytest.mark.parametrize("mistake", ["tau_x2", "depth_axis_only", "no_warm_start"])
def test_fista_tv_fixed_point_catches_planted_mistakes(monkeypatch, mistake):
    """Negative controls of the pin above: the same long run with a planted
    mistake in the TV branch of the oracle's FISTA (a doubled tau, TV along
    depth only, the dual warm start dropped) is not at the minimiser."""
    import oracle.oct_oracle as OO
    real = OO.prox_tv

    def planted(v, tau, axes, n_inner, p0=None, bound=None):
        if mistake == "tau_x2":
            return real(v, 2 * tau, axes, n_inner, p0=p0, bound=bound)
        if mistake == "depth_axis_only":
            x, p = real(v, tau, axes[:1], n_inner, p0=None if p0 is None else p0[:1], bound=bound)
            return x, np.concatenate([p, np.zeros_like(p)])
        return real(v, tau, axes, n_inner, p0=None, bound=bound)
    monkeypatch.setattr(OO, "prox_tv", planted)
    g, mask, A, y = _dense_problem()
    L = np.linalg.svd(A, compute_uv=False)[0] ** 2
    delta = 1 / (1.05 * L)
    lam = 0.02
    z, _ = O.fista(y, g, mask, O.PEN_TV, lam, delta, 3000, tv_inner=10)
    monkeypatch.setattr(OO, "prox_tv", real)
    fp, kkt, _, _ = _tv_fixed_point_error(g, mask, y, z, lam, delta)
    assert fp > 1e-5 and kkt > 1e-3


def test_lambda_max_is_the_zero_solution_threshold():
    """lambda_max = ||Phi^H (s y)||_inf is the l1 weight at and above which
    x = 0 solves eq. (2) + lambda ||x||_1: FISTA from zero stays exactly zero
    at lambda_max (1 + 1e-9) and leaves it at 0.99 lambda_max.  The case is
    masked and y is nonzero on the unobserved pixels, so a threshold that
    ignored the mask would fail one of the two."""
    g = O.Geometry(n_depth=16, n_x=8, n_k=24)
    rng = np.random.default_rng(41)
    mask = (rng.random((1, 8, 24)) < 0.6).astype(np.uint8)
    y = rng.standard_normal(O.meas_shape(g))
    lmax = O.lambda_max(y, g, mask)
    assert lmax != pytest.approx(O.lambda_max(y, g, None), rel=1e-3)
    delta = O.step_size(O.lipschitz(g, mask, iters=100))
    z, _ = O.fista(y, g, mask, O.PEN_L1, lmax * (1 + 1e-9), delta, 40)
    assert np.all(z == 0)
    z, _ = O.fista(y, g, mask, O.PEN_L1, 0.99 * lmax, delta, 40)
    assert np.count_nonzero(z) > 0


@pytest.mark.parametrize("pen", ["l1", "tv", "haar"])
def test_nothing_observed_gives_zero_lipschitz_and_zero_solution(pen):
    """An all-zero mask makes Phi = 0: the power iteration's estimate of
    ||Phi^H Phi|| is exactly 0, every step size is admissible (delta = 1), and
    FISTA from zero stays exactly at zero, the minimiser of lambda R(x), for
    any weight and any (finite) measurements."""
    g = O.Geometry(n_depth=16, n_x=8, n_k=24)
    mask = np.zeros((1, 8, 24), dtype=np.uint8)
    L = O.lipschitz(g, mask, iters=5)
    assert L == 0.0
    assert O.step_size(L) == 1.0
    y = np.random.default_rng(42).standard_normal(O.meas_shape(g))
    penalty = {"l1": O.PEN_L1, "tv": O.PEN_TV, "haar": O.PEN_HAAR}[pen]
    z, _ = O.fista(y, g, mask, penalty, 0.1, O.step_size(L), 5, haar_levels=2)
    assert np.all(z == 0)


def test_fista_tv_reduces_objective():
    g, mask, A, y = _dense_problem()
    L = np.linalg.svd(A, compute_uv=False)[0] ** 2
    delta = 1 / (1.05 * L)
    lam = 0.02

    def F(z):
        return O.data_loss(z, y, g, mask) + lam * O.tv_value(z, (3, 2))
    z10, _ = O.fista(y, g, mask, O.PEN_TV, lam, delta, 10, tv_inner=50)
    z200, _ = O.fista(y, g, mask, O.PEN_TV, lam, delta, 200, tv_inner=50)
    assert F(z200) < F(z10) < F(np.zeros_like(z10))


# --- power iteration start (SplitMix64) and NCC (eq. (17)) ---------------------------
def test_splitmix64_published_sequence():
    """SplitMix64 seeded with 0 produces e220a8397b1dcdaf, 6e789e6aa1b965f4,
    06c45d188009454f, f88bb8a8724c81ec (Vigna's reference sequence)."""
    v = O.splitmix64(np.arange(4, dtype=np.uint64), 0)
    assert [int(a) for a in v] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                   0x06C45D188009454F, 0xF88BB8A8724C81EC]
    u = O.counter_uniform(np.arange(100000, dtype=np.uint64), 7)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.01


def test_ncc_closed_forms():
    rng = np.random.default_rng(13)
    z = cn(rng, 500)
    assert O.ncc(z, z) == pytest.approx(1.0, abs=1e-14)
    assert O.ncc((0.3 - 2j) * z, z) == pytest.approx(1.0, abs=1e-14)
    assert O.ncc(z * np.exp(1j * rng.uniform(0, 6, 500)), z) == pytest.approx(1.0, abs=1e-14)
    w = cn(rng, 500)
    assert -1.0 <= O.ncc(w, z) < 0.5
