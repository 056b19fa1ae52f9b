"""Pins for the oracle's observation-model linearisation (order 3: the
proposal of eq. two-lin-prop with h_t replaced by N(H_t z + c_t, R_t) from
the statistical linear regression of eq. coeffs) and for the quadratic-mean
Gaussian family (CPU only).

* the quadratic family's log h, gradient and Hessian against central
  differences;
* H, c, R recomputed from moments taken by Gauss-Hermite quadrature of the
  reference variable (no closed forms) give the oracle's v and Lambda, with
  several sites on one latent and unobserved (NaN) sites;
* at a zero reference variance the regression is the Taylor linearisation:
  v is the exact gradient of log h and Lambda the Gauss-Newton curvature, and
  a tiny reference variance is continuous with it;
* a linear observation mean makes order 3 equal to order 2 for any reference
  variance, so linear-Gaussian emissions accept every step;
* log r under order 3 against the dense brute-force Hastings ratio;
* 4e5-step chains under order 3 (Taylor and a positive reference variance)
  reproduce the posterior moments of an N = 2, d = 1 model by quadrature;
* where log h's own curvature makes the exact second-order proposal
  undefined, the regression's curvature is negative and order 3 is defined.
"""
import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss

import oracle
from tests.oracle_util import fd_grad, mvn_logpdf, prior_moments


def _quad_model(dx, site, beta, s, g2, rng):
    G = rng.standard_normal((dx, dx))
    F = 0.7 * G / np.max(np.abs(np.linalg.eigvals(G)))
    A = rng.standard_normal((dx, dx))
    Q = A @ A.T / dx + 0.2 * np.eye(dx)
    return oracle.Model(m0=rng.standard_normal(dx) * 0.2, P0=np.eye(dx), F=F, Q=Q,
                        emit=oracle.EMIT_GAUSS_QUAD, b=0.1 * rng.standard_normal(dx),
                        site=np.asarray(site, np.int32), scale=s, obs_beta=beta, slr_var=g2)


def test_quadratic_family_derivatives_vs_fd():
    rng = np.random.default_rng(1)
    M = _quad_model(3, [0, 2, 2, 1], 0.35, 0.6, 0.0, rng)
    yt = rng.standard_normal(4) + 0.5
    yt[3] = np.nan
    x = rng.standard_normal(3)
    lh, v, Lam = oracle.emission(M, yt, x)
    f = lambda z: oracle.emission(M, yt, z)[0]
    np.testing.assert_allclose(v, fd_grad(f, x, 1e-6), rtol=1e-7, atol=1e-8)
    H = np.stack([fd_grad(lambda z, j=j: oracle.emission(M, yt, z)[1][j], x, 1e-6)
                  for j in range(3)])
    np.testing.assert_allclose(Lam, H, rtol=1e-6, atol=1e-7)
    # log h is the Gaussian log density of y around the quadratic mean (less its constant)
    m = x[M.site] + 0.35 * x[M.site] ** 2
    obs = ~np.isnan(yt)
    assert abs(lh - np.sum(-0.5 * ((yt - m) / 0.6) ** 2 * obs, where=obs)) < 1e-12


def _slr_by_quadrature(M, yt, xt, n=40):
    """(v, Lambda) of N(y; H z + c, R) at z = x with H, c, R from eq. coeffs and
    the moments of eq. general-GSLR-coeffs taken by Gauss-Hermite quadrature."""
    g2 = M.slr_var
    e, w = hermegauss(n)
    w = w / w.sum()
    beta = M.obs_beta if M.emit == oracle.EMIT_GAUSS_QUAD else 0.0
    obs = [k for k in range(len(yt)) if not np.isnan(yt[k])]
    dx = len(xt)

    def mean(z):
        return z + beta * z * z

    po = len(obs)
    mu = np.zeros(po)
    C = np.zeros((po, dx))
    S = np.diag(np.full(po, M.scale ** 2))
    for a, k in enumerate(obs):
        i = M.site[k]
        z = xt[i] + np.sqrt(g2) * e
        mu[a] = w @ mean(z)
        C[a, i] = w @ ((mean(z) - mu[a]) * (z - xt[i]))
    for a, k in enumerate(obs):
        for b, l in enumerate(obs):
            i, j = M.site[k], M.site[l]
            if i == j:
                z = xt[i] + np.sqrt(g2) * e
                S[a, b] += w @ ((mean(z) - mu[a]) * (mean(z) - mu[b]))
            else:  # independent coordinates: a 2-D rule
                zi = xt[i] + np.sqrt(g2) * e[:, None]
                zj = xt[j] + np.sqrt(g2) * e[None, :]
                S[a, b] += np.sum(w[:, None] * w[None, :] * (mean(zi) - mu[a]) * (mean(zj) - mu[b]))
    Gam = g2 * np.eye(dx)
    H = C @ np.linalg.inv(Gam)
    c = mu - H @ xt
    R = S - H @ Gam @ H.T
    Ri = np.linalg.inv(R)
    yo = np.array([yt[k] for k in obs])
    return H.T @ Ri @ (yo - c - H @ xt), -H.T @ Ri @ H


@pytest.mark.parametrize("emit,beta,g2", [(oracle.EMIT_GAUSS_QUAD, 0.4, 0.3),
                                          (oracle.EMIT_GAUSS_QUAD, -0.25, 1.2),
                                          (oracle.EMIT_GAUSS_SITE, 0.0, 0.5)])
def test_regression_matches_quadrature_moments(emit, beta, g2):
    rng = np.random.default_rng(7)
    M = _quad_model(4, [0, 3, 3, 1, 0, 2], beta, 0.5, g2, rng)
    M.emit = emit
    yt = rng.standard_normal(6)
    yt[4] = np.nan
    xt = rng.standard_normal(4)
    v, Lam, rc = oracle.obs_linearise(M, yt, xt)
    assert rc == 0
    v_ref, L_ref = _slr_by_quadrature(M, yt, xt)
    np.testing.assert_allclose(v, v_ref, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(Lam, L_ref, rtol=1e-10, atol=1e-12)


def test_zero_reference_variance_is_taylor_linearisation():
    rng = np.random.default_rng(8)
    M = _quad_model(3, [0, 1, 1, 2], 0.3, 0.7, 0.0, rng)
    yt = rng.standard_normal(4)
    xt = rng.standard_normal(3)
    v, Lam, rc = oracle.obs_linearise(M, yt, xt)
    assert rc == 0
    _, v_ex, Lam_ex = oracle.emission(M, yt, xt)
    np.testing.assert_allclose(v, v_ex, rtol=1e-12, atol=1e-13)   # exact gradient
    # Gauss-Newton: -J^T R^-1 J with J the finite-difference Jacobian of the mean
    mean = lambda z: z[M.site] + 0.3 * z[M.site] ** 2
    J = np.stack([fd_grad(lambda z, k=k: mean(z)[k], xt, 1e-6) for k in range(4)])
    np.testing.assert_allclose(Lam, -J.T @ J / 0.49, rtol=1e-8, atol=1e-9)
    assert np.abs(Lam - Lam_ex).max() > 1e-3   # differs from the exact Hessian
    M.slr_var = 1e-12
    v2, Lam2, _ = oracle.obs_linearise(M, yt, xt)
    np.testing.assert_allclose(v2, v, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(Lam2, Lam, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("emit,g2", [(oracle.EMIT_GAUSS_SITE, 0.0), (oracle.EMIT_GAUSS_SITE, 0.8),
                                     (oracle.EMIT_GAUSS_QUAD, 0.8)])
def test_linear_observation_mean_gives_order2(emit, g2):
    rng = np.random.default_rng(9)
    M = _quad_model(3, [0, 2, 2], 0.0, 0.5, g2, rng)
    M.emit = emit
    N = 7
    y = rng.standard_normal((N, 3))
    y[2, 1] = np.nan
    x = rng.standard_normal((N, 3))
    u = x + 0.3 * rng.standard_normal((N, 3))
    a = oracle.linearise(M, y, x, u, 0.4, 2)
    b = oracle.linearise(M, y, x, u, 0.4, 3)
    assert a[3] == 0 and b[3] == 0
    np.testing.assert_allclose(b[0], a[0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(b[1], a[1], rtol=1e-12, atol=1e-12)
    xi = rng.standard_normal((20, 2, N, 3))
    r = oracle.mh_chain(M, y, np.zeros((N, 3)), 0.4, 3, xi, rng.random(20))
    assert r["accepted"].all() and np.abs(r["log_ratio"]).max() < 1e-9


def _brute_log_ratio(M, y, x, xs, u, delta, order):
    N, dx = x.shape
    mu, S = prior_moments(N, M.m0, M.P0, M.F, M.Q, M.b)

    def log_target(z):
        lp = mvn_logpdf(z.ravel(), mu, S)
        lp += sum(oracle.emission(M, y[t], z[t])[0] for t in range(N))
        lp += sum(mvn_logpdf(u[t], z[t], delta / 2 * np.eye(dx)) for t in range(N))
        return lp

    def log_q(z, at):
        om, Om, _, rc = oracle.linearise(M, y, at, u, delta, order)
        assert rc == 0
        Oinv = np.zeros((N * dx, N * dx))
        for t in range(N):
            Oinv[t * dx:(t + 1) * dx, t * dx:(t + 1) * dx] = np.linalg.inv(Om[t])
        Sinv = np.linalg.inv(S)
        Pc = np.linalg.inv(Sinv + Oinv)
        mc = Pc @ (Sinv @ mu + Oinv @ om.ravel())
        return mvn_logpdf(z.ravel(), mc, 0.5 * (Pc + Pc.T))

    return log_target(xs) - log_target(x) + log_q(x, xs) - log_q(xs, x)


@pytest.mark.parametrize("g2,N,dx", [(0.0, 4, 2), (0.5, 3, 3)])
def test_order3_log_ratio_vs_dense_brute_force(g2, N, dx):
    rng = np.random.default_rng(50 + N)
    M = _quad_model(dx, rng.integers(0, dx, size=dx + 1), 0.3, 0.5, g2, rng)
    y = rng.standard_normal((N, dx + 1))
    x = 0.3 * rng.standard_normal((N, dx))
    delta = 0.3
    xi_u, xi_x = rng.standard_normal((2, N, dx))
    r = oracle.mh_step(M, y, x, delta, 3, xi_u, xi_x, 0.5)
    assert r["status"] == 0
    u = x + np.sqrt(delta / 2) * xi_u
    ref = _brute_log_ratio(M, y, x, r["xstar"], u, delta, 3)
    assert abs(r["log_ratio"] - ref) < 1e-8 * max(1.0, abs(ref))


def _quadrature_posterior(M, y, lim=8.0, n=801):
    g = np.linspace(-lim, lim, n)
    X0, X1 = np.meshgrid(g, g, indexing="ij")
    lp = (-0.5 * (X0 - M.m0[0]) ** 2 / M.P0[0, 0]
          - 0.5 * (X1 - M.F[0, 0] * X0 - M.b[0]) ** 2 / M.Q[0, 0])
    for t, X in ((0, X0), (1, X1)):
        lp = lp - 0.5 * ((y[t, 0] - X - M.obs_beta * X * X) / M.scale) ** 2
    w = np.exp(lp - lp.max())
    w /= w.sum()
    return np.array([(w * X0).sum(), (w * X1).sum(), (w * X0 ** 2).sum(), (w * X1 ** 2).sum()])


@pytest.mark.parametrize("g2", [0.0, 0.3])
def test_order3_chain_matches_quadrature(g2):
    """y_t = x_t + 0.2 x_t^2 + N(0, 0.5^2) (the mean's second root lies far
    out in the prior's tail, so the posterior has one mode)."""
    M = oracle.Model(m0=np.array([0.2]), P0=np.array([[1.0]]), F=np.array([[0.6]]),
                     Q=np.array([[0.5]]), emit=oracle.EMIT_GAUSS_QUAD, b=np.array([0.1]),
                     site=np.array([0], np.int32), scale=0.5, obs_beta=0.2, slr_var=g2)
    y = np.array([[1.5], [0.4]])
    ref = _quadrature_posterior(M, y)
    n = 400_000
    rng = np.random.default_rng(4321)
    xi = rng.standard_normal((n, 2, 2, 1))
    un = rng.random(n)
    r = oracle.mh_chain(M, y, np.zeros((2, 1)), 1.0, 3, xi, un)
    assert (r["status"] == 0).all()
    s = r["samples"][:, :, 0]
    acc = r["accepted"].mean()
    assert 0.1 < acc < 0.99
    f = np.concatenate([s, s ** 2], axis=1)[n // 20:]
    nb = 200
    bm = f[: (len(f) // nb) * nb].reshape(nb, -1, 4).mean(1)
    se = bm.std(0, ddof=1) / np.sqrt(nb)
    z = (f.mean(0) - ref) / se
    assert np.abs(z).max() < 5.0, (z, f.mean(0), ref)


def test_exact_second_order_undefined_where_regression_is_not():
    """At x = 0 with y = 1.5, beta = 0.4, s = 1 the exact curvature of log h is
    (2 beta r - (1 + 2 beta x)^2) / s^2 = 0.2, above 2/delta = 1/6 for delta =
    12, so the second-order proposal is undefined; the regression's curvature
    is negative whatever the state."""
    M = oracle.Model(m0=np.zeros(1), P0=np.eye(1), F=np.array([[0.6]]), Q=np.array([[0.5]]),
                     emit=oracle.EMIT_GAUSS_QUAD, site=np.array([0], np.int32), scale=1.0,
                     obs_beta=0.4)
    y = np.array([[1.5], [1.5]])
    x = np.zeros((2, 1))
    u = x.copy()
    assert oracle.linearise(M, y, x, u, 12.0, 2)[3] != 0
    om, Om, _, rc = oracle.linearise(M, y, x, u, 12.0, 3)
    assert rc == 0 and np.all(Om[:, 0, 0] > 0)
    rng = np.random.default_rng(3)
    for g2 in (0.0, 0.7):
        M.slr_var = g2
        for _ in range(50):
            xt = 4 * rng.standard_normal(1)
            yt = 4 * rng.standard_normal(1)
            _, Lam, rc = oracle.obs_linearise(M, yt, xt)
            assert rc == 0 and Lam[0, 0] <= 0.0
