"""Pins for the oracle's emission linearisation and MH step (CPU only).

* v_t, Lambda_t vs central finite differences of log h_t (every family);
* the stochastic-volatility log h_t vs scipy's normal log-density, the
  multivariate-t log h_t vs scipy's multivariate-t log-density;
* the linearised potential plus the auxiliary Gaussian equals the pseudo-
  observation Gaussian up to a constant in z (eq. gaussian-FK-proposal,
  eq. second-order), and order 2 is exact for Gaussian emissions;
* log r vs a dense brute-force evaluation of the Hastings ratio on the
  augmented target pi(x, u) with the proposal density computed by conditioning
  the full joint Gaussian (no Kalman recursion);
* acceptance exactly 1 for linear-Gaussian emissions under order 2 (the
  linear-Gaussian tiny workload, 100 steps);
* a long oracle chain on N = 2, d = 1 non-Gaussian models reproduces the
  posterior mean and second moment computed by 2-D quadrature;
* the factorised step (dx one-dimensional filters and samplers) equals the
  dense step on models whose prior and Omega_t are diagonal, and refuses the
  models that do not factorise.
"""
import numpy as np
import pytest

import oracle
from paper_2303_00301_amd import workloads as W
from tests.oracle_util import fd_grad, mvn_logpdf, prior_moments


def _model(emit, dx, rng, dy=None):
    G = rng.standard_normal((dx, dx))
    F = 0.7 * G / np.max(np.abs(np.linalg.eigvals(G)))
    A = rng.standard_normal((dx, dx))
    Q = A @ A.T / dx + 0.2 * np.eye(dx)
    kw = dict(m0=rng.standard_normal(dx) * 0.2, P0=np.eye(dx), F=F, Q=Q, emit=emit,
              b=0.1 * rng.standard_normal(dx))
    if emit == oracle.EMIT_GAUSSIAN:
        dy = dy or dx
        C = rng.standard_normal((dy, dy))
        kw.update(H=rng.standard_normal((dy, dx)), R=C @ C.T / dy + 0.3 * np.eye(dy))
    elif emit in (oracle.EMIT_POISSON_LOG, oracle.EMIT_STOCH_VOL):
        dy = dy or dx
        kw.update(site=rng.integers(0, dx, size=dy).astype(np.int32))
    elif emit == oracle.EMIT_MVT:
        dy = dy or dx
        C = rng.standard_normal((dy, dy))
        kw.update(site=rng.integers(0, dx, size=dy).astype(np.int32), nu=2.5,
                  R=C @ C.T / dy + 0.5 * np.eye(dy))
    else:
        dy = dy or dx
        kw.update(site=rng.integers(0, dx, size=dy).astype(np.int32), nu=3.0, scale=0.5)
    return oracle.Model(**kw), dy


def _y(M, dy, N, rng):
    if M.emit == oracle.EMIT_POISSON_LOG:
        return rng.poisson(1.5, size=(N, dy)).astype(float)
    return rng.standard_normal((N, dy))


@pytest.mark.parametrize("emit", [0, 1, 2, 3, 4])
def test_emission_gradient_hessian_fd(emit):
    rng = np.random.default_rng(10 + emit)
    for dx in (1, 3, 5):
        M, dy = _model(emit, dx, rng, dy=dx + 1)
        yt = _y(M, dy, 1, rng)[0]
        xt = 0.5 * rng.standard_normal(dx)
        lh, v, Lam = oracle.emission(M, yt, xt)
        f = lambda z: oracle.emission(M, yt, z)[0]
        g = fd_grad(f, xt, 1e-5)
        np.testing.assert_allclose(v, g, rtol=1e-7, atol=1e-7)
        Hs = np.stack([fd_grad(lambda z: oracle.emission(M, yt, z)[1][i], xt, 1e-5)
                       for i in range(dx)])
        np.testing.assert_allclose(Lam, Hs, rtol=1e-6, atol=1e-6)


def test_stoch_vol_log_h_is_normal_log_density():
    """Stochastic volatility: log h = sum_k log N(y_k; 0, exp(x_site[k])) up to the
    constant -dy log(2 pi)/2 (scipy's normal log-density as the reference)."""
    from scipy.stats import norm
    rng = np.random.default_rng(77)
    for dx, dy in ((1, 1), (4, 6), (30, 30)):
        M, _ = _model(oracle.EMIT_STOCH_VOL, dx, rng, dy=dy)
        for _ in range(3):
            yt = 2.0 * rng.standard_normal(dy)
            xt = 1.5 * rng.standard_normal(dx)
            lh = oracle.emission(M, yt, xt)[0]
            ref = norm.logpdf(yt, 0.0, np.exp(0.5 * xt[M.site])).sum() + 0.5 * dy * np.log(2 * np.pi)
            assert abs(lh - ref) < 1e-10 * max(1.0, abs(ref))


def test_mvt_log_h_is_multivariate_t_log_density():
    """Multivariate t with precision R: log h(y | x) equals scipy's multivariate-t
    log-density of y - x[site] (shape R^-1, nu degrees of freedom) plus the
    dropped constant -log G((nu + p)/2) + log G(nu/2) + (p/2) log(nu pi) - (1/2) logdet R."""
    from scipy.special import gammaln
    from scipy.stats import multivariate_t
    rng = np.random.default_rng(78)
    for dx, dy in ((1, 1), (4, 6), (16, 16)):
        M, _ = _model(oracle.EMIT_MVT, dx, rng, dy=dy)
        const = (-gammaln(0.5 * (M.nu + dy)) + gammaln(0.5 * M.nu) + 0.5 * dy * np.log(M.nu * np.pi)
                 - 0.5 * np.linalg.slogdet(M.R)[1])
        for _ in range(3):
            yt = 2.0 * rng.standard_normal(dy)
            xt = 1.5 * rng.standard_normal(dx)
            lh = oracle.emission(M, yt, xt)[0]
            ref = multivariate_t(loc=xt[M.site], shape=np.linalg.inv(M.R), df=M.nu).logpdf(yt)
            assert abs(lh - (ref + const)) < 1e-10 * max(1.0, abs(ref))


def test_lattice_precision():
    """tau^D for Manhattan distance D <= 1 on the 8 x 8 lattice: unit diagonal,
    tau for the 2-4 lattice neighbours, zero elsewhere, symmetric positive definite."""
    R = W.lattice_precision(8, -0.25, 1)
    assert np.array_equal(np.diag(R), np.ones(64))
    off = R - np.eye(64)
    assert np.array_equal(R, R.T)
    nnz = (off != 0).sum(1)
    assert nnz.min() == 2 and nnz.max() == 4 and nnz.sum() == 2 * 2 * 8 * 7
    assert set(np.unique(off)) == {0.0, -0.25}
    assert R[0, 1] == -0.25 and R[0, 8] == -0.25 and R[0, 9] == 0.0 and R[7, 8] == 0.0
    assert np.linalg.eigvalsh(R).min() > 0.0


@pytest.mark.parametrize("emit,order", [(0, 1), (0, 2), (1, 1), (1, 2), (2, 1), (2, 2), (3, 1),
                                        (3, 2), (4, 1), (4, 2)])
def test_linearised_proposal_is_pseudo_observation_gaussian(emit, order):
    """vᵀ(z-x) + ½(z-x)ᵀΛ(z-x) + log N(u; z, δ/2 I) - log N(ω; z, Ω) is constant in z."""
    rng = np.random.default_rng(20 + emit)
    dx, N, delta = 3, 1, 0.4
    M, dy = _model(emit, dx, rng)
    y = _y(M, dy, N, rng)
    x = 0.3 * rng.standard_normal((N, dx))
    u = x + np.sqrt(delta / 2) * rng.standard_normal((N, dx))
    om, Om, _, rc = oracle.linearise(M, y, x, u, delta, order)
    assert rc == 0
    _, v, Lam = oracle.emission(M, y[0], x[0])
    if order == 1:
        Lam = 0 * Lam
        np.testing.assert_allclose(Om[0], delta / 2 * np.eye(dx), atol=1e-14)
    vals = []
    for _ in range(5):
        z = rng.standard_normal(dx)
        dz = z - x[0]
        lin = v @ dz + 0.5 * dz @ Lam @ dz
        vals.append(lin + mvn_logpdf(u[0], z, delta / 2 * np.eye(dx)) - mvn_logpdf(om[0], z, Om[0]))
    assert np.ptp(vals) < 1e-9


def test_second_order_exact_for_gaussian_emissions():
    """log h(y|z) + log N(u; z, δ/2) - log N(ω; z, Ω) is constant in z, and (ω, Ω)
    do not depend on the linearisation point."""
    rng = np.random.default_rng(3)
    M, dy = _model(0, 3, rng, dy=2)
    y = _y(M, dy, 1, rng)
    delta = 0.7
    u = rng.standard_normal((1, 3))
    om1, Om1, _, _ = oracle.linearise(M, y, rng.standard_normal((1, 3)), u, delta, 2)
    om2, Om2, _, _ = oracle.linearise(M, y, rng.standard_normal((1, 3)), u, delta, 2)
    np.testing.assert_allclose(om1, om2, atol=1e-12)
    np.testing.assert_allclose(Om1, Om2, atol=1e-12)
    vals = [oracle.emission(M, y[0], z)[0] + mvn_logpdf(u[0], z, delta / 2 * np.eye(3))
            - mvn_logpdf(om1[0], z, Om1[0]) for z in rng.standard_normal((4, 3))]
    assert np.ptp(vals) < 1e-9


def _brute_log_ratio(M, y, x, xs, u, delta, order):
    """log [pi(x*, u) q(x | u, x*)] - log [pi(x, u) q(x* | u, x)] by dense algebra."""
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


@pytest.mark.parametrize("emit,order,N,dx", [(0, 1, 4, 2), (0, 2, 3, 2), (1, 1, 5, 1), (1, 2, 4, 2),
                                             (2, 1, 3, 3), (2, 2, 5, 2), (3, 1, 4, 2),
                                             (3, 2, 3, 3), (4, 1, 3, 3), (4, 2, 4, 2)])
def test_log_ratio_vs_dense_brute_force(emit, order, N, dx):
    rng = np.random.default_rng(40 + 3 * emit + order)
    M, dy = _model(emit, dx, rng)
    y = _y(M, dy, N, rng)
    x = 0.3 * rng.standard_normal((N, dx))
    delta = 0.3
    xi_u, xi_x = rng.standard_normal((2, N, dx))
    r = oracle.mh_step(M, y, x, delta, order, xi_u, xi_x, 0.5)
    assert r["status"] == 0
    u = x + np.sqrt(delta / 2) * xi_u
    ref = _brute_log_ratio(M, y, x, r["xstar"], u, delta, order)
    assert abs(r["log_ratio"] - ref) < 1e-8 * max(1.0, abs(ref))
    # the forward log Z is the Gaussian marginal of the pseudo-observations
    om, Om, _, _ = oracle.linearise(M, y, x, u, delta, order)
    mu, S = prior_moments(N, M.m0, M.P0, M.F, M.Q, M.b)
    Ob = np.zeros((N * dx, N * dx))
    for t in range(N):
        Ob[t * dx:(t + 1) * dx, t * dx:(t + 1) * dx] = Om[t]
    assert abs(r["logZ_fwd"] - mvn_logpdf(om.ravel(), mu, S + Ob)) < 1e-9


def test_acceptance_is_one_for_linear_gaussian_order2():
    w = W.linear_gaussian_tiny()
    M = oracle.Model(**w.oracle_kwargs())
    xi = w.normals(100)
    un = w.uniforms(100)
    r = oracle.mh_chain(M, w.y, w.x_init(), w.delta, 2, xi, un)
    assert (r["status"] == 0).all()
    assert np.abs(r["log_ratio"]).max() < 1e-9
    assert r["accepted"].all()


def test_first_order_is_not_exact_for_gaussian():
    """Sanity: the first-order proposal leaves a non-zero log ratio."""
    w = W.linear_gaussian_tiny()
    M = oracle.Model(**w.oracle_kwargs())
    xi = w.normals(5)
    r = oracle.mh_chain(M, w.y, w.x_init(), w.delta, 1, xi, w.uniforms(5))
    assert np.abs(r["log_ratio"]).max() > 1e-3


def test_swap_negates_log_ratio():
    """Swapping the roles of x and x* (same u) negates log r (Hastings ratio)."""
    rng = np.random.default_rng(9)
    M, dy = _model(2, 2, rng)
    N, delta = 6, 0.5
    y = _y(M, dy, N, rng)
    x = 0.2 * rng.standard_normal((N, 2))
    xi_u, xi_x = rng.standard_normal((2, N, 2))
    r = oracle.mh_step(M, y, x, delta, 2, xi_u, xi_x, 0.5)
    u = x + np.sqrt(delta / 2) * xi_u
    xs = r["xstar"]
    f = _brute_log_ratio(M, y, x, xs, u, delta, 2)
    b = _brute_log_ratio(M, y, xs, x, u, delta, 2)
    assert abs(f + b) < 1e-9
    assert abs(r["log_ratio"] - f) < 1e-8


def _quadrature_posterior(M, y, lim=8.0, n=801):
    g = np.linspace(-lim, lim, n)
    X0, X1 = np.meshgrid(g, g, indexing="ij")
    q = M.Q[0, 0]
    lp = -0.5 * (X0 - M.m0[0]) ** 2 / M.P0[0, 0] - 0.5 * (X1 - M.F[0, 0] * X0 - M.b[0]) ** 2 / q
    for t, X in ((0, X0), (1, X1)):
        if M.emit == oracle.EMIT_POISSON_LOG:
            lp = lp + y[t, 0] * X - np.exp(X)
        elif M.emit == oracle.EMIT_STOCH_VOL:
            from scipy.stats import norm
            lp = lp + norm.logpdf(y[t, 0], 0.0, np.exp(0.5 * X))
        elif M.emit == oracle.EMIT_MVT:
            lp = lp - 0.5 * (M.nu + 1) * np.log1p((y[t, 0] - X) ** 2 * M.R[0, 0] / M.nu)
        else:
            a = M.nu * M.scale ** 2
            lp = lp - 0.5 * (M.nu + 1) * np.log1p((y[t, 0] - X) ** 2 / a)
    w = np.exp(lp - lp.max())
    w /= w.sum()
    return np.array([(w * X0).sum(), (w * X1).sum(), (w * X0 ** 2).sum(), (w * X1 ** 2).sum()])


@pytest.mark.parametrize("emit,order,delta,factorised", [(1, 2, 1.5, False), (2, 2, 2.0, False),
                                                       (2, 1, 1.0, False), (3, 2, 1.5, False),
                                                       (4, 1, 1.0, True), (1, 2, 1.5, True)])
def test_long_chain_matches_quadrature(emit, order, delta, factorised):
    """N = 2, d = 1: a 4e5-step chain must reproduce the posterior moments of
    (x_0, x_1) within 5 batch-means standard errors; a wrong Hastings ratio
    biases the chain's stationary law.  The factorised chains run the
    one-dimensional filter/sampler step."""
    kw = dict(m0=np.array([0.2]), P0=np.array([[1.0]]), F=np.array([[0.6]]),
              Q=np.array([[0.5]]), emit=emit, b=np.array([0.1]), site=np.array([0], np.int32))
    if emit == oracle.EMIT_STUDENT_T:
        kw.update(nu=3.0, scale=0.5)
        y = np.array([[2.5], [-1.0]])
    elif emit == oracle.EMIT_STOCH_VOL:
        y = np.array([[2.0], [0.3]])
    elif emit == oracle.EMIT_MVT:
        kw.update(nu=1.0, R=np.array([[2.0]]))
        y = np.array([[2.5], [-1.0]])
    else:
        y = np.array([[4.0], [0.0]])
    M = oracle.Model(**kw)
    ref = _quadrature_posterior(M, y)
    n = 400_000
    rng = np.random.default_rng(1234 + emit + order)
    xi = rng.standard_normal((n, 2, 2, 1))
    un = rng.random(n)
    r = oracle.mh_chain(M, y, np.zeros((2, 1)), delta, order, xi, un, factorised=factorised)
    s = r["samples"][:, :, 0]
    acc = r["accepted"].mean()
    assert 0.1 < acc < 0.99
    f = np.concatenate([s, s ** 2], axis=1)[n // 20:]
    nb = 200
    bm = f[: (len(f) // nb) * nb].reshape(nb, -1, 4).mean(1)
    se = bm.std(0, ddof=1) / np.sqrt(nb)
    z = (f.mean(0) - ref) / se
    assert np.abs(z).max() < 5.0, (z, f.mean(0), ref)


def _diagonal_model(emit, dx, rng, dy=None):
    M, dy = _model(emit, dx, rng, dy=dy)
    M.F = np.diag(rng.uniform(0.5, 1.0, dx))
    M.Q = np.diag(rng.uniform(0.2, 1.0, dx))
    M.P0 = np.diag(rng.uniform(0.5, 1.5, dx))
    return M, dy


@pytest.mark.parametrize("emit,order", [(1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1)])
def test_factorised_step_equals_dense_step(emit, order):
    """Diagonal P0, F, Q and diagonal Omega_t: dx one-dimensional filters and
    samplers give the dense step's x*, log Z and log r (three chained steps)."""
    rng = np.random.default_rng(60 + 2 * emit + order)
    dx, N, delta = 5, 7, 0.3
    M, dy = _diagonal_model(emit, dx, rng, dy=6)
    y = _y(M, dy, N, rng)
    x = 0.3 * rng.standard_normal((N, dx))
    for k in range(3):
        xi_u, xi_x = rng.standard_normal((2, N, dx))
        un = rng.random()
        a = oracle.mh_step(M, y, x, delta, order, xi_u, xi_x, un)
        b = oracle.mh_step_factorised(M, y, x, delta, order, xi_u, xi_x, un)
        assert a["status"] == 0 and b["status"] == 0
        np.testing.assert_allclose(b["xstar"], a["xstar"], rtol=0, atol=1e-12)
        for key in ("log_ratio", "logZ_fwd", "logZ_rev"):
            assert abs(a[key] - b[key]) < 1e-10 * max(1.0, abs(a[key])), key
        assert a["accepted"] == b["accepted"]
        x = a["x_out"]


def test_factorised_step_refuses_coupled_models():
    rng = np.random.default_rng(66)
    N, dx, delta = 4, 3, 0.3
    M, dy = _diagonal_model(oracle.EMIT_MVT, dx, rng)
    y = _y(M, dy, N, rng)
    x = 0.3 * rng.standard_normal((N, dx))
    xi_u, xi_x = rng.standard_normal((2, N, dx))
    # order 2: the multivariate-t Hessian couples the coordinates
    assert oracle.mh_step_factorised(M, y, x, delta, 2, xi_u, xi_x, 0.5)["status"] == -1
    M2, _ = _diagonal_model(oracle.EMIT_POISSON_LOG, dx, rng)
    M2.F[0, 1] = 0.1
    assert oracle.mh_step_factorised(M2, _y(M2, dx, N, rng), x, delta, 1, xi_u, xi_x,
                                     0.5)["status"] == -1
