"""Pins for the oracle's Kalman filter, RTS sampler and smoother (CPU only).

* dense joint-Gaussian brute force for log p(y_{0:T}) and the smoothing
  marginals at T <= 8 (App. A, eq. smoothing-app);
* sequential vs associative-scan orderings of the filter and the sampler,
  including pathwise equality of samples under shared noise (Prop.
  "prefix-sum sampling");
* FFBS sample moments vs the RTS smoother over 1e5 draws;
* the two-step AR(rho) failure-mode model (Sec. "Failure modes"), whose
  posterior of x_0 is available in closed form.
"""
import numpy as np
import pytest

import oracle
from oracle import scan_ops
from tests.oracle_util import dense_lgssm


def _random_lgssm(rng, N, dx, dy, per_t_R=False, bias=True):
    G = rng.standard_normal((dx, dx))
    F = 0.8 * G / np.max(np.abs(np.linalg.eigvals(G)))
    A = rng.standard_normal((dx, dx))
    Q = A @ A.T / dx + 0.1 * np.eye(dx)
    B = rng.standard_normal((dx, dx))
    P0 = B @ B.T / dx + 0.5 * np.eye(dx)
    m0 = rng.standard_normal(dx)
    b = rng.standard_normal(dx) * 0.3 if bias else None
    H = rng.standard_normal((dy, dx))
    if per_t_R:
        R = []
        for _ in range(N):
            C = rng.standard_normal((dy, dy))
            R.append(C @ C.T / dy + 0.2 * np.eye(dy))
        R = np.stack(R)
    else:
        C = rng.standard_normal((dy, dy))
        R = C @ C.T / dy + 0.2 * np.eye(dy)
    y = rng.standard_normal((N, dy))
    return m0, P0, F, b, Q, H, R, y


@pytest.mark.parametrize("seed,N,dx,dy,per_t", [(0, 1, 1, 1, False), (1, 5, 2, 1, False),
                                                 (2, 8, 3, 2, True), (3, 7, 2, 3, True),
                                                 (4, 8, 4, 4, False)])
def test_kf_and_smoother_vs_dense_joint_gaussian(seed, N, dx, dy, per_t):
    rng = np.random.default_rng(seed)
    m0, P0, F, b, Q, H, R, y = _random_lgssm(rng, N, dx, dy, per_t_R=per_t)
    out = oracle.kf(m0, P0, F, Q, H, R, y, b=b, R_per_t=per_t)
    assert out["rc"] == 0
    R_list = [R[t] if per_t else R for t in range(N)]
    ll, ms_ref, Ps_ref, _, _ = dense_lgssm(N, m0, P0, F, Q, [H] * N, R_list, y, b=b)
    assert abs(out["logZ"] - ll) < 1e-10 * max(1.0, abs(ll))
    ms, Ps, G, rc = oracle.rts_smooth(F, out["mf"], out["Pf"], out["mp"], out["Pp"])
    assert rc == 0
    np.testing.assert_allclose(ms, ms_ref, atol=1e-10, rtol=1e-10)
    np.testing.assert_allclose(Ps, Ps_ref, atol=1e-10, rtol=1e-10)
    # the last filtering marginal is the last smoothing marginal
    np.testing.assert_allclose(out["mf"][-1], ms_ref[-1], atol=1e-10)


@pytest.mark.parametrize("seed,N,dx", [(21, 1, 2), (22, 6, 3), (23, 5, 1)])
def test_kf_sampler_time_varying_dynamics_vs_dense(seed, N, dx):
    """Per-step F_t, b_t (the linearised dynamics of nonlinear models): log p(y)
    and smoothing marginals from the filter and smoother, and the pathwise
    sampler's law: with zero noise it returns the smoothing mean, and the
    columns of its noise map L (one sample per unit vector) give L L^T = the
    posterior covariance of the whole path."""
    rng = np.random.default_rng(seed)
    m0, P0, _, _, Q, H, R, y = _random_lgssm(rng, N, dx, 2)
    Fs = np.stack([0.9 * np.linalg.qr(rng.standard_normal((dx, dx)))[0] for _ in range(N)])
    bs = 0.3 * rng.standard_normal((N, dx))
    out = oracle.kf(m0, P0, Fs, Q, H, R, y, b=bs)
    assert out["rc"] == 0
    ll, ms_ref, Ps_ref, pm, pc = dense_lgssm(N, m0, P0, Fs, Q, [H] * N, [R] * N, y, b=bs)
    assert abs(out["logZ"] - ll) < 1e-10 * max(1.0, abs(ll))
    ms, Ps, _, rc = oracle.rts_smooth(Fs, out["mf"], out["Pf"], out["mp"], out["Pp"])
    assert rc == 0
    np.testing.assert_allclose(ms, ms_ref, atol=1e-10, rtol=1e-10)
    np.testing.assert_allclose(Ps, Ps_ref, atol=1e-10, rtol=1e-10)
    x0, rc = oracle.rts_sample(Fs, out["mf"], out["Pf"], out["mp"], out["Pp"], np.zeros((N, dx)))
    assert rc == 0
    np.testing.assert_allclose(x0.ravel(), pm, atol=1e-10)
    Lmap = np.zeros((N * dx, N * dx))
    for k in range(N * dx):
        e = np.zeros(N * dx)
        e[k] = 1.0
        xk, _ = oracle.rts_sample(Fs, out["mf"], out["Pf"], out["mp"], out["Pp"], e.reshape(N, dx))
        Lmap[:, k] = xk.ravel() - x0.ravel()
    np.testing.assert_allclose(Lmap @ Lmap.T, pc, atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_element_normalisers_give_log_likelihood(seed):
    """Elements carrying log c (the normaliser of p(y | x_prev)): under any
    bracketing the prefix's log c equals the sequential filter's
    sum_{s <= t} ell_s, and a single element's log c is a plain Gaussian log
    density."""
    rng = np.random.default_rng(300 + seed)
    N, dx, dy = 9, 3, 2
    m0, P0, F, b, Q, H, R, y = _random_lgssm(rng, N, dx, dy)
    out = oracle.kf(m0, P0, F, Q, H, R, y, b=b)
    cum = np.cumsum(out["ell"])
    el = scan_ops.filter_elements(m0, P0, F, b, Q, H, R, y)
    lc = scan_ops.filter_log_norms(m0, P0, F, b, Q, H, R, y)
    assert abs(lc[0] - out["ell"][0]) < 1e-12
    from tests.oracle_util import mvn_logpdf
    assert abs(lc[3] - mvn_logpdf(y[3], H @ b, H @ Q @ H.T + R)) < 1e-12
    pairs = list(zip(el, lc))

    def op(a, c):
        return (scan_ops.filter_combine(a[0], c[0]),
                scan_ops.filter_combine_log_norm(a[0], a[1], c[0], c[1]))

    for pref in (scan_ops.scan_fold(pairs, op), scan_ops.scan_random_tree(pairs, op, rng),
                 scan_ops.scan_random_tree(pairs, op, rng)):
        np.testing.assert_allclose([p[1] for p in pref], cum, rtol=1e-11, atol=1e-11)
    # a sign error in the quadratic term is detected
    def bad(a, c):
        _, bi, Ci, _, _ = a[0]
        _, _, _, ej_, Jj = c[0]
        v = ej_ - Jj @ bi
        Z = np.eye(dx) + Ci @ Jj
        good = scan_ops.filter_combine_log_norm(a[0], a[1], c[0], c[1])
        return (scan_ops.filter_combine(a[0], c[0]), good - v @ np.linalg.solve(Z, Ci @ v))
    wrong = scan_ops.scan_fold(pairs, bad)
    assert np.abs(np.array([p[1] for p in wrong]) - cum).max() > 1e-3


@pytest.mark.parametrize("seed,N,dx,tv", [(31, 1, 2, False), (32, 2, 2, True), (33, 3, 1, False),
                                          (34, 6, 3, True), (35, 9, 2, False), (36, 12, 2, True)])
def test_dnc_sampler_law_vs_dense(seed, N, dx, tv):
    """Divide-and-conquer sampler (App. A, divide-and-conquer strategies): with
    zero noise it returns the posterior mean, and its noise map L satisfies
    L L^T = the posterior covariance of the whole path (dense conditioning), so
    it draws from the same law as the RTS sampler, on bisection trees of
    several shapes (N = 1, 2, 3, 6, 9, 12)."""
    rng = np.random.default_rng(seed)
    m0, P0, F, b, Q, H, R, y = _random_lgssm(rng, N, dx, 2)
    if tv:
        F = np.stack([0.9 * np.linalg.qr(rng.standard_normal((dx, dx)))[0] for _ in range(N)])
        b = 0.3 * rng.standard_normal((N, dx))
    out = oracle.kf(m0, P0, F, Q, H, R, y, b=b)
    assert out["rc"] == 0
    _, _, _, pm, pc = dense_lgssm(N, m0, P0, F, Q, [H] * N, [R] * N, y, b=b)
    x0, rc = oracle.dnc_sample(F, Q, out["mf"], out["Pf"], np.zeros((N, dx)), b=b)
    assert rc == 0
    np.testing.assert_allclose(x0.ravel(), pm, atol=1e-10)
    Lmap = np.zeros((N * dx, N * dx))
    for k in range(N * dx):
        e = np.zeros(N * dx)
        e[k] = 1.0
        xk, _ = oracle.dnc_sample(F, Q, out["mf"], out["Pf"], e.reshape(N, dx), b=b)
        Lmap[:, k] = xk.ravel() - x0.ravel()
    np.testing.assert_allclose(Lmap @ Lmap.T, pc, atol=1e-10)
    # a different noise map from the RTS sampler: the paths differ for the same normals
    if N >= 3:
        xi = rng.standard_normal((N, dx))
        xa, _ = oracle.dnc_sample(F, Q, out["mf"], out["Pf"], xi, b=b)
        xb, _ = oracle.rts_sample(F, out["mf"], out["Pf"], out["mp"], out["Pp"], xi)
        assert np.abs(xa - xb).max() > 1e-6


def test_kf_time_varying_H_vs_dense():
    rng = np.random.default_rng(11)
    N, dx, dy = 6, 3, 2
    m0, P0, F, b, Q, _, R, y = _random_lgssm(rng, N, dx, dy, per_t_R=True)
    Hs = rng.standard_normal((N, dy, dx))
    out = oracle.kf(m0, P0, F, Q, Hs, R, y, b=b, H_per_t=True, R_per_t=True)
    ll, ms_ref, _, _, _ = dense_lgssm(N, m0, P0, F, Q, list(Hs), list(R), y, b=b)
    assert abs(out["logZ"] - ll) < 1e-10 * abs(ll)


def test_lag_one_covariance_vs_dense():
    """Cov(x_{t+1}, x_t | y) = P^s_{t+1} G_t^T (used by the Fisher score)."""
    rng = np.random.default_rng(5)
    N, dx, dy = 6, 3, 2
    m0, P0, F, b, Q, H, R, y = _random_lgssm(rng, N, dx, dy)
    out = oracle.kf(m0, P0, F, Q, H, R, y, b=b)
    ms, Ps, G, _ = oracle.rts_smooth(F, out["mf"], out["Pf"], out["mp"], out["Pp"])
    _, _, _, _, pc = dense_lgssm(N, m0, P0, F, Q, [H] * N, [R] * N, y, b=b)
    for t in range(N - 1):
        ref = pc[(t + 1) * dx:(t + 2) * dx, t * dx:(t + 1) * dx]
        np.testing.assert_allclose(Ps[t + 1] @ G[t].T, ref, atol=1e-10)


@pytest.mark.parametrize("seed", range(6))
def test_filter_scan_orderings_match_sequential(seed):
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(1, 40))
    dx = int(rng.integers(1, 6))
    dy = int(rng.integers(1, 5))
    m0, P0, F, b, Q, H, R, y = _random_lgssm(rng, N, dx, dy, per_t_R=bool(seed % 2))
    out = oracle.kf(m0, P0, F, Q, H, R, y, b=b, R_per_t=bool(seed % 2))
    el = scan_ops.filter_elements(m0, P0, F, b, Q, H, R, y)
    for pref in (scan_ops.scan_fold(el, scan_ops.filter_combine),
                 scan_ops.scan_random_tree(el, scan_ops.filter_combine, rng),
                 scan_ops.scan_random_tree(el, scan_ops.filter_combine, rng)):
        for t in range(N):
            A, bb, Cm, eta, J = pref[t]
            np.testing.assert_allclose(A, 0.0, atol=1e-12)
            np.testing.assert_allclose(J, 0.0, atol=1e-12)
            np.testing.assert_allclose(eta, 0.0, atol=1e-12)
            np.testing.assert_allclose(bb, out["mf"][t], atol=1e-9, rtol=1e-9)
            np.testing.assert_allclose(Cm, out["Pf"][t], atol=1e-9, rtol=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_filter_operator_is_associative(seed):
    rng = np.random.default_rng(200 + seed)
    dx, dy, N = 3, 2, 6
    m0, P0, F, b, Q, H, R, y = _random_lgssm(rng, N, dx, dy, per_t_R=True)
    el = scan_ops.filter_elements(m0, P0, F, b, Q, H, R, y)
    a, bb, c = el[1], el[2], el[3]
    op = scan_ops.filter_combine
    lhs, rhs = op(op(a, bb), c), op(a, op(bb, c))
    for u, v in zip(lhs, rhs):
        np.testing.assert_allclose(u, v, atol=1e-10, rtol=1e-10)
    # a planted mistake (transposed Z) must break associativity or the fold
    def bad(ei, ej):
        Ai, bi, Ci, ei_, Ji = ei
        Aj, bj, Cj, ej_, Jj = ej
        Z = np.eye(dx) + Jj @ Ci
        Cm = Aj @ np.linalg.solve(Z, Ci) @ Aj.T + Cj
        return (Aj @ np.linalg.solve(Z, Ai), Aj @ np.linalg.solve(Z, bi + Ci @ ej_) + bj, Cm,
                Ai.T @ np.linalg.solve(Z.T, ej_ - Jj @ bi) + ei_,
                Ai.T @ np.linalg.solve(Z.T, Jj) @ Ai + Ji)
    out = oracle.kf(m0, P0, F, Q, H, R, y, b=b, R_per_t=True)
    pref = scan_ops.scan_fold(el, bad)
    assert max(np.abs(pref[t][1] - out["mf"][t]).max() for t in range(N)) > 1e-6


@pytest.mark.parametrize("seed", range(6))
def test_sampler_scan_matches_rts_smoother_and_pathwise_sampler(seed):
    rng = np.random.default_rng(300 + seed)
    N = int(rng.integers(1, 40))
    dx = int(rng.integers(1, 6))
    dy = int(rng.integers(1, 4))
    m0, P0, F, b, Q, H, R, y = _random_lgssm(rng, N, dx, dy)
    out = oracle.kf(m0, P0, F, Q, H, R, y, b=b)
    ms, Ps, _, _ = oracle.rts_smooth(F, out["mf"], out["Pf"], out["mp"], out["Pp"])
    se = scan_ops.sampling_elements(F, out["mf"], out["Pf"], out["mp"], out["Pp"])
    for scan in (scan_ops.scan_fold, lambda e, op: scan_ops.scan_random_tree(e, op, rng)):
        suf = scan_ops.suffix_scan(se, scan_ops.sampling_combine, scan)
        for t in range(N):
            np.testing.assert_allclose(suf[t][0], 0.0, atol=1e-12)
            np.testing.assert_allclose(suf[t][1], ms[t], atol=1e-9, rtol=1e-9)
            np.testing.assert_allclose(suf[t][2], Ps[t], atol=1e-9, rtol=1e-9)
    xi = rng.standard_normal((N, dx))
    x_seq, rc = oracle.rts_sample(F, out["mf"], out["Pf"], out["mp"], out["Pp"], xi)
    assert rc == 0
    pe = scan_ops.path_elements(se, xi)
    suf = scan_ops.suffix_scan(pe, scan_ops.path_combine,
                               lambda e, op: scan_ops.scan_random_tree(e, op, rng))
    x_par = np.stack([u for (_, u) in suf])
    np.testing.assert_allclose(x_par, x_seq, atol=1e-9, rtol=1e-9)


def test_ffbs_moments_match_rts_smoother():
    """1e5 pathwise draws: per-coordinate mean, variance and lag-one covariance
    within 5 Monte-Carlo standard errors (Bonferroni over all checks)."""
    rng = np.random.default_rng(7)
    N, dx, dy = 12, 2, 1
    m0, P0, F, b, Q, H, R, y = _random_lgssm(rng, N, dx, dy)
    out = oracle.kf(m0, P0, F, Q, H, R, y, b=b)
    ms, Ps, G, _ = oracle.rts_smooth(F, out["mf"], out["Pf"], out["mp"], out["Pp"])
    M = 100_000
    xi = rng.standard_normal((M, N, dx))
    X = np.empty((M, N, dx))
    for k in range(M):
        X[k], rc = oracle.rts_sample(F, out["mf"], out["Pf"], out["mp"], out["Pp"], xi[k])
    mean = X.mean(0)
    var = X.var(0)
    sd = np.sqrt(np.einsum("tii->ti", Ps))
    z_mean = (mean - ms) / (sd / np.sqrt(M))
    # Var of the sample variance of a Gaussian: 2 s^4 / M
    z_var = (var - sd ** 2) / (np.sqrt(2.0 / M) * sd ** 2)
    lag = np.einsum("kti,ktj->tij", X[:, 1:] - ms[1:], X[:, :-1] - ms[:-1]) / M
    lag_ref = np.stack([Ps[t + 1] @ G[t].T for t in range(N - 1)])
    sd_lag = np.sqrt((np.einsum("tii->ti", Ps)[1:, :, None] * np.einsum("tii->ti", Ps)[:-1, None, :]
                      + lag_ref ** 2) / M)
    z_lag = (lag - lag_ref) / sd_lag
    n_checks = z_mean.size + z_var.size + z_lag.size
    from scipy.stats import norm
    thr = norm.isf(0.001 / n_checks / 2)
    assert np.abs(z_mean).max() < thr
    assert np.abs(z_var).max() < thr
    assert np.abs(z_lag).max() < thr


@pytest.mark.parametrize("rho,r2", [(0.0, 1.0), (0.5, 0.1), (0.9, 0.001), (0.999, 0.5)])
def test_two_step_ar_closed_form(rho, r2):
    """x_0 ~ N(0,1), x_1 = rho x_0 + N(0, 1-rho^2), y = x_1 + N(0, r^2), y = 5
    observed at the second step only: x_0 | y ~ N(5 rho/(1+r^2), 1 - rho^2/(1+r^2))."""
    y = np.array([[0.0], [5.0]])
    Hs = np.array([[[0.0]], [[1.0]]])
    Rs = np.array([[[1.0]], [[r2]]])
    F = np.array([[rho]])
    Q = np.array([[1 - rho ** 2]]) if rho < 1 else np.array([[1e-12]])
    out = oracle.kf(np.zeros(1), np.eye(1), F, Q, Hs, Rs, y, H_per_t=True, R_per_t=True)
    ms, Ps, _, rc = oracle.rts_smooth(F, out["mf"], out["Pf"], out["mp"], out["Pp"])
    m0 = rho * 5 / (1 + r2)
    s0 = 1 - rho ** 2 / (1 + r2)
    assert abs(ms[0, 0] - m0) < 1e-12
    assert abs(Ps[0, 0, 0] - s0) < 1e-12
    # log p(y_1) = log N(5; 0, 1 + r^2); the H=0 step contributes log N(0; 0, 1)
    ll1 = -0.5 * (np.log(2 * np.pi * (1 + r2)) + 25 / (1 + r2))
    assert abs(out["ell"][1] - ll1) < 1e-12
    assert abs(out["ell"][0] + 0.5 * np.log(2 * np.pi)) < 1e-14
