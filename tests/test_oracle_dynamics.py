"""Pins for the oracle's nonlinear dynamics and the Gaussian-at-sites emission
(CPU only).

* Lorenz-63 and Lorenz-96 Euler steps: one value by hand, the energy identity
  of their quadratic terms (sum_i x_i beta_i reduces to the linear part), and
  the Jacobian against central finite differences;
* the extended linearisation reproduces f at the linearisation point and its
  first-order change;
* log r of a step with nonlinear dynamics against a dense brute-force Hastings
  ratio: the target log pi(z, u) evaluated with the true transition density,
  the proposal density by conditioning the joint Gaussian of the linearised
  model (no Kalman recursion); swapping x and x* negates it;
* Gaussian at sites: scipy's normal density, finite differences, NaN entries
  as unobserved sites, and order-2 exactness (acceptance 1) with linear
  dynamics.
"""
import numpy as np
import pytest

import oracle
from tests.oracle_util import fd_grad, mvn_logpdf, prior_moments_tv

TH63 = (10.0, 28.0, 8.0 / 3.0, 0.01)


def _l63(**kw):
    Q = kw.pop("Q", 0.05 * np.eye(3))
    return oracle.Model(m0=np.array([1.0, -1.0, 20.0]), P0=np.eye(3), F=None, Q=Q, dyn=1,
                        dyn_par=TH63, **kw)


def _l96(d, **kw):
    A = np.random.default_rng(d).standard_normal((d, d))
    Q = kw.pop("Q", 0.02 * (A @ A.T / d + np.eye(d)))
    return oracle.Model(m0=np.zeros(d), P0=np.eye(d), F=None, Q=Q, dyn=2,
                        dyn_par=(8.0, 0.01, 0.0, 0.0), **kw)


def test_lorenz63_step_by_hand():
    M = _l63(emit=5, site=np.array([1, 2], np.int32), scale=1.0)
    f, _ = oracle.dyn(M, [1.0, 2.0, 3.0])
    # beta = (10 (2 - 1), 28 - 2 - 3, 2 - 8 (3)) = (10, 23, -6)
    np.testing.assert_allclose(f, [1.1, 2.23, 2.94], rtol=0, atol=1e-15)


@pytest.mark.parametrize("which,d", [(63, 3), (96, 4), (96, 7)])
def test_dynamics_energy_identity_and_jacobian(which, d):
    rng = np.random.default_rng(which + d)
    M = _l63(emit=5, site=np.array([0], np.int32), scale=1.0) if which == 63 else \
        _l96(d, emit=5, site=np.array([0], np.int32), scale=1.0)
    dt = TH63[3] if which == 63 else 0.01
    for _ in range(3):
        x = 3.0 * rng.standard_normal(d)
        f, J = oracle.dyn(M, x)
        beta = (f - x) / dt
        if which == 63:
            t1, t2, t3, _ = TH63
            lin = t1 * (x[1] - x[0]) * x[0] + (t2 * x[0] - x[1]) * x[1] - t3 * x[2] ** 2
        else:
            lin = -np.sum(x * x) + 8.0 * np.sum(x)
        assert abs(x @ beta - lin) < 1e-9 * max(1.0, abs(lin))
        Jfd = np.stack([fd_grad(lambda z: oracle.dyn(M, z)[0][i], x, 1e-6) for i in range(d)])
        np.testing.assert_allclose(J, Jfd, rtol=1e-7, atol=1e-7)


def test_extended_linearisation():
    rng = np.random.default_rng(3)
    M = _l96(6, emit=5, site=np.array([0], np.int32), scale=1.0)
    N = 5
    a = rng.standard_normal((N, 6))
    F, b = oracle.dyn_linearise(M, a)
    assert np.all(F[0] == 0) and np.all(b[0] == 0)
    for t in range(1, N):
        f, J = oracle.dyn(M, a[t - 1])
        np.testing.assert_allclose(F[t] @ a[t - 1] + b[t], f, atol=1e-13)
        np.testing.assert_allclose(F[t], J, atol=0)
        h = 1e-4 * rng.standard_normal(6)
        f2, _ = oracle.dyn(M, a[t - 1] + h)
        assert np.abs(F[t] @ (a[t - 1] + h) + b[t] - f2).max() < 1e-6


def _brute_log_ratio(M, y, x, xs, u, delta, order):
    N, dx = x.shape

    def log_target(z):
        lp = mvn_logpdf(z[0], M.m0, M.P0)
        for t in range(1, N):
            lp += mvn_logpdf(z[t], oracle.dyn(M, z[t - 1])[0], M.Q)
        lp += sum(oracle.emission(M, y[t], z[t])[0] for t in range(N))
        lp += sum(mvn_logpdf(u[t], z[t], delta / 2 * np.eye(dx)) for t in range(N))
        return lp

    def log_q(z, at):
        om, Om, _, rc = oracle.linearise(M, y, at, u, delta, order)
        assert rc == 0
        F, b = oracle.dyn_linearise(M, at)
        mu, S = prior_moments_tv(N, M.m0, M.P0, F, M.Q, b)
        Oinv = np.zeros((N * dx, N * dx))
        for t in range(N):
            Oinv[t * dx:(t + 1) * dx, t * dx:(t + 1) * dx] = np.linalg.inv(Om[t])
        Sinv = np.linalg.inv(S)
        Pc = np.linalg.inv(Sinv + Oinv)
        mc = Pc @ (Sinv @ mu + Oinv @ om.ravel())
        return mvn_logpdf(z.ravel(), mc, 0.5 * (Pc + Pc.T))

    return log_target(xs) - log_target(x) + log_q(x, xs) - log_q(xs, x)


@pytest.mark.parametrize("which,order,N", [(63, 2, 4), (63, 1, 3), (96, 2, 3), (96, 1, 4)])
def test_nonlinear_log_ratio_vs_dense_brute_force(which, order, N):
    rng = np.random.default_rng(90 + which + order)
    if which == 63:
        M = _l63(emit=5, site=np.array([1, 2], np.int32), scale=np.sqrt(5.0))
        d = 3
        x = np.array([1.0, -1.0, 20.0]) + 0.5 * rng.standard_normal((N, 3))
    else:
        d = 5
        M = _l96(d, emit=2, site=np.array([0, 2, 4], np.int32), nu=3.0, scale=0.5)
        x = rng.standard_normal((N, d))
    y = x[:, M.site] + rng.standard_normal((N, len(M.site)))
    y[1, 0] = np.nan   # one unobserved site
    delta = 0.05
    xi_u, xi_x = rng.standard_normal((2, N, d))
    r = oracle.mh_step(M, y, x, delta, order, xi_u, xi_x, 0.5)
    assert r["status"] == 0
    u = x + np.sqrt(delta / 2) * xi_u
    ref = _brute_log_ratio(M, y, x, r["xstar"], u, delta, order)
    assert abs(r["log_ratio"] - ref) < 1e-8 * max(1.0, abs(ref)), (r["log_ratio"], ref)
    back = _brute_log_ratio(M, y, r["xstar"], x, u, delta, order)
    assert abs(ref + back) < 1e-9 * max(1.0, abs(ref))


def test_gauss_site_emission():
    from scipy.stats import norm
    rng = np.random.default_rng(5)
    M = oracle.Model(m0=np.zeros(4), P0=np.eye(4), F=np.eye(4), Q=np.eye(4), emit=5,
                     site=np.array([0, 3, 3, 1], np.int32), scale=1.7)
    yt = rng.standard_normal(4)
    xt = rng.standard_normal(4)
    lh, v, Lam = oracle.emission(M, yt, xt)
    ref = norm.logpdf(yt, xt[M.site], 1.7).sum() + 4 * (0.5 * np.log(2 * np.pi) + np.log(1.7))
    assert abs(lh - ref) < 1e-12
    np.testing.assert_allclose(v, fd_grad(lambda z: oracle.emission(M, yt, z)[0], xt, 1e-5),
                               atol=1e-8)
    np.testing.assert_allclose(Lam, np.diag([-1, -1, 0, -2]) / 1.7 ** 2, atol=1e-15)
    # a NaN entry is an unobserved site: same as dropping it
    y2 = yt.copy()
    y2[1] = np.nan
    M3 = oracle.Model(m0=M.m0, P0=M.P0, F=M.F, Q=M.Q, emit=5, site=np.array([0, 3, 1], np.int32),
                      scale=1.7)
    a = oracle.emission(M, y2, xt)
    b = oracle.emission(M3, yt[[0, 2, 3]], xt)
    assert a[0] == b[0]
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


def test_gauss_site_order2_exact_with_linear_dynamics():
    rng = np.random.default_rng(8)
    d, N = 3, 12
    M = oracle.Model(m0=np.zeros(d), P0=np.eye(d), F=0.9 * np.eye(d) + 0.05, Q=0.3 * np.eye(d),
                     emit=5, site=np.array([1, 2], np.int32), scale=2.0)
    y = rng.standard_normal((N, 2))
    y[::3, 0] = np.nan
    x = rng.standard_normal((N, d))
    for k in range(5):
        xi = rng.standard_normal((2, N, d))
        r = oracle.mh_step(M, y, x, 0.7, 2, xi[0], xi[1], 0.5)
        assert r["status"] == 0 and abs(r["log_ratio"]) < 1e-9
        x = r["x_out"]
