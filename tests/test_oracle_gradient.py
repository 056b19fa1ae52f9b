"""Pin for the oracle's Fisher-identity score of log p(y | theta) (CPU only):
central finite differences of the oracle's own log-likelihood in FP64,
theta = (F, log diag Q, H, log diag R)."""
import numpy as np
import pytest

import oracle
from paper_2303_00301_amd import workloads as W


def _unflat(v, dx, dy):
    i = 0
    F = v[i:i + dx * dx].reshape(dx, dx); i += dx * dx
    lq = v[i:i + dx]; i += dx
    H = v[i:i + dy * dx].reshape(dy, dx); i += dy * dx
    lr = v[i:i + dy]
    return F, lq, H, lr


@pytest.mark.parametrize("N,dx,dy,seed", [(64, 4, 3, 0), (200, 6, 2, 1), (256, 8, 4, 2)])
def test_fisher_score_vs_central_fd(N, dx, dy, seed):
    pw = W.lgssm_params(N=N, dx=dx, dy=dy, seed=seed)
    t0 = pw.theta0
    ll, dF, dq, dH, dr = oracle.fisher_score(pw.m0, pw.P0, t0.F, t0.logq, t0.H, t0.logr, pw.y)
    assert np.isfinite(ll)
    assert abs(ll - oracle.lgssm_loglik(pw.m0, pw.P0, t0.F, t0.logq, t0.H, t0.logr, pw.y)) < 1e-9
    v0 = t0.flat()
    f = lambda v: oracle.lgssm_loglik(pw.m0, pw.P0, *_unflat(v, dx, dy), pw.y)
    h = 1e-4
    g = np.zeros_like(v0)
    for i in range(v0.size):
        e = np.zeros_like(v0)
        e[i] = h
        g[i] = (f(v0 + e) - f(v0 - e)) / (2 * h)
    gF, gq, gH, gr = _unflat(g, dx, dy)
    for a, b in ((dF, gF), (dq, gq), (dH, gH), (dr, gr)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert rel < 1e-5, rel


def test_fisher_score_directional_fd_larger():
    """16 random directions at a larger size (N = 2048, dx = 16, dy = 8)."""
    pw = W.lgssm_params(N=2048, dx=16, dy=8, seed=3)
    t0 = pw.theta0
    dx, dy = 16, 8
    _, dF, dq, dH, dr = oracle.fisher_score(pw.m0, pw.P0, t0.F, t0.logq, t0.H, t0.logr, pw.y)
    g = np.concatenate([dF.ravel(), dq, dH.ravel(), dr])
    v0 = t0.flat()
    f = lambda v: oracle.lgssm_loglik(pw.m0, pw.P0, *_unflat(v, dx, dy), pw.y)
    rng = np.random.default_rng(0)
    h = 1e-4
    for _ in range(16):
        d = rng.standard_normal(v0.size)
        d /= np.linalg.norm(d)
        fd = (f(v0 + h * d) - f(v0 - h * d)) / (2 * h)
        assert abs(fd - g @ d) < 1e-5 * max(1.0, np.linalg.norm(g)), (fd, g @ d)


@pytest.mark.parametrize("N,dx,dy,seed", [(1, 2, 1, 7), (6, 3, 2, 8), (8, 4, 3, 9)])
def test_lgssm_loglik_vs_dense_joint_gaussian(N, dx, dy, seed):
    """The theta-parameterised log-likelihood equals log N(y; E y, Cov y) of the
    joint Gaussian with Q = diag(exp(logq)), R = diag(exp(logr))."""
    from tests.oracle_util import dense_lgssm
    pw = W.lgssm_params(N=N, dx=dx, dy=dy, seed=seed)
    t0 = pw.theta0
    Q = np.diag(np.exp(t0.logq))
    R = np.diag(np.exp(t0.logr))
    ll_dense = dense_lgssm(N, pw.m0, pw.P0, t0.F, Q, [t0.H] * N, [R] * N, pw.y)[0]
    ll = oracle.lgssm_loglik(pw.m0, pw.P0, t0.F, t0.logq, t0.H, t0.logr, pw.y)
    assert abs(ll - ll_dense) < 1e-9 * max(1.0, abs(ll_dense))
