"""Brute-force references used to pin the oracle (dense Gaussian algebra with
numpy/scipy library routines; no Kalman recursions)."""
from __future__ import annotations

import numpy as np


def mvn_logpdf(x, mean, cov):
    x = np.asarray(x, float).ravel()
    mean = np.asarray(mean, float).ravel()
    L = np.linalg.cholesky(cov)
    z = np.linalg.solve(L, x - mean)
    return -0.5 * (len(x) * np.log(2 * np.pi) + 2 * np.log(np.diag(L)).sum() + z @ z)


def prior_moments(N, m0, P0, F, Q, b=None):
    """Mean [N*d] and covariance [N*d, N*d] of x_{0:N-1} under the Gaussian
    dynamics, built from Cov(x_s, x_t) = Var(x_s) (F^{t-s})^T for s <= t."""
    d = len(m0)
    b = np.zeros(d) if b is None else np.asarray(b, float)
    mu = np.zeros((N, d))
    V = [None] * N
    mu[0] = m0
    V[0] = np.asarray(P0, float)
    for t in range(1, N):
        mu[t] = F @ mu[t - 1] + b
        V[t] = F @ V[t - 1] @ F.T + Q
    S = np.zeros((N * d, N * d))
    for s in range(N):
        Fp = np.eye(d)
        for t in range(s, N):
            blk = V[s] @ Fp.T
            S[t * d:(t + 1) * d, s * d:(s + 1) * d] = blk.T
            S[s * d:(s + 1) * d, t * d:(t + 1) * d] = blk
            Fp = F @ Fp
    return mu.ravel(), S


def prior_moments_tv(N, m0, P0, F, Q, b=None):
    """Mean and covariance of x_{0:N-1} for per-step dynamics x_t = F[t] x_{t-1}
    + b[t] + N(0, Q) (F [N,d,d], b [N,d]; entry 0 unused), from the linear
    system (I - Fblk) X = c + e with Fblk holding F[t] at block (t, t-1),
    c = (m0, b[1], ..., b[N-1]) and e ~ N(0, blkdiag(P0, Q, ..., Q))."""
    d = len(m0)
    n = N * d
    M = np.eye(n)
    c = np.zeros(n)
    E = np.zeros((n, n))
    c[:d] = m0
    E[:d, :d] = P0
    for t in range(1, N):
        M[t * d:(t + 1) * d, (t - 1) * d:t * d] = -np.asarray(F[t], float)
        if b is not None:
            c[t * d:(t + 1) * d] = b[t]
        E[t * d:(t + 1) * d, t * d:(t + 1) * d] = Q
    Mi = np.linalg.inv(M)
    S = Mi @ E @ Mi.T
    return Mi @ c, 0.5 * (S + S.T)


def dense_lgssm(N, m0, P0, F, Q, H_list, R_list, y, b=None):
    """log p(y), smoothing means [N,d] and covariances [N,d,d] by conditioning
    the joint Gaussian of (x_{0:N-1}, y_{0:N-1}).  F (and b) may be per-step,
    [N,d,d] ([N,d])."""
    d = len(m0)
    if np.ndim(F) == 3:
        mu, S = prior_moments_tv(N, m0, P0, F, Q, b)
    else:
        mu, S = prior_moments(N, m0, P0, F, Q, b)
    dys = [H.shape[0] for H in H_list]
    Hb = np.zeros((sum(dys), N * d))
    Rb = np.zeros((sum(dys), sum(dys)))
    r = 0
    for t in range(N):
        Hb[r:r + dys[t], t * d:(t + 1) * d] = H_list[t]
        Rb[r:r + dys[t], r:r + dys[t]] = R_list[t]
        r += dys[t]
    yv = np.concatenate([np.asarray(y[t], float) for t in range(N)])
    Syy = Hb @ S @ Hb.T + Rb
    ll = mvn_logpdf(yv, Hb @ mu, Syy)
    K = np.linalg.solve(Syy, Hb @ S).T
    pm = mu + K @ (yv - Hb @ mu)
    pc = S - K @ Hb @ S
    ms = pm.reshape(N, d)
    Ps = np.stack([pc[t * d:(t + 1) * d, t * d:(t + 1) * d] for t in range(N)])
    return ll, ms, Ps, pm, pc


def fd_grad(f, x, h):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x)
        e.flat[i] = h
        g.flat[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g
