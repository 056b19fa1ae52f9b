"""Associative-scan form of the Kalman filter and the RTS sampler, in numpy FP64.

TEST INFRASTRUCTURE ONLY (part of the oracle; see ``oracle/__init__.py``).

These are the element/operator definitions that make filtering and pathwise
sampling prefix sums (App. A, "Prefix-sums and the parallel Kalman filter" and
"Parallel Rauch--Tung--Striebel sampler"), written out plainly so that tests can
check that any bracketing of the scan reproduces the sequential filter and
sampler of ``akf_oracle.c``.

Filtering element for step t (the pair p(x_t | y_t, x_{t-1}), p(y_t | x_{t-1})),
LGSSM  x_t = F x_{t-1} + b + N(0,Q),  y_t = H x_t + N(0,R_t):
    p(x_t | y_t, x_{t-1}) = N(x_t; A x_{t-1} + b_e, C)
    p(y_t | x_{t-1})      propto exp(-1/2 x^T J x + eta^T x)
obtained by conditioning the joint Gaussian of (x_t, y_t) given x_{t-1}.  The
first element carries the prior instead (A = 0, eta = 0, J = 0).

The operator integrates out the shared intermediate state; with Z = I + C_i J_j:
    A  = A_j Z^{-1} A_i
    b  = A_j Z^{-1} (b_i + C_i eta_j) + b_j
    C  = A_j Z^{-1} C_i A_j^T + C_j
    eta = A_i^T Z^{-T} (eta_j - J_j b_i) + eta_i
    J  = A_i^T Z^{-T} J_j A_i + J_i
(i is the earlier element).  The prefix up to t has A = 0, J = 0, eta = 0,
b = m^f_t, C = P^f_t.  Carrying the normaliser log c of p(y | x_prev) with each
element (filter_log_norms, filter_combine_log_norm) makes the prefix's log c the
log marginal likelihood log p(y_{0:t}), with no second pass.

Sampling element (eq. backward, eq. EgL_comb):  E_t = P^f_t F^T (P^p_{t+1})^{-1},
g_t = m^f_t - E_t m^p_{t+1}, L_t = P^f_t - E_t F P^f_t; terminal (0, m^f, P^f).
Operator (earlier i, later j): (E_i E_j, E_i g_j + g_i, E_i L_j E_i^T + L_i).
The suffix scan yields the RTS smoother marginals (g~_t, L~_t); on path elements
(E_t, U_t = g_t + chol(L_t) xi_t) with (E_i E_j, E_i U_j + U_i) it yields a
pathwise sample (Prop. "prefix-sum sampling").
"""
from __future__ import annotations

import numpy as np


def filter_elements(m0, P0, F, b, Q, H, R, y):
    """Elements e_t = (A, b, C, eta, J) for t = 0..N-1.  R is [N,dy,dy] or [dy,dy]."""
    N = y.shape[0]
    dx = len(m0)
    b = np.zeros(dx) if b is None else np.asarray(b, float)
    R = np.asarray(R, float)
    out = []
    for t in range(N):
        Rt = R[t] if R.ndim == 3 else R
        if t == 0:
            S = H @ P0 @ H.T + Rt
            K = np.linalg.solve(S, H @ P0).T
            A = np.zeros((dx, dx))
            be = m0 + K @ (y[0] - H @ m0)
            Cm = P0 - K @ S @ K.T
            eta = np.zeros(dx)
            J = np.zeros((dx, dx))
        else:
            S = H @ Q @ H.T + Rt
            K = np.linalg.solve(S, H @ Q).T
            IKH = np.eye(dx) - K @ H
            A = IKH @ F
            be = b + K @ (y[t] - H @ b)
            Cm = IKH @ Q
            HF = H @ F
            eta = HF.T @ np.linalg.solve(S, y[t] - H @ b)
            J = HF.T @ np.linalg.solve(S, HF)
        out.append((A, be, 0.5 * (Cm + Cm.T), eta, 0.5 * (J + J.T)))
    return out


def filter_combine(ei, ej):
    Ai, bi, Ci, ei_, Ji = ei
    Aj, bj, Cj, ej_, Jj = ej
    d = Ai.shape[0]
    Z = np.eye(d) + Ci @ Jj
    ZiAi = np.linalg.solve(Z, Ai)
    A = Aj @ ZiAi
    bb = Aj @ np.linalg.solve(Z, bi + Ci @ ej_) + bj
    Cm = Aj @ np.linalg.solve(Z, Ci) @ Aj.T + Cj
    ZtT = Z.T
    eta = Ai.T @ np.linalg.solve(ZtT, ej_ - Jj @ bi) + ei_
    J = Ai.T @ np.linalg.solve(ZtT, Jj) @ Ai + Ji
    return (A, bb, 0.5 * (Cm + Cm.T), eta, 0.5 * (J + J.T))


def filter_log_norms(m0, P0, F, b, Q, H, R, y):
    """log c_t of each filtering element: p(y_t | x_{t-1}) = exp(log c_t + eta^T x
    - 1/2 x^T J x), so log c_t = log N(y_t; H b, S_t) with S_t = H Q H^T + R_t
    (t >= 1, the density at x_{t-1} = 0), and log c_0 = log N(y_0; H m0, H P0 H^T + R_0)."""
    N = y.shape[0]
    dx = len(m0)
    b = np.zeros(dx) if b is None else np.asarray(b, float)
    R = np.asarray(R, float)
    out = []
    for t in range(N):
        Rt = R[t] if R.ndim == 3 else R
        P, mu = (P0, m0) if t == 0 else (Q, b)
        S = H @ P @ H.T + Rt
        r = y[t] - H @ mu
        _, logdet = np.linalg.slogdet(S)
        out.append(-0.5 * (len(r) * np.log(2 * np.pi) + logdet + r @ np.linalg.solve(S, r)))
    return out


def filter_combine_log_norm(ei, lci, ej, lcj):
    """log c of e_i (x) e_j: the x-independent part of
    int N(x; A_i x_p + b_i, C_i) exp(log c_j + eta_j^T x - 1/2 x^T J_j x) dx,
    a Gaussian integral: with Z = I + C_i J_j and v = eta_j - J_j b_i,
    log c_i + log c_j - 1/2 log det Z + eta_j^T b_i - 1/2 b_i^T J_j b_i
    + 1/2 v^T Z^{-1} C_i v."""
    _, bi, Ci, _, _ = ei
    _, _, _, ej_, Jj = ej
    d = Ci.shape[0]
    Z = np.eye(d) + Ci @ Jj
    v = ej_ - Jj @ bi
    _, logdet = np.linalg.slogdet(Z)
    return (lci + lcj - 0.5 * logdet + ej_ @ bi - 0.5 * bi @ Jj @ bi
            + 0.5 * v @ np.linalg.solve(Z, Ci @ v))


def sampling_elements(F, mf, Pf, mp, Pp):
    """(E, g, L) for t = 0..N-1 (terminal element last)."""
    N = mf.shape[0]
    out = []
    for t in range(N - 1):
        E = np.linalg.solve(Pp[t + 1], F @ Pf[t]).T
        g = mf[t] - E @ mp[t + 1]
        L = Pf[t] - E @ F @ Pf[t]
        out.append((E, g, 0.5 * (L + L.T)))
    dx = mf.shape[1]
    out.append((np.zeros((dx, dx)), mf[-1].copy(), Pf[-1].copy()))
    return out


def sampling_combine(ei, ej):
    Ei, gi, Li = ei
    Ej, gj, Lj = ej
    L = Ei @ Lj @ Ei.T + Li
    return (Ei @ Ej, Ei @ gj + gi, 0.5 * (L + L.T))


def path_elements(samp_elems, xi):
    """(E_t, U_t) with U_t = g_t + chol(L_t) xi_t (lower factor, positive diagonal)."""
    return [(E, g + np.linalg.cholesky(L) @ xi[t]) for t, (E, g, L) in enumerate(samp_elems)]


def path_combine(ei, ej):
    Ei, Ui = ei
    Ej, Uj = ej
    return (Ei @ Ej, Ei @ Uj + Ui)


# ---------------------------------------------------------------------------
# Square-root form (the filter the paper points to for FP32 robustness in its
# stochastic-volatility section).  Covariances are carried as factors: the
# filtering element holds U with C = U U^T and Z with J = Z Z^T, and every
# covariance update is a triangularisation.  All functions take a dtype so that
# tests can run them in float32; the default is float64.
#
# tria(M), M [r, c] with c >= r: the lower-triangular L [r, r] with
# non-negative diagonal and L L^T = M M^T (from a QR factorisation of M^T).
#
# Element of step t >= 1 for the pseudo-observation omega_t = x_t + N(0, Om_t)
# (H = I, diagonal Om_t), from the block triangularisation
#     tria([[Om^{1/2}, L_Q], [0, L_Q]]) = [[P11, 0], [P21, P22]]:
# P11 P11^T = S = Q + Om, P21 = Q P11^{-T}, P22 P22^T = Q - Q S^{-1} Q = C, so
#     K = P21 P11^{-1},  A = F - K F,  b = b_dyn + K w,  U = P22,
#     Z = F^T P11^{-T},  eta = Z P11^{-1} w,  w = omega_t - b_dyn,
#     log c = -1/2 (d log 2 pi + 2 sum log diag P11 + |P11^{-1} w|^2);
# step 0 uses the prior factor L_0 in place of L_Q, m0 in place of b_dyn, and
# has A = 0, Z = 0, eta = 0.
#
# Combine (i earlier, j later), from
#     tria([[U_i^T Z_j, I], [Z_j, 0]]) = [[X11, 0], [X21, X22]]:
# X11 X11^T = W = I + U_i^T J_j U_i, X21 = J_j U_i X11^{-T},
# X22 X22^T = J_j (I + C_i J_j)^{-1}.  With G = U_i X11^{-T} and
# M = I - G X21^T = (I + C_i J_j)^{-1} (Woodbury):
#     A = A_j M A_i,  b = A_j M (b_i + C_i eta_j) + b_j,
#     U = tria([A_j G, U_j])           (C_i - C_i J_j M C_i = G G^T),
#     eta = A_i^T M^T c + eta_i,  c = eta_j - J_j b_i,
#     Z = tria([A_i^T X22, Z_i]),
#     log c = log c_i + log c_j - sum log diag X11 + 1/2 b_i^T (eta_j + c)
#             + 1/2 |X11^{-1} U_i^T c|^2.
#
# Sampling element from tria([[L_Q, F U^f_t], [0, U^f_t]]) = [[P11, 0],
# [P21, P22]]: P11 P11^T = P^p_{t+1}, E_t = P21 P11^{-1}, chol(L_t) = P22,
# g_t = m^f_t - E_t (F m^f_t + b_dyn).
# ---------------------------------------------------------------------------
def tria(M, dtype=np.float64):
    M = np.asarray(M, dtype)
    R = np.linalg.qr(M.T, mode="r")
    L = R.T[:, :M.shape[0]]
    s = np.where(np.diag(L) < 0, -1, 1).astype(dtype)
    return L * s


def _lower_solve(L, B):
    """L^{-1} B for lower-triangular L (B a vector or matrix)."""
    return np.linalg.solve(L, B)


def _right_solve(B, L):
    """B L^{-1} for lower-triangular L."""
    return np.linalg.solve(L.T, B.T).T


def sqrt_filter_elements(m0, P0, F, b, Q, om, Om, dtype=np.float64):
    """Square-root elements (A, b, U, eta, Z, log c) for t = 0..N-1; Om [N, d] holds
    the diagonal pseudo-observation variances."""
    N, d = om.shape
    F = np.asarray(F, dtype)
    b = np.zeros(d, dtype) if b is None else np.asarray(b, dtype)
    LQ = np.linalg.cholesky(np.asarray(Q, np.float64)).astype(dtype)
    L0 = np.linalg.cholesky(np.asarray(P0, np.float64)).astype(dtype)
    Zd = np.zeros((d, d), dtype)
    out = []
    for t in range(N):
        Ls, mu = (L0, np.asarray(m0, dtype)) if t == 0 else (LQ, b)
        Psi = tria(np.block([[np.diag(np.sqrt(Om[t])).astype(dtype), Ls], [Zd, Ls]]), dtype)
        P11, P21, P22 = Psi[:d, :d], Psi[d:, :d], Psi[d:, d:]
        K = _right_solve(P21, P11)
        w = np.asarray(om[t], dtype) - mu
        s = _lower_solve(P11, w)
        lc = -0.5 * (d * np.log(2 * np.pi) + 2 * np.sum(np.log(np.diag(P11).astype(np.float64)))
                     + float(s @ s))
        if t == 0:
            el = (Zd.copy(), mu + K @ w, P22, np.zeros(d, dtype), Zd.copy())
        else:
            Z = _lower_solve(P11, F).T
            el = (F - K @ F, mu + K @ w, P22, Z @ s, Z)
        out.append(el + (lc,))
    return out


def sqrt_filter_combine(ei, ej, dtype=np.float64):
    Ai, bi, Ui, eti, Zi, lci = ei
    Aj, bj, Uj, etj, Zj, lcj = ej
    d = Ai.shape[0]
    I = np.eye(d, dtype=dtype)
    X = tria(np.block([[Ui.T @ Zj, I], [Zj, np.zeros((d, d), dtype)]]), dtype)
    X11, X21, X22 = X[:d, :d], X[d:, :d], X[d:, d:]
    G = _lower_solve(X11, Ui.T).T
    Mm = I - G @ X21.T
    c = etj - Zj @ (Zj.T @ bi)
    h = _lower_solve(X11, Ui.T @ c)
    lc = (lci + lcj - np.sum(np.log(np.diag(X11).astype(np.float64)))
          + 0.5 * float(bi @ (etj + c)) + 0.5 * float(h @ h))
    return (Aj @ Mm @ Ai, Aj @ (Mm @ (bi + Ui @ (Ui.T @ etj))) + bj,
            tria(np.hstack([Aj @ G, Uj]), dtype), Ai.T @ (Mm.T @ c) + eti,
            tria(np.hstack([Ai.T @ X22, Zi]), dtype), lc)


def sqrt_sampling_elements(F, b, Q, mf, Uf, dtype=np.float64):
    """(E, g, chol L) for t = 0..N-1 from filtering means and factors U^f_t."""
    N, d = mf.shape
    F = np.asarray(F, dtype)
    b = np.zeros(d, dtype) if b is None else np.asarray(b, dtype)
    LQ = np.linalg.cholesky(np.asarray(Q, np.float64)).astype(dtype)
    out = []
    for t in range(N - 1):
        Psi = tria(np.block([[LQ, F @ Uf[t]], [np.zeros((d, d), dtype), Uf[t]]]), dtype)
        P11, P21, P22 = Psi[:d, :d], Psi[d:, :d], Psi[d:, d:]
        E = _right_solve(P21, P11)
        out.append((E, mf[t] - E @ (F @ mf[t] + b), P22))
    out.append((np.zeros((d, d), dtype), np.asarray(mf[-1], dtype), np.asarray(Uf[-1], dtype)))
    return out


def scan_fold(elems, op):
    """Inclusive prefix scan by left fold: out[t] = e_0 op ... op e_t."""
    out = [elems[0]]
    for e in elems[1:]:
        out.append(op(out[-1], e))
    return out


def scan_random_tree(elems, op, rng):
    """Inclusive prefix scan with a random bracketing.

    The range is split at a random point; the left half's prefixes are computed
    recursively, the right half's prefixes recursively, and the left total is
    combined on the left of every right prefix.  Every output is a product over
    the same sequence under a different association, which only agrees with
    scan_fold when op is associative.
    """
    n = len(elems)
    if n == 1:
        return [elems[0]]
    k = int(rng.integers(1, n))
    left = scan_random_tree(elems[:k], op, rng)
    right = scan_random_tree(elems[k:], op, rng)
    tot = left[-1]
    return left + [op(tot, r) for r in right]


def suffix_scan(elems, op, prefix_scan):
    """Suffix scan out[t] = e_t op ... op e_{N-1}, via a prefix scan of the reversed
    sequence with the operands swapped."""
    rev = prefix_scan(list(reversed(elems)), lambda a, b: op(b, a))
    return list(reversed(rev))
