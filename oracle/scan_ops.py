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
