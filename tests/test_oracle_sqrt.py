"""Pins for the square-root form of the parallel filter and sampler in
oracle/scan_ops.py (CPU only).

* tria(M) is lower triangular with a non-negative diagonal and reproduces
  M M^T; for a full-rank M it is the Cholesky factor of M M^T (LAPACK);
* square-root elements carry the standard elements of the same step: equal
  A, b, eta, U U^T = C, Z Z^T = J, and the same log normaliser;
* the square-root combine under random bracketings reproduces the oracle's
  sequential Kalman filter (means, covariances from the factors, cumulative
  log-likelihood), and a combine with a planted sign error does not;
* square-root sampling elements give the standard (E, g) and a factor of L;
* in float32 the standard-form sampler loses accuracy with the condition
  number of Q while the square-root form keeps it (the reason the paper gives
  for the square-root filter): at cond(Q) = 1e6 the standard form misses x*
  by more than 1e-4 smoothing standard deviations and the square-root form
  stays within 3e-5.
"""
import numpy as np

import oracle
from oracle import scan_ops as so


def _model(rng, d, cond):
    G = rng.standard_normal((d, d))
    F = 0.9 * G / np.max(np.abs(np.linalg.eigvals(G)))
    U, _ = np.linalg.qr(rng.standard_normal((d, d)))
    Q = (U * (np.logspace(0, -np.log10(cond), d) * 0.1)) @ U.T
    Q = 0.5 * (Q + Q.T)
    A = rng.standard_normal((d, d))
    P0 = A @ A.T / d + 0.5 * np.eye(d)
    return 0.3 * rng.standard_normal(d), P0, F, 0.1 * rng.standard_normal(d), Q


def _pseudo_obs(rng, N, d):
    return 0.5 * rng.standard_normal((N, d)), rng.uniform(0.01, 0.05, (N, d))


def test_tria_is_a_lower_factor():
    rng = np.random.default_rng(1)
    for r, c in [(1, 1), (3, 5), (6, 12), (8, 8)]:
        M = rng.standard_normal((r, c))
        L = so.tria(M)
        assert L.shape == (r, r)
        assert np.allclose(np.triu(L, 1), 0.0)
        assert np.all(np.diag(L) >= 0)
        np.testing.assert_allclose(L @ L.T, M @ M.T, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(L, np.linalg.cholesky(M @ M.T), rtol=1e-10, atol=1e-12)


def test_sqrt_elements_carry_the_standard_elements():
    rng = np.random.default_rng(2)
    d, N = 5, 7
    m0, P0, F, b, Q = _model(rng, d, 1e3)
    om, Om = _pseudo_obs(rng, N, d)
    R = np.stack([np.diag(o) for o in Om])
    std = so.filter_elements(m0, P0, F, b, Q, np.eye(d), R, om)
    lcs = so.filter_log_norms(m0, P0, F, b, Q, np.eye(d), R, om)
    sq = so.sqrt_filter_elements(m0, P0, F, b, Q, om, Om)
    for (A, be, C, eta, J), lc, (A2, b2, U, eta2, Z, lc2) in zip(std, lcs, sq):
        np.testing.assert_allclose(A2, A, atol=1e-12)
        np.testing.assert_allclose(b2, be, atol=1e-12)
        np.testing.assert_allclose(U @ U.T, C, atol=1e-12)
        np.testing.assert_allclose(eta2, eta, atol=1e-12)
        np.testing.assert_allclose(Z @ Z.T, J, atol=1e-11)
        assert abs(lc2 - lc) < 1e-11


def _scan_check(op, rng, d=4, N=11):
    m0, P0, F, b, Q = _model(rng, d, 1e4)
    om, Om = _pseudo_obs(rng, N, d)
    ref = oracle.kf(m0, P0, F, Q, np.eye(d), np.stack([np.diag(o) for o in Om]), om, b=b,
                    R_per_t=True)
    el = so.sqrt_filter_elements(m0, P0, F, b, Q, om, Om)
    errs = []
    for pref in (so.scan_fold(el, op), so.scan_random_tree(el, op, rng),
                 so.scan_random_tree(el, op, rng)):
        m = np.array([p[1] for p in pref])
        P = np.array([p[2] @ p[2].T for p in pref])
        lz = np.array([p[5] for p in pref])
        errs.append(max(np.abs(m - ref["mf"]).max(), np.abs(P - ref["Pf"]).max(),
                        np.abs(lz - np.cumsum(ref["ell"])).max()))
        # a prefix from t = 0 is a filtering moment pair
        assert all(np.abs(p[0]).max() < 1e-12 and np.abs(p[4]).max() < 1e-12 for p in pref)
    return max(errs)


def test_sqrt_combine_reproduces_the_sequential_filter_under_any_bracketing():
    rng = np.random.default_rng(3)
    assert _scan_check(so.sqrt_filter_combine, rng) < 1e-10


def test_sqrt_combine_with_a_planted_sign_error_fails():
    rng = np.random.default_rng(3)

    def bad(ei, ej):
        Ai, bi, Ui, eti, Zi, lci = ei
        Aj, bj, Uj, etj, Zj, lcj = ej
        d = Ai.shape[0]
        X = so.tria(np.block([[Ui.T @ Zj, np.eye(d)], [Zj, np.zeros((d, d))]]))
        X11, X21 = X[:d, :d], X[d:, :d]
        G = np.linalg.solve(X11, Ui.T).T
        Mm = np.eye(d) + G @ X21.T  # sign error
        good = so.sqrt_filter_combine(ei, ej)
        return (Aj @ Mm @ Ai,) + good[1:]

    assert _scan_check(bad, rng) > 1e-3


def test_sqrt_sampling_elements_match_the_standard_ones():
    rng = np.random.default_rng(4)
    d, N = 6, 9
    m0, P0, F, b, Q = _model(rng, d, 1e3)
    om, Om = _pseudo_obs(rng, N, d)
    ref = oracle.kf(m0, P0, F, Q, np.eye(d), np.stack([np.diag(o) for o in Om]), om, b=b,
                    R_per_t=True)
    std = so.sampling_elements(F, ref["mf"], ref["Pf"], ref["mp"], ref["Pp"])
    Uf = np.linalg.cholesky(ref["Pf"])
    sq = so.sqrt_sampling_elements(F, b, Q, ref["mf"], Uf)
    for (E, g, L), (E2, g2, Lc) in zip(std, sq):
        np.testing.assert_allclose(E2, E, atol=1e-10)
        np.testing.assert_allclose(g2, g, atol=1e-10)
        np.testing.assert_allclose(Lc @ Lc.T, L, atol=1e-12)


def _fp32_sampler_errors(d, cond, N=400, seed=0):
    rng = np.random.default_rng(seed)
    m0, P0, F, b, Q = _model(rng, d, cond)
    om, Om = _pseudo_obs(rng, N, d)
    ref = oracle.kf(m0, P0, F, Q, np.eye(d), np.stack([np.diag(o) for o in Om]), om, b=b,
                    R_per_t=True)
    xi = rng.standard_normal((N, d))
    x_ref, rc = oracle.rts_sample(F, ref["mf"], ref["Pf"], ref["mp"], ref["Pp"], xi)
    assert rc == 0
    _, Ps, _, _ = oracle.rts_smooth(F, ref["mf"], ref["Pf"], ref["mp"], ref["Pp"])
    sd = np.sqrt(np.einsum("tii->ti", Ps))
    f = np.float32
    mf, Pf, F32, Q32, b32 = (ref["mf"].astype(f), ref["Pf"].astype(f), F.astype(f),
                             Q.astype(f), b.astype(f))
    xi32 = xi.astype(f)
    # standard form, every operation in float32
    els = []
    for t in range(N - 1):
        Pp = F32 @ Pf[t] @ F32.T + Q32
        E = np.linalg.solve(Pp, F32 @ Pf[t]).T
        L = Pf[t] - E @ F32 @ Pf[t]
        L = 0.5 * (L + L.T)
        els.append((E, mf[t] - E @ (F32 @ mf[t] + b32) + np.linalg.cholesky(L) @ xi32[t]))
    els.append((np.zeros((d, d), f), mf[-1] + np.linalg.cholesky(Pf[-1]) @ xi32[-1]))
    x_std = np.array([e[1] for e in so.suffix_scan(els, so.path_combine, so.scan_fold)])
    # square-root form in float32 (triangularisations from float32 inputs)
    sq = so.sqrt_sampling_elements(F, b, Q, mf, np.linalg.cholesky(ref["Pf"]).astype(f), f)
    els = [(E, g + Lc @ xi32[t]) for t, (E, g, Lc) in enumerate(sq)]
    x_sq = np.array([e[1] for e in so.suffix_scan(els, so.path_combine, so.scan_fold)])
    return (np.abs(x_std - x_ref) / sd).max(), (np.abs(x_sq - x_ref) / sd).max()


def test_float32_square_root_sampler_keeps_accuracy_where_the_standard_form_loses_it():
    e_std, e_sq = _fp32_sampler_errors(16, 1e6)
    assert e_std > 1e-4, e_std
    assert e_sq < 3e-5, e_sq
    # at a benign condition number both forms are fine in float32
    e_std, e_sq = _fp32_sampler_errors(16, 1e1, seed=1)
    assert e_std < 3e-5 and e_sq < 3e-5, (e_std, e_sq)
