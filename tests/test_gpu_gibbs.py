"""GPU parity of the Gibbs sweep over (theta, x) of the linear-Gaussian model
(akf_gibbs_init / akf_gibbs_sweep) against the oracle's sweep (MI355X only).

Each sweep is compared from the oracle's own state: before it, the GPU
sampler is restarted at the oracle's theta and path (akf_gibbs_init, whose log
posterior and gradient are checked too), both take the same normals and
uniforms, and every output is compared: the proposal's log alpha, the
decision (a tie band around log u), theta, its log posterior and gradient, the
refreshed path and the path steps.  Both sides compute in FP64.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import gibbs as OG  # noqa: E402
from paper_2303_00301_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

LP_TOL = 1e-9         # relative, log posterior (a sum of N terms in FP64)
GRAD_TOL = 1e-7       # norm-wise relative, as the adjoint's own bar
X_TOL = 1e-8          # refreshed path, relative to max(1, |x|)
TIE_BAND = 1e-6       # |log alpha - log u| below this: either decision passes


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2303_00301_amd import sampler
    return sampler


def dev():
    return torch.device("cuda", 0)


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev())


def N_(t):
    return t.detach().cpu().numpy()


def _normals(rng, p, N, dx, k):
    return (rng.standard_normal(p), rng.uniform(1e-3, 1.0), rng.standard_normal((N, dx)),
            rng.standard_normal((k, 2, N, dx)), rng.uniform(1e-3, 1.0, size=k))


def _check_init(S, pw, theta, x, sd, block=0):
    model = S.LGSSM(pw.m0, pw.P0, pw.y, device=dev())
    G = S.gibbs_init(model, T(theta), T(x), prior_sd=sd, block=block)
    lp_ref, g_ref = OG.gibbs_init(pw.m0, pw.P0, pw.y, theta, sd)
    torch.cuda.synchronize()
    assert int(N_(G.status)[0]) == 0
    lp = float(N_(G.logpost)[0])
    assert abs(lp - lp_ref) <= LP_TOL * max(1.0, abs(lp_ref)), (lp, lp_ref)
    g = N_(G.grad)
    assert np.linalg.norm(g - g_ref) <= GRAD_TOL * np.linalg.norm(g_ref)
    return G, lp_ref, g_ref


def _compare_sweep(S, pw, G, lp_ref, g_ref, theta, x, sd, eps, draws, block=0):
    xi_t, u_t, xi_x, xi_p, u_p = draws
    k = len(u_p)
    print(f"gibbs sweep N={pw.N} dx={len(pw.m0)} dy={pw.y.shape[1]} eps={eps} k={k}", flush=True)
    out = S.gibbs_sweep(G, eps, T(xi_t), T([u_t]), T(xi_x), delta=0.5,
                        xi_path=T(xi_p) if k else None, u_path=T(u_p) if k else None)
    ref = OG.gibbs_sweep(pw.m0, pw.P0, pw.y, theta, lp_ref, g_ref, x, sd, eps, xi_t, u_t, xi_x,
                         0.5, xi_p, u_p)
    torch.cuda.synchronize()
    st = N_(out["status"])
    assert st[1] == 0
    la = float(N_(out["log_alpha"])[0])
    la_ref = ref["log_alpha"]
    acc = int(N_(out["accepted_theta"])[0])
    if np.isfinite(la_ref):
        assert abs(la - la_ref) <= 1e-8 * max(1.0, abs(ref["logpost_prop"])), (la, la_ref)
        if abs(la_ref - np.log(u_t)) > TIE_BAND:
            assert acc == int(ref["accepted_theta"]), (la, la_ref, np.log(u_t))
    else:
        assert acc == 0
        assert st[0] != 0 or not np.isfinite(la)
    if acc != int(ref["accepted_theta"]):
        return None  # a tie: the two chains legitimately part here
    np.testing.assert_allclose(N_(G.theta), ref["theta"], rtol=1e-14, atol=1e-14)
    lp = float(N_(G.logpost)[0])
    assert abs(lp - ref["logpost"]) <= LP_TOL * max(1.0, abs(ref["logpost"]))
    assert (np.linalg.norm(N_(G.grad) - ref["grad"])
            <= GRAD_TOL * np.linalg.norm(ref["grad"]))
    xg = N_(G.x)
    np.testing.assert_allclose(xg, ref["x"], rtol=X_TOL, atol=X_TOL)
    if k:
        assert np.all(N_(out["path_status"]) == 0)
        np.testing.assert_array_equal(N_(out["path_accepted"]), ref["path_accepted"])
        n, d = pw.y.shape[0], len(pw.m0)
        np.testing.assert_allclose(N_(out["path_log_ratio"]), ref["path_log_ratio"], rtol=0,
                                   atol=1e-9 * n * d)
    return ref


@pytest.mark.parametrize("N,dx,dy,eps,k,block", [
    (300, 4, 3, 0.004, 1, 0),      # small steps: mostly accepted
    (300, 4, 3, 0.05, 0, 0),       # large steps: mostly rejected; the refresh alone
    (257, 6, 9, 0.003, 2, 5),      # dy > dx, ragged scan blocks
    (1, 2, 1, 0.3, 1, 0),          # one time step
])
def test_gibbs_sweeps_match_oracle(S, N, dx, dy, eps, k, block):
    pw = W.lgssm_params(N=N, dx=dx, dy=dy, seed=11 + dx)
    sd = 10.0
    rng = np.random.default_rng(500 + N + dx)
    theta = pw.theta0.flat()
    x = np.zeros((N, dx))
    p = theta.size
    decisions = []
    for _ in range(5):
        G, lp_ref, g_ref = _check_init(S, pw, theta, x, sd, block)
        ref = _compare_sweep(S, pw, G, lp_ref, g_ref, theta, x, sd, eps,
                             _normals(rng, p, N, dx, k), block)
        if ref is None:
            break
        decisions.append(ref["accepted_theta"])
        theta, x = ref["theta"], ref["x"]
    assert decisions


def test_gibbs_decisions_both_ways(S):
    """Across the sweeps of one chain both outcomes occur and each matches."""
    pw = W.lgssm_params(N=200, dx=3, dy=2, seed=21)
    sd = 10.0
    rng = np.random.default_rng(77)
    theta = pw.theta0.flat()
    x = np.zeros((200, 3))
    seen = set()
    for eps in (0.002, 0.002, 0.3, 0.3, 0.3, 0.002):
        G, lp_ref, g_ref = _check_init(S, pw, theta, x, sd)
        ref = _compare_sweep(S, pw, G, lp_ref, g_ref, theta, x, sd, eps,
                             _normals(rng, theta.size, 200, 3, 1))
        assert ref is not None
        seen.add(bool(ref["accepted_theta"]))
        theta, x = ref["theta"], ref["x"]
    assert seen == {True, False}


def test_gibbs_free_running_sweeps_match_oracle_chain(S):
    """Ten sweeps in a row on the GPU without restarts (the state buffer and
    the cached gradient carried by the library) equal the oracle's chain."""
    pw = W.lgssm_params(N=120, dx=3, dy=2, seed=31)
    sd, eps = 10.0, 0.004
    rng = np.random.default_rng(9)
    theta = pw.theta0.flat()
    x = np.zeros((120, 3))
    G, lp, g = _check_init(S, pw, theta, x, sd)
    for _ in range(10):
        draws = _normals(rng, theta.size, 120, 3, 1)
        ref = _compare_sweep(S, pw, G, lp, g, theta, x, sd, eps, draws)
        assert ref is not None
        theta, x, lp, g = ref["theta"], ref["x"], ref["logpost"], ref["grad"]


def test_gibbs_rejects_a_proposal_whose_filter_fails(S):
    pw = W.lgssm_params(N=50, dx=2, dy=1, seed=6)
    sd = 10.0
    theta = pw.theta0.flat()
    x = np.zeros((50, 2))
    G, lp_ref, g_ref = _check_init(S, pw, theta, x, sd)
    xi_t = np.zeros(theta.size)
    xi_t[4] = 1e6                      # logq_0 -> exp overflows
    draws = (xi_t, 0.5, np.random.default_rng(1).standard_normal((50, 2)),
             np.zeros((0, 2, 50, 2)), np.zeros(0))
    out = S.gibbs_sweep(G, 1.0, T(draws[0]), T([0.5]), T(draws[2]))
    torch.cuda.synchronize()
    assert int(N_(out["accepted_theta"])[0]) == 0
    np.testing.assert_array_equal(N_(G.theta), theta)
    assert float(N_(G.logpost)[0]) == pytest.approx(lp_ref, rel=1e-12)
    ref = OG.gibbs_sweep(pw.m0, pw.P0, pw.y, theta, lp_ref, g_ref, x, sd, 1.0, *draws[:3], 0.5,
                         draws[3], draws[4])
    assert not ref["accepted_theta"]
    np.testing.assert_allclose(N_(G.x), ref["x"], rtol=X_TOL, atol=X_TOL)


def test_gibbs_sweep_full_size(S):
    """One sweep at the differentiation workload's size (d_x = 32, d_y = 16,
    T = 16384, 1584 parameters) with one path step."""
    pw = W.lgssm_params()
    sd, eps = 10.0, 2e-4
    theta = pw.theta0.flat()
    x = np.zeros((pw.N, 32))
    rng = np.random.default_rng(5)
    G, lp_ref, g_ref = _check_init(S, pw, theta, x, sd)
    ref = _compare_sweep(S, pw, G, lp_ref, g_ref, theta, x, sd, eps,
                         _normals(rng, theta.size, pw.N, 32, 1))
    assert ref is not None
