"""GPU parity of first-order runs that form the auxiliary model's matrices
once per call (akf_mh_run_first_order) against the FP64 oracle.

Under first-order proposals Omega_t = delta/2 I for every path, so all
covariances of the auxiliary model are shared by every step of a run and the
oracle's plain step (which re-forms them each time) must give the same chain.
The GPU runs a whole chain in one call; the oracle follows it step by step
from the same state, taking the GPU's accept decision only inside the tie band
of the stated log-ratio tolerance.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2303_00301_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

ELL_TOL = 1e-8        # log Z, relative to max(1, |log Z|), plus 1e-9 N
LR_TOL_PER_TD = 1e-9  # log ratio, per (time step, coordinate)
TIE_BAND = 1e-6


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2303_00301_amd import sampler
    return sampler


def dev():
    return torch.device("cuda", 0)


def T(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev())


def N_(t):
    return t.detach().cpu().numpy()


def _follow(S, M_or, M_dev, y, x0, delta, xi, un, block=0):
    """Run the chain on the GPU in one call; replay it on the oracle."""
    n = xi.shape[0]
    x_gpu = T(x0)
    out = S.mh_run(M_dev, T(y), x_gpu, delta, 1, T(xi), T(un), block=block, reuse_matrices=True)
    torch.cuda.synchronize()
    st, acc = N_(out["status"]), N_(out["accepted"])
    lr, lzf, lzr = N_(out["log_ratio"]), N_(out["logZ_fwd"]), N_(out["logZ_rev"])
    N, d = x0.shape
    x = x0.copy()
    n_acc = 0
    for k in range(n):
        r = oracle.mh_step(M_or, y, x, delta, 1, xi[k][0], xi[k][1], float(un[k]))
        assert int(st[k]) == r["status"], (k, int(st[k]), r["status"])
        if r["status"] == 0:
            lr_tol = LR_TOL_PER_TD * N * d + 1e-9 * max(1.0, abs(r["log_ratio"]))
            assert abs(lr[k] - r["log_ratio"]) <= lr_tol, (k, lr[k], r["log_ratio"], lr_tol)
            for g, key in ((lzf[k], "logZ_fwd"), (lzr[k], "logZ_rev")):
                tol = ELL_TOL * max(1.0, abs(r[key])) + 1e-9 * N
                assert abs(g - r[key]) <= tol, (k, key, g, r[key])
            if abs(np.log(un[k]) - r["log_ratio"]) > max(TIE_BAND, lr_tol):
                assert int(acc[k]) == r["accepted"], k
            x = r["xstar"] if acc[k] else x
        else:
            assert int(acc[k]) == 0 and r["accepted"] == 0
        n_acc += int(acc[k])
    np.testing.assert_allclose(N_(x_gpu), x, rtol=1e-7, atol=1e-8)
    return n_acc


@pytest.mark.parametrize("N,block", [(200, 0), (37, 5), (1, 0)])
def test_poisson_chain(S, N, block):
    """d = 8 Poisson log-link, ragged scan blocks, and the single-step series."""
    w = W.poisson_ar1(N=N)
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    x0 = np.log(w.y + 0.5)
    _follow(S, M_or, M_dev, w.y, x0, w.delta, w.normals(5), w.uniforms(5), block=block)


@pytest.mark.parametrize("N,block", [(301, 16), (64, 1)])
def test_latent_field_chain(S, N, block):
    """d = 64 (no padding), Student-t at sites."""
    w = W.latent_field(N=N)
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    x0 = w.x_true + 0.05 * np.random.default_rng(1).standard_normal(w.x_true.shape)
    _follow(S, M_or, M_dev, w.y, x0, 0.2 * w.delta, w.normals(3), w.uniforms(3), block=block)


def test_stoch_vol_chain(S):
    """d = 30 (padded to 32), stochastic volatility, T = 250."""
    w = W.stoch_vol(order=1)
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    n_acc = _follow(S, M_or, M_dev, w.y, w.x_true.copy(), w.delta, w.normals(6), w.uniforms(6))
    assert n_acc >= 1


def test_gaussian_general_H_chain(S):
    """Gaussian emission with dy < dx (order 1 keeps Omega = delta/2 I)."""
    rng = np.random.default_rng(77)
    N, dx, dy = 50, 6, 3
    G = rng.standard_normal((dx, dx))
    F = 0.9 * G / np.max(np.abs(np.linalg.eigvals(G)))
    A = rng.standard_normal((dx, dx))
    Q = A @ A.T / dx + 0.2 * np.eye(dx)
    H = rng.standard_normal((dy, dx))
    C = rng.standard_normal((dy, dy))
    R = C @ C.T / dy + 0.3 * np.eye(dy)
    kw = dict(m0=0.1 * rng.standard_normal(dx), P0=np.eye(dx), F=F, Q=Q, emit=0,
              b=0.05 * rng.standard_normal(dx), H=H, R=R)
    y = rng.standard_normal((N, dy))
    M_or = oracle.Model(**kw)
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw)
    xi = rng.standard_normal((4, 2, N, dx))
    un = rng.random(4)
    _follow(S, M_or, M_dev, y, 0.2 * rng.standard_normal((N, dx)), 0.4, xi, un)


def test_multivariate_t_chain(S):
    """Multivariate-t emission (first order only) on a coupled d = 16 prior."""
    rng = np.random.default_rng(91)
    N, d = 40, 16
    G = rng.standard_normal((d, d))
    F = 0.8 * G / np.max(np.abs(np.linalg.eigvals(G)))
    A = rng.standard_normal((d, d))
    Q = A @ A.T / d + 0.3 * np.eye(d)
    C = rng.standard_normal((d, d))
    kw = dict(m0=np.zeros(d), P0=np.eye(d), F=F, Q=Q, emit=4, site=np.arange(d, dtype=np.int32),
              nu=1.0, R=C @ C.T / d + 0.5 * np.eye(d))
    y = 2.0 * rng.standard_normal((N, d))
    M_or = oracle.Model(**kw)
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw)
    xi = rng.standard_normal((3, 2, N, d))
    _follow(S, M_or, M_dev, y, 0.5 * rng.standard_normal((N, d)), 0.05, xi, rng.random(3))


def test_matches_plain_run(S):
    """The same chain as akf_mh_run at order 1, to FP64 rounding, with a
    workspace reused by two calls (the second call forms its matrices again)."""
    w = W.poisson_ar1(N=300)
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    xi, un, y = T(w.normals(8)), T(w.uniforms(8)), T(w.y)
    x0 = T(np.log(w.y + 0.5))
    xa, xb = x0.clone(), x0.clone()
    ws = S.Workspace(dev())
    a = S.mh_run(M_dev, y, xa, w.delta, 1, xi, un)
    b1 = S.mh_run(M_dev, y, xb, w.delta, 1, xi[:4], un[:4], ws=ws, reuse_matrices=True)
    lr1 = N_(b1["log_ratio"]).copy()
    b2 = S.mh_run(M_dev, y, xb, w.delta, 1, xi[4:], un[4:], ws=ws, reuse_matrices=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(N_(a["accepted"]),
                                  np.concatenate([N_(b1["accepted"]), N_(b2["accepted"])]))
    np.testing.assert_allclose(np.concatenate([lr1, N_(b2["log_ratio"])]), N_(a["log_ratio"]),
                               rtol=0, atol=1e-9 * 300 * 8)
    np.testing.assert_allclose(N_(xb), N_(xa), rtol=1e-9, atol=1e-10)


def test_rejects_factorised(S):
    w = W.poisson_ar1(N=16)
    M_dev = S.DeviceModel.from_workload(w, device=dev()).diagonal()
    with pytest.raises(ValueError):
        S.mh_run(M_dev, T(w.y), T(np.zeros((16, 8))), w.delta, 1, T(w.normals(1)),
                 T(w.uniforms(1)), factorised=True, reuse_matrices=True)


def test_latent_field_full_size(S):
    """d = 64, N = 4096 (the latent-field benchmark's size), two steps."""
    w = W.latent_field()
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    _follow(S, M_or, M_dev, w.y, w.x_true.copy(), 0.2 * w.delta, w.normals(2), w.uniforms(2))


def test_single_coordinate(S):
    """d = 1 (one active coordinate of a 16-wide team), Student-t, N = 50."""
    rng = np.random.default_rng(55)
    N = 50
    kw = dict(m0=np.zeros(1), P0=np.eye(1), F=np.array([[0.7]]), Q=np.array([[0.4]]), emit=2,
              site=np.array([0], np.int32), nu=3.0, scale=0.5)
    M_or = oracle.Model(**kw)
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw)
    y = rng.standard_normal((N, 1))
    _follow(S, M_or, M_dev, y, 0.3 * rng.standard_normal((N, 1)), 0.6,
            rng.standard_normal((5, 2, N, 1)), rng.random(5))
