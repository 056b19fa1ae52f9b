"""GPU parity of order-2 runs that reuse the auxiliary model's matrices after
rejected steps (akf_mh_run_reuse) against the FP64 oracle.

Under second-order proposals Omega_t depends on x only, so after a rejection
the next forward proposal (same x, new u) has the covariances of the forward
proposal before it; the oracle's plain step re-forms them every time and must
give the same chain.  The GPU runs a whole chain in one call; the oracle
follows it step by step from the same state, taking the GPU's accept decision
only inside the tie band of the stated log-ratio tolerance.  Every case checks
that the chain rejected at least once before its last step, so that a kept
forward proposal ran.
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
    """Run the order-2 chain on the GPU in one call; replay it on the oracle.
    Returns the GPU's accept flags."""
    n = xi.shape[0]
    x_gpu = T(x0)
    out = S.mh_run(M_dev, T(y), x_gpu, delta, 2, T(xi), T(un), block=block, reuse_matrices=True)
    torch.cuda.synchronize()
    st, acc = N_(out["status"]), N_(out["accepted"])
    lr, lzf, lzr = N_(out["log_ratio"]), N_(out["logZ_fwd"]), N_(out["logZ_rev"])
    N, d = x0.shape
    x = x0.copy()
    for k in range(n):
        r = oracle.mh_step(M_or, y, x, delta, 2, xi[k][0], xi[k][1], float(un[k]))
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
    np.testing.assert_allclose(N_(x_gpu), x, rtol=1e-7, atol=1e-8)
    return acc


def _rejected_before_last(acc):
    return bool(np.any(acc[:-1] == 0))


@pytest.mark.parametrize("N,block", [(200, 0), (37, 5)])
def test_poisson_chain(S, N, block):
    """d = 8 Poisson log-link (diagonal Hessian), ragged scan blocks; a large
    delta makes rejections frequent."""
    w = W.poisson_ar1(N=N)
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    acc = _follow(S, M_or, M_dev, w.y, np.log(w.y + 0.5), 4.0 * w.delta, w.normals(6),
                  w.uniforms(6), block=block)
    assert _rejected_before_last(acc)


@pytest.mark.parametrize("N,block,scale", [(301, 16, 3.0), (64, 1, 10.0)])
def test_latent_field_chain(S, N, block, scale):
    """d = 64, Student-t at sites, a multiple of the benchmark's delta (chosen so
    that the oracle's chain rejects before its last step)."""
    w = W.latent_field(N=N)
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    x0 = w.x_true + 0.05 * np.random.default_rng(2).standard_normal(w.x_true.shape)
    acc = _follow(S, M_or, M_dev, w.y, x0, scale * w.delta, w.normals(6), w.uniforms(6),
                  block=block)
    assert _rejected_before_last(acc)


def test_stoch_vol_chain(S):
    """d = 30 (padded to 32), stochastic volatility, T = 250."""
    w = W.stoch_vol(order=2)
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    acc = _follow(S, M_or, M_dev, w.y, w.x_true.copy(), 2.0 * w.delta, w.normals(8),
                  w.uniforms(8))
    assert _rejected_before_last(acc)


def test_single_step_series(S):
    """N = 1 (no scan tree): every step's kept forward proposal is one team."""
    w = W.poisson_ar1(N=1)
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    _follow(S, M_or, M_dev, w.y, np.log(w.y + 0.5), 2.0, w.normals(6), w.uniforms(6))


def test_matches_plain_run(S):
    """The same chain as akf_mh_run at order 2, to FP64 rounding: the same accept
    decisions, log ratios and final path."""
    w = W.latent_field(N=512)
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    xi, un, y = T(w.normals(10)), T(w.uniforms(10)), T(w.y)
    x0 = T(w.x_true)
    xa, xb = x0.clone(), x0.clone()
    a = S.mh_run(M_dev, y, xa, 2.0 * w.delta, 2, xi, un)
    b = S.mh_run(M_dev, y, xb, 2.0 * w.delta, 2, xi, un, reuse_matrices=True)
    torch.cuda.synchronize()
    acc = N_(a["accepted"])
    assert _rejected_before_last(acc) and acc.sum() >= 1
    np.testing.assert_array_equal(N_(b["accepted"]), acc)
    np.testing.assert_array_equal(N_(b["status"]), N_(a["status"]))
    np.testing.assert_allclose(N_(b["log_ratio"]), N_(a["log_ratio"]), rtol=0,
                               atol=LR_TOL_PER_TD * 512 * 64)
    # the kept and the plain sampler round differently; the bar of the oracle
    # comparisons
    np.testing.assert_allclose(N_(xb), N_(xa), rtol=1e-7, atol=1e-8)


def test_rejects_gaussian_order2(S):
    rng = np.random.default_rng(3)
    N, dx, dy = 20, 4, 2
    kw = dict(m0=np.zeros(dx), P0=np.eye(dx), F=0.5 * np.eye(dx), Q=np.eye(dx), emit=0,
              H=rng.standard_normal((dy, dx)), R=np.eye(dy))
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw)
    with pytest.raises(Exception, match="dense Omega"):
        S.mh_run(M_dev, T(np.zeros((N, dy))), T(np.zeros((N, dx))), 0.5, 2,
                 T(rng.standard_normal((1, 2, N, dx))), T([0.5]), reuse_matrices=True)


def test_latent_field_full_size(S):
    """d = 64, N = 4096 (the benchmark's workload and launch configuration),
    four steps with a rejection before the last."""
    w = W.latent_field()
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    acc = _follow(S, M_or, M_dev, w.y, w.x_true.copy(), 3.0 * w.delta, w.normals(4),
                  w.uniforms(4))
    assert _rejected_before_last(acc)


def test_single_coordinate(S):
    """d = 1 (one active coordinate of a 16-wide team), Student-t, N = 50; the
    oracle's chain rejects six steps, then accepts one."""
    rng = np.random.default_rng(56)
    N = 50
    kw = dict(m0=np.zeros(1), P0=np.eye(1), F=np.array([[0.7]]), Q=np.array([[0.4]]), emit=2,
              site=np.array([0], np.int32), nu=3.0, scale=0.5)
    M_or = oracle.Model(**kw)
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw)
    y = rng.standard_normal((N, 1))
    _follow(S, M_or, M_dev, y, 0.3 * rng.standard_normal((N, 1)), 0.1,
            rng.standard_normal((8, 2, N, 1)), rng.random(8))


def test_reuse_run_graph_replay_matches_eager(S):
    """The reuse run decides its branch on the device, so a K-step call can be
    captured in a graph: replays with fresh normals (one of them accepting
    every step, one rejecting every step) equal eager calls from the same start,
    bit for bit, with eager work and host synchronisations between replays."""
    w = W.latent_field(N=96)
    M = S.DeviceModel.from_workload(w, device=dev())
    y = T(w.y)
    K = 4
    gen = torch.Generator(device=dev())
    gen.manual_seed(17)
    xi = torch.empty((K, 2, w.N, w.dx), dtype=torch.float64, device=dev())
    un = torch.empty((K,), dtype=torch.float64, device=dev())
    ws = S.Workspace(dev())
    x_cap = T(w.x_true)
    xi.normal_(generator=gen)
    un.uniform_(generator=gen)
    delta = 2.0 * w.delta
    S.mh_run(M, y, x_cap, delta, 2, xi, un, ws=ws, reuse_matrices=True)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = S.mh_run(M, y, x_cap, delta, 2, xi, un, ws=ws, reuse_matrices=True)
    torch.cuda.synchronize()
    x = T(w.x_true)
    rejected = False
    for rep in range(5):
        xi.normal_(generator=gen)
        un.uniform_(generator=gen)
        un.clamp_(min=1e-300)
        if rep == 2:
            un.fill_(1e-300)  # accepts unless a proposal fails
        if rep == 3:
            un.fill_(1.0)  # log U = 0: rejects unless log r > 0
        start = x.clone()
        x_cap.copy_(start)
        g.replay()
        torch.cuda.synchronize()
        eager = S.mh_run(M, y, x, delta, 2, xi, un, ws=ws, reuse_matrices=True)
        torch.cuda.synchronize()
        assert torch.equal(x_cap, x), rep
        for k in ("log_ratio", "accepted", "logZ_fwd", "logZ_rev", "status"):
            assert torch.equal(out[k], eager[k]), (rep, k)
        acc = N_(eager["accepted"])
        rejected = rejected or bool(np.any(acc[:-1] == 0))
    assert rejected
