"""GPU parity of order 3, the proposal built on the observation model's
linearisation (eq. observation-approx: h_t replaced around the path by the
Gaussian N(H_t z + c_t, R_t) of the statistical linear regression of eq. coeffs
with the moments of eq. general-GSLR-coeffs; eq. two-lin-prop), against the
oracle's order-3 step, with the bounds of test_gpu_parity.

Cases: quadratic-mean Gaussian observations with several sites on one latent
and unobserved (NaN) sites, at the Taylor limit and at positive reference
variances, d from 1 to 40 with ragged blocks; Gaussian-at-sites observations,
where the regression is exact and order 3 must equal order 2; and the full-size
quadratic-observation field (d = 64, N = 4096) in the benchmark's launch
configuration."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2303_00301_amd import workloads as W  # noqa: E402
from tests.test_gpu_parity import S, T, N_, dev, _compare_step, MEAN_TOL  # noqa: E402,F401

pytestmark = pytest.mark.gpu


def _quad_kw(rng, dx, site, beta, scale, g2):
    G = rng.standard_normal((dx, dx))
    F = 0.7 * G / max(1e-12, np.max(np.abs(np.linalg.eigvals(G))))
    A = rng.standard_normal((dx, dx))
    Q = A @ A.T / dx + 0.2 * np.eye(dx)
    return dict(m0=0.2 * rng.standard_normal(dx), P0=np.eye(dx), F=F, Q=Q,
                emit=W.EMIT_GAUSS_QUAD, b=0.1 * rng.standard_normal(dx),
                site=np.asarray(site, np.int32), scale=scale, obs_beta=beta, slr_var=g2)


def _simulate_obs(rng, kw, N, nan_frac=0.1):
    """A path from the prior and observations from the quadratic family, with a
    fraction of the entries unobserved."""
    dx = kw["m0"].shape[0]
    L = np.linalg.cholesky(kw["Q"])
    x = np.zeros((N, dx))
    x[0] = kw["m0"] + rng.standard_normal(dx)
    for t in range(1, N):
        x[t] = kw["F"] @ x[t - 1] + kw["b"] + L @ rng.standard_normal(dx)
    z = x[:, kw["site"]]
    y = z + kw["obs_beta"] * z * z + kw["scale"] * rng.standard_normal(z.shape)
    y[rng.random(y.shape) < nan_frac] = np.nan
    return x, y


QUAD_CASES = [
    # N, dx, sites, beta, scale, g2, delta, block
    (37, 3, [0, 2, 2, 1], 0.35, 0.6, 0.0, 0.3, 0),
    (37, 3, [0, 2, 2, 1], 0.35, 0.6, 0.3, 0.3, 4),
    (1, 1, [0, 0, 0], -0.4, 0.5, 0.2, 0.5, 0),
    (200, 16, list(range(0, 16, 2)) + [0, 0, 4], 0.2, 0.5, 0.1, 0.2, 0),
    (129, 40, list(range(0, 40, 3)) + [3, 9, 9], -0.3, 0.4, 0.2, 0.1, 7),
]


@pytest.mark.parametrize("N,dx,sites,beta,scale,g2,delta,block", QUAD_CASES)
def test_quadratic_observations_order3_steps(S, N, dx, sites, beta, scale, g2, delta, block):
    rng = np.random.default_rng(7000 + 13 * N + dx)
    kw = _quad_kw(rng, dx, sites, beta, scale, g2)
    x_true, y = _simulate_obs(rng, kw, N)
    M_or = oracle.Model(**kw)
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw)
    x = x_true + 0.05 * rng.standard_normal(x_true.shape)
    for _ in range(3):
        xi = rng.standard_normal((2, N, dx))
        r = _compare_step(S, M_or, M_dev, y, x, delta, 3, xi, float(rng.random()), block=block)
        x = r["x_out"]


def test_gaussian_sites_order3_equals_order2(S):
    """Gaussian-at-sites observations have a linear mean: the regression is
    exact whatever the reference variance, so the order-3 step is the order-2
    step (same kernels, same arithmetic, up to rounding of the two formulas)."""
    rng = np.random.default_rng(71)
    N, dx = 150, 12
    kw = _quad_kw(rng, dx, [0, 3, 3, 7, 11], 0.0, 0.7, 0.4)
    kw["emit"] = W.EMIT_GAUSS_SITE
    _, y = _simulate_obs(rng, kw, N, nan_frac=0.2)
    M_or = oracle.Model(**kw)
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw)
    x = 0.1 * rng.standard_normal((N, dx))
    for _ in range(3):
        xi = rng.standard_normal((2, N, dx))
        un = float(rng.random())
        r = _compare_step(S, M_or, M_dev, y, x, 0.3, 3, xi, un)
        o2 = S.mh_step(M_dev, T(y), T(x), 0.3, 2, T(xi), T([un]))
        o3 = S.mh_step(M_dev, T(y), T(x), 0.3, 3, T(xi), T([un]))
        torch.cuda.synchronize()
        assert int(N_(o2["accepted"])[0]) == int(N_(o3["accepted"])[0])
        for k in ("log_ratio", "logZ_fwd", "logZ_rev"):
            a, b = float(N_(o3[k])[0]), float(N_(o2[k])[0])
            assert abs(a - b) <= 1e-10 * max(1.0, abs(b)), (k, a, b)
        np.testing.assert_allclose(N_(o3["x_out"]), N_(o2["x_out"]), rtol=1e-10, atol=1e-12)
        x = r["x_out"]


def test_quadratic_field_full_size(S):
    """d = 64, N = 4096, 32 sites with a quadratic mean, order 3 with a positive
    reference variance, in the benchmark's launch configuration: one step from
    near the simulated path, and one whose uniform forces acceptance so that
    x* is compared element by element, scaled by the forward auxiliary model's
    smoothing standard deviations."""
    w = W.quadratic_obs_field()
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    xi = w.normals(2)
    un = w.uniforms(1)
    x = w.x_true.copy()
    _compare_step(S, M_or, M_dev, w.y, x, w.delta, 3, xi[0], un[0])
    r = _compare_step(S, M_or, M_dev, w.y, x, w.delta, 3, xi[1], 1e-300)
    assert r["status"] == 0 and r["accepted"] == 1
    u = x + np.sqrt(w.delta / 2) * xi[1][0]
    om, Om, _, rc = oracle.linearise(M_or, w.y, x, u, w.delta, 3)
    assert rc == 0
    kf = oracle.kf(w.m0, w.P0, w.F, w.Q, np.eye(w.dx), Om, om, b=w.b, R_per_t=True)
    _, Ps, _, _ = oracle.rts_smooth(w.F, kf["mf"], kf["Pf"], kf["mp"], kf["Pp"])
    out = S.mh_step(M_dev, T(w.y), T(x), w.delta, 3, T(xi[1]), T([1e-300]))
    torch.cuda.synchronize()
    err = np.abs(N_(out["x_out"]) - r["xstar"]) / np.sqrt(np.einsum("tii->ti", Ps))
    assert err.max() < MEAN_TOL, err.max()
