"""GPU parity of the MH step with nonlinear dynamics (extended linearisation
of Lorenz-63 / Lorenz-96 Euler steps, per-step F_t, b_t in the filter and
sampler, dynamics-mismatch terms in log r) and of the Gaussian-at-sites
emission with unobserved (NaN) sites, against the FP64 oracle (MI355X only).
Steps are compared one at a time from the oracle's state."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2303_00301_amd import workloads as W  # noqa: E402
from tests.test_gpu_parity import T, _compare_step, dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2303_00301_amd import sampler
    return sampler


@pytest.mark.parametrize("delta,block", [(1.0, 0), (1e4, 0), (1.0, 37)])
def test_lorenz63_full_size_steps(S, delta, block):
    """Lorenz-63 SDE on the 2e-4 grid over [0, 2] (N = 10001), x_2, x_3 observed
    every 50 steps: three chained second-order steps against the oracle."""
    w = W.lorenz63()
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    xi = w.normals(3)
    un = w.uniforms(3)
    x = w.x_true.copy()
    for k in range(3):
        r = _compare_step(S, M_or, M_dev, w.y, x, delta, 2, xi[k], un[k], block=block)
        x = r["x_out"]


def test_lorenz63_from_prior_start(S):
    """From the prior-simulated start (far from the posterior), first order."""
    w = W.lorenz63(N=3001)
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    xi = w.normals(2)
    un = w.uniforms(2)
    x = w.extra["x_start"].copy()
    for k in range(2):
        r = _compare_step(S, M_or, M_dev, w.y, x, 0.1, 1, xi[k], un[k])
        x = r["x_out"]


@pytest.mark.parametrize("N,d,order,block", [(37, 5, 2, 4), (130, 17, 1, 0), (64, 33, 2, 5),
                                             (2048, 40, 2, 0)])
def test_lorenz96_steps(S, N, d, order, block):
    """Lorenz-96 on rings of 5 to 40 coordinates (team sizes 16, 32, 64),
    Student-t observations of every other coordinate."""
    w = W.lorenz96(N=N, d=d, n_sites=max(1, d // 2))
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev())
    xi = w.normals(2)
    un = w.uniforms(2)
    x = w.x_true.copy()
    for k in range(2):
        r = _compare_step(S, M_or, M_dev, w.y, x, w.delta, order, xi[k], un[k], block=block)
        x = r["x_out"]


def test_gauss_site_linear_dynamics_exact(S):
    """Gaussian at sites with NaN gaps and linear dynamics: order 2 is exact, so
    every step accepts with |log r| ~ 0 on the GPU too."""
    rng = np.random.default_rng(12)
    N, d = 200, 6
    kw = dict(m0=np.zeros(d), P0=np.eye(d), F=0.9 * np.eye(d) + 0.02, Q=0.3 * np.eye(d), emit=5,
              site=np.array([0, 2, 5], np.int32), scale=1.5)
    y = rng.standard_normal((N, 3))
    y[rng.random((N, 3)) < 0.4] = np.nan
    M_or = oracle.Model(**kw)
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw)
    x = rng.standard_normal((N, d))
    for k in range(3):
        xi = rng.standard_normal((2, N, d))
        r = _compare_step(S, M_or, M_dev, y, x, 0.5, 2, xi, float(rng.random()))
        assert r["accepted"] == 1 and abs(r["log_ratio"]) < 1e-9
        x = r["x_out"]


def test_nonlinear_dynamics_rejections(S):
    from paper_2303_00301_amd._lib import AkfError
    w = W.lorenz63(N=20)
    M = S.DeviceModel.from_workload(w, device=dev())
    om = T(np.zeros((20, 3)))
    with pytest.raises(AkfError, match="linear dynamics"):
        S.aux_filter(M, om, T(np.ones((20, 3))))
