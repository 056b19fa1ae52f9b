"""GPU parity of the factorised step (dx scalar filters and samplers) and of
the multivariate-t emission (MI355X only).

The factorised step is compared with the oracle's factorised step (itself
pinned to the dense oracle step on the CPU) step by step from the oracle's
state, at the spatio-temporal workload's full size (8 x 8 lattice, T = 1024)
and on ragged sizes that leave idle threads, span several time chunks and
reduce to one step or one coordinate.  The dense GPU path with the
multivariate-t emission is compared with the dense oracle, and the two GPU
paths with each other.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2303_00301_amd import workloads as W  # noqa: E402
from tests.test_gpu_parity import N_, T, _compare_step, dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2303_00301_amd import sampler
    return sampler


def _diag_model(emit, N, d, rng, dy=None):
    dy = dy or d
    kw = dict(m0=0.3 * rng.standard_normal(d), P0=np.diag(rng.uniform(0.5, 1.5, d)),
              F=np.diag(rng.uniform(0.5, 1.0, d)), Q=np.diag(rng.uniform(0.2, 1.0, d)), emit=emit,
              b=0.1 * rng.standard_normal(d), site=rng.integers(0, d, size=dy).astype(np.int32))
    if emit == 2:
        kw.update(nu=3.0, scale=0.5)
    if emit == 4:
        C = rng.standard_normal((dy, dy))
        kw.update(nu=1.5, R=C @ C.T / dy + 0.5 * np.eye(dy))
    if emit == 1:
        y = rng.poisson(1.5, size=(N, dy)).astype(float)
    else:
        y = 1.5 * rng.standard_normal((N, dy))
    return kw, y


def test_spatio_temporal_full_size_steps(S):
    """8 x 8 lattice, T = 1024, multivariate t (nu = 1), first order: three
    chained steps of the factorised GPU step against the factorised oracle."""
    w = W.spatio_temporal()
    M_or = oracle.Model(**w.oracle_kwargs())
    M_dev = S.DeviceModel.from_workload(w, device=dev()).diagonal()
    xi = w.normals(3)
    un = w.uniforms(3)
    x = w.x_true.copy()
    for k in range(3):
        r = _compare_step(S, M_or, M_dev, w.y, x, w.delta, 1, xi[k], un[k], factorised=True)
        x = r["x_out"]


# (emission, order, N, d)
FACT_CASES = [(4, 1, 1, 1), (4, 1, 3, 1), (1, 1, 5, 3), (2, 2, 255, 3), (4, 1, 257, 64),
              (1, 2, 3000, 6), (3, 2, 4099, 3), (4, 1, 700, 33), (2, 1, 129, 64)]


@pytest.mark.parametrize("emit,order,N,d", FACT_CASES)
def test_factorised_steps_ragged(S, emit, order, N, d):
    """Ragged N (idle threads, one step, several 2048-step chunks) and d (one
    coordinate up to 64), every non-Gaussian family, both orders where defined."""
    rng = np.random.default_rng(5000 + 13 * N + d + emit)
    kw, y = _diag_model(emit, N, d, rng, dy=max(1, d - 1) if d > 2 else d)
    M_or = oracle.Model(**kw)
    M_dev = S.DeviceModel.from_arrays(N, device=dev(), **kw).diagonal()
    x = 0.3 * rng.standard_normal((N, d))
    if emit == 1:
        x = x + np.log(1.5)
    for k in range(2):
        xi = rng.standard_normal((2, N, d))
        r = _compare_step(S, M_or, M_dev, y, x, 0.3, order, xi, float(rng.random()),
                          factorised=True)
        x = r["x_out"]


@pytest.mark.parametrize("N,d", [(40, 16), (97, 64)])
def test_dense_path_multivariate_t(S, N, d):
    """The dense GPU step with the multivariate-t emission (first order)
    against the dense oracle, on a coupled prior."""
    rng = np.random.default_rng(6000 + N + d)
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
    x = 0.5 * rng.standard_normal((N, d))
    for k in range(2):
        xi = rng.standard_normal((2, N, d))
        r = _compare_step(S, M_or, M_dev, y, x, 0.05, 1, xi, float(rng.random()))
        x = r["x_out"]


def test_factorised_equals_dense_gpu(S):
    """Both GPU paths on the spatio-temporal model (shortened to T = 300): same
    x*, log Z and log r within FP64 rounding."""
    w = W.spatio_temporal(N=300)
    M_dense = S.DeviceModel.from_workload(w, device=dev())
    M_fact = M_dense.diagonal()
    xi = T(w.normals(1)[0])
    un = T(w.uniforms(1))
    x = T(w.x_true)
    a = S.mh_step(M_dense, T(w.y), x, w.delta, 1, xi, un)
    b = S.mh_step(M_fact, T(w.y), x, w.delta, 1, xi, un, factorised=True)
    torch.cuda.synchronize()
    assert int(N_(a["status"])[0]) == 0 and int(N_(b["status"])[0]) == 0
    for k in ("log_ratio", "logZ_fwd", "logZ_rev"):
        va, vb = float(N_(a[k])[0]), float(N_(b[k])[0])
        assert abs(va - vb) <= 1e-9 * 300 * 64 + 1e-9 * max(1.0, abs(va)), (k, va, vb)


def test_factorised_rejections(S):
    w = W.spatio_temporal(N=8, side=2)
    M = S.DeviceModel.from_workload(w, device=dev())
    Md = M.diagonal()
    xi = T(w.normals(1)[0])
    un = T(w.uniforms(1))
    x = T(w.x_true)
    from paper_2303_00301_amd._lib import AkfError
    with pytest.raises(AkfError, match="first-order proposals only"):
        S.mh_step(Md, T(w.y), x, w.delta, 2, xi, un, factorised=True)
    with pytest.raises(AkfError, match="first-order proposals only"):
        S.mh_step(M, T(w.y), x, w.delta, 2, xi, un)
    with pytest.raises(AkfError):
        S.mh_step(M, T(w.y), x, w.delta, 1, xi, un, factorised=True)
    Mc = S.DeviceModel.from_arrays(8, w.m0, w.P0, w.F + 0.01, w.Q, 4, R=w.R, site=w.site,
                                   nu=1.0, device=dev())
    with pytest.raises(AkfError, match="not diagonal"):
        Mc.diagonal()
