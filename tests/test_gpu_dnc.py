"""GPU parity of the divide-and-conquer path sampler (App. A,
divide-and-conquer strategies; MI355X only).

* pathwise against the oracle's divide-and-conquer sampler (same noise map)
  on bisection trees of several shapes, d from 1 to 64;
* at the benchmark size (d = 64, N = 4096): with zero noise both GPU samplers
  return the smoothing mean (oracle RTS smoother), and the path is affine in
  the noise (x(a + b) - x(0) = x(a) - x(0) + x(b) - x(0)), properties that
  hold at any size.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from tests.test_gpu_parity import MEAN_TOL, N_, T, _stable_model, dev  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2303_00301_amd import sampler
    return sampler


def _moments(rng, N, d):
    m0, P0, F, b, Q = _stable_model(rng, d)
    om = rng.standard_normal((N, d))
    Om = rng.uniform(0.1, 1.0, size=(N, d))
    ref = oracle.kf(m0, P0, F, Q, np.eye(d), np.stack([np.diag(o) for o in Om]), om, b=b,
                    R_per_t=True)
    assert ref["rc"] == 0
    return m0, P0, F, b, Q, ref


@pytest.mark.parametrize("N,d", [(1, 2), (2, 3), (3, 1), (17, 5), (100, 16), (257, 33),
                                 (300, 64), (1000, 8)])
def test_dnc_sample_matches_oracle(S, N, d):
    rng = np.random.default_rng(7000 + N + d)
    m0, P0, F, b, Q, ref = _moments(rng, N, d)
    xi = rng.standard_normal((N, d))
    x_ref, rc = oracle.dnc_sample(F, Q, ref["mf"], ref["Pf"], xi, b=b)
    assert rc == 0
    M = S.DeviceModel.from_arrays(N, m0, P0, F, Q, 1, b=b, device=dev())
    x, st = S.dnc_sample(M, T(ref["mf"]), T(ref["Pf"]), T(xi))
    torch.cuda.synchronize()
    assert int(N_(st)[0]) == 0
    ms, Ps, _, _ = oracle.rts_smooth(F, ref["mf"], ref["Pf"], ref["mp"], ref["Pp"])
    err = np.abs(N_(x) - x_ref) / np.sqrt(np.einsum("tii->ti", Ps))
    assert err.max() < MEAN_TOL, err.max()


def test_dnc_full_size_mean_and_linearity(S):
    """d = 64, N = 4096: zero noise gives the smoothing mean on both GPU
    samplers; the noise map is affine."""
    rng = np.random.default_rng(7100)
    N, d = 4096, 64
    m0, P0, F, b, Q, ref = _moments(rng, N, d)
    ms, Ps, _, _ = oracle.rts_smooth(F, ref["mf"], ref["Pf"], ref["mp"], ref["Pp"])
    M = S.DeviceModel.from_arrays(N, m0, P0, F, Q, 1, b=b, device=dev())
    mf, Pf = T(ref["mf"]), T(ref["Pf"])
    sd = np.sqrt(np.einsum("tii->ti", Ps))
    z = T(np.zeros((N, d)))
    x0, st = S.dnc_sample(M, mf, Pf, z)
    r0, st2 = S.rts_sample(M, mf, Pf, z)
    a, b_ = rng.standard_normal((2, N, d))
    xa, _ = S.dnc_sample(M, mf, Pf, T(a))
    xb, _ = S.dnc_sample(M, mf, Pf, T(b_))
    xab, _ = S.dnc_sample(M, mf, Pf, T(a + b_))
    torch.cuda.synchronize()
    assert int(N_(st)[0]) == 0 and int(N_(st2)[0]) == 0
    assert (np.abs(N_(x0) - ms) / sd).max() < MEAN_TOL
    assert (np.abs(N_(r0) - ms) / sd).max() < MEAN_TOL
    lin = N_(xab) - N_(x0) - (N_(xa) - N_(x0)) - (N_(xb) - N_(x0))
    assert (np.abs(lin) / sd).max() < MEAN_TOL
