"""The GPU sampler targets the right law (MI355X only).

Step parity with the oracle checks each MH step; this checks the chain as a
whole: 256 independent batched chains on N = 2, d = 1 non-Gaussian models
(the same models whose oracle chains are pinned to quadrature), each fed fresh
normals and uniforms between graph-replayed runs, must reproduce the posterior
mean and second moment of (x_0, x_1) from 2-D quadrature within 5 standard
errors (per-chain means as independent batches).  A wrong Hastings ratio or
proposal on the GPU biases the stationary law."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from tests.test_oracle_mh import _quadrature_posterior  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2303_00301_amd import sampler
    return sampler


@pytest.mark.parametrize("emit,order,delta", [(2, 2, 2.0), (3, 2, 1.5), (1, 2, 1.5), (2, 1, 1.0)])
def test_batched_chains_reproduce_quadrature_posterior(S, emit, order, delta):
    dev = torch.device("cuda", 0)
    kw = dict(m0=np.array([0.2]), P0=np.array([[1.0]]), F=np.array([[0.6]]),
              Q=np.array([[0.5]]), emit=emit, b=np.array([0.1]), site=np.array([0], np.int32))
    if emit == 2:
        kw.update(nu=3.0, scale=0.5)
        y = np.array([[2.5], [-1.0]])
    elif emit == 3:
        y = np.array([[2.0], [0.3]])
    else:
        y = np.array([[4.0], [0.0]])
    ref = _quadrature_posterior(oracle.Model(**kw), y)
    n_chains, n_steps, R, burn = 256, 5, 400, 40
    X = torch.zeros((n_chains, 2, 1), dtype=torch.float64, device=dev)
    XI = torch.empty((n_chains, n_steps, 2, 2, 1), dtype=torch.float64, device=dev)
    U = torch.empty((n_chains, n_steps), dtype=torch.float64, device=dev)
    M = S.DeviceModel.from_arrays(2, device=dev, **kw)
    yd = torch.as_tensor(y, dtype=torch.float64, device=dev)
    chains = [dict(model=M, y=yd, x=X[c], xi=XI[c], unif=U[c], delta=delta, order=order)
              for c in range(n_chains)]
    plan = S.BatchPlan(chains, n_steps, block=2)
    gen = torch.Generator(device=dev)
    gen.manual_seed(1000 + 10 * emit + order)
    samples = torch.empty((R, n_chains, 2), dtype=torch.float64, device=dev)
    for r in range(R):
        XI.normal_(generator=gen)
        U.uniform_(generator=gen).clamp_(min=1e-300)
        plan.run(use_graph=True)
        samples[r] = X[:, :, 0]
    torch.cuda.synchronize()
    plan.close()
    s = samples[burn:].cpu().numpy()                    # [R - burn, chains, 2]
    f = np.concatenate([s, s ** 2], axis=2)             # x0, x1, x0^2, x1^2
    per_chain = f.mean(axis=0)                          # [chains, 4]
    est = per_chain.mean(axis=0)
    se = per_chain.std(axis=0, ddof=1) / np.sqrt(n_chains)
    moved = (np.abs(np.diff(s, axis=0)).sum(axis=2) > 0).mean()
    assert 0.05 < moved < 1.0, moved
    z = (est - ref) / se
    assert np.abs(z).max() < 5.0, (z, est, ref)
