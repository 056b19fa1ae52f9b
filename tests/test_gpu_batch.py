"""Batched chains on the GPU (MI355X only): the batched persistent launches
(eager and hipGraph replay) give the same per-chain results as plain per-chain
runs with the same block size, normals and uniforms; the autotuner writes and
reuses its cache.

Batched chains scan their block elements with the work-efficient up/down
tree, a single chain with the Hillis-Steele scan; the two associate the
combines differently, so they agree to FP64 rounding (not bit for bit), and
the accept decisions agree away from ties."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2303_00301_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


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


def _chains(S, ws, n_steps):
    out = []
    for k, w in enumerate(ws):
        x0 = np.log(w.y + 0.5)
        out.append(dict(model=S.DeviceModel.from_workload(w, device=dev()), y=T(w.y), x=T(x0),
                        x0=x0, xi=T(w.normals(n_steps)), unif=T(w.uniforms(n_steps)),
                        delta=w.delta, order=2,
                        log_ratio=torch.empty(n_steps, dtype=torch.float64, device=dev()),
                        accepted=torch.empty(n_steps, dtype=torch.int32, device=dev()),
                        logZ_fwd=torch.empty(n_steps, dtype=torch.float64, device=dev()),
                        logZ_rev=torch.empty(n_steps, dtype=torch.float64, device=dev()),
                        status=torch.empty(n_steps, dtype=torch.int32, device=dev())))
    return out


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_equals_plain_per_chain(S, use_graph):
    ws = W.ragged_poisson_batch(n_chains=10, n_min=5, n_max=300, seed=9)
    n_steps = 3
    chains = _chains(S, ws, n_steps)
    plan = S.BatchPlan(chains, n_steps, block=8)
    info = plan.info()
    assert {c["D"] for c in info["classes"]} <= {16, 32}
    plan.run(use_graph=use_graph)
    torch.cuda.synchronize()
    for c in chains:
        x = T(c["x0"])
        ref = S.mh_run(c["model"], c["y"], x, c["delta"], 2, c["xi"], c["unif"], block=8)
        torch.cuda.synchronize()
        assert torch.equal(c["status"], ref["status"])
        assert torch.equal(c["accepted"], ref["accepted"])
        torch.testing.assert_close(c["x"], x, rtol=1e-9, atol=1e-11)
        for k in ("log_ratio", "logZ_fwd", "logZ_rev"):
            torch.testing.assert_close(c[k], ref[k], rtol=1e-9, atol=1e-9, msg=k)
    plan.close()


def test_batched_first_step_matches_oracle(S):
    ws = W.ragged_poisson_batch(n_chains=4, n_min=20, n_max=120, seed=3)
    chains = _chains(S, ws, 1)
    plan = S.BatchPlan(chains, 1, block=5)
    plan.run()
    torch.cuda.synchronize()
    for w, c in zip(ws, chains):
        M = oracle.Model(**w.oracle_kwargs())
        xi = w.normals(1)[0]
        r = oracle.mh_step(M, w.y, c["x0"], w.delta, 2, xi[0], xi[1], w.uniforms(1)[0])
        assert int(c["status"].item()) == r["status"]
        assert abs(c["log_ratio"].item() - r["log_ratio"]) < 1e-7 * max(1, abs(r["log_ratio"]))
        np.testing.assert_allclose(c["x"].cpu().numpy(), r["x_out"], rtol=1e-7, atol=1e-8)
    plan.close()


def test_graph_replays_match_eager(S):
    ws = W.ragged_poisson_batch(n_chains=6, n_min=30, n_max=200, seed=4)
    n_steps = 4
    a = _chains(S, ws, n_steps)
    b = _chains(S, ws, n_steps)
    pa = S.BatchPlan(a, n_steps, block=16)
    pb = S.BatchPlan(b, n_steps, block=16)
    pa.run(use_graph=False)
    pb.run(use_graph=True)
    torch.cuda.synchronize()
    for ca, cb in zip(a, b):
        assert torch.equal(ca["x"], cb["x"])
        assert torch.equal(ca["log_ratio"], cb["log_ratio"])
    # a second replay of the same graph continues the chains like eager steps do
    pa.run(use_graph=False)
    pb.run(use_graph=True)
    torch.cuda.synchronize()
    for ca, cb in zip(a, b):
        assert torch.equal(ca["x"], cb["x"])
    pa.close()
    pb.close()


def test_autotuner_cache(S, tmp_path):
    ws = W.ragged_poisson_batch(n_chains=5, n_min=50, n_max=400, seed=6)
    chains = _chains(S, ws, 1)
    cache = str(tmp_path / "tune.jsonl")
    p1 = S.BatchPlan(chains, 1, block=0, tune_cache=cache)
    i1 = p1.info()
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == len(i1["classes"])
    p2 = S.BatchPlan(chains, 1, block=0, tune_cache=cache)
    assert [c["block"] for c in p2.info()["classes"]] == [c["block"] for c in i1["classes"]]
    assert len(open(cache).read().strip().splitlines()) == len(lines)
    p1.close()
    p2.close()


def test_batch_with_every_team_width(S):
    """Chains of d = 8, 20 and 64 in one batch (all three team widths): every
    chain equals its own akf_mh_run, and the first step of the d = 64 chain
    equals the oracle's."""
    ws = W.ragged_poisson_batch(n_chains=6, n_min=40, n_max=120, dims=(8, 20, 64), seed=13)
    assert {w.dx for w in ws} == {8, 20, 64}
    n_steps = 2
    chains = _chains(S, ws, n_steps)
    plan = S.BatchPlan(chains, n_steps, block=8)
    assert {c["D"] for c in plan.info()["classes"]} == {16, 32, 64}
    plan.run(use_graph=True)
    torch.cuda.synchronize()
    for c in chains:
        x = T(c["x0"])
        ref = S.mh_run(c["model"], c["y"], x, c["delta"], 2, c["xi"], c["unif"], block=8)
        torch.cuda.synchronize()
        assert torch.equal(c["status"], ref["status"])
        assert torch.equal(c["accepted"], ref["accepted"])
        torch.testing.assert_close(c["x"], x, rtol=1e-9, atol=1e-11)
        for k in ("log_ratio", "logZ_fwd", "logZ_rev"):
            torch.testing.assert_close(c[k], ref[k], rtol=1e-9, atol=1e-9, msg=k)
    plan.close()
    k64 = next(k for k, w in enumerate(ws) if w.dx == 64)
    w = ws[k64]
    xi = w.normals(n_steps)
    r = oracle.mh_step(oracle.Model(**w.oracle_kwargs()), w.y, np.log(w.y + 0.5), w.delta, 2,
                       xi[0][0], xi[0][1], float(w.uniforms(n_steps)[0]))
    assert int(chains[k64]["status"].cpu()[0]) == r["status"]
    lr = float(chains[k64]["log_ratio"].cpu()[0])
    assert abs(lr - r["log_ratio"]) <= 1e-9 * w.N * w.dx + 1e-9 * max(1.0, abs(r["log_ratio"]))
