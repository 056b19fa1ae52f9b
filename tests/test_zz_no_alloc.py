"""akf_mh_step_noalloc (the MH step on the library's fixed scratch array) against
akf_mh_step (the same step on a caller workspace), through the C ABI.

Two calls in a row on one device share the array; the second is smaller than
the first, so it runs on what the first left behind.  Both entry points run
the same kernels on the same inputs, so the decision, status and accept flag
must agree exactly and every float output to within the FP64 path's own
rounding band (the kernels are deterministic; no reduction order depends on
the workspace address)."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2303_00301_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_2303_00301_amd import sampler
    return sampler


def _dev():
    return torch.device("cuda", 0)


def _T(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=_dev())


def _both(S, w, block=0):
    """One step of each entry point from the same state, normals and uniform."""
    M = S.DeviceModel.from_workload(w, device=_dev())
    xi = _T(w.normals(1)[0])
    un = _T(w.uniforms(1)[:1])
    y, x = _T(w.y), _T(w.x_true)
    ref = S.mh_step(M, y, x, w.delta, w.order, xi, un, block=block)
    out = dict(x_out=torch.empty_like(x),
               log_ratio=torch.empty(1, dtype=torch.float64, device=_dev()),
               logZ_fwd=torch.empty(1, dtype=torch.float64, device=_dev()),
               logZ_rev=torch.empty(1, dtype=torch.float64, device=_dev()),
               accepted=torch.empty(1, dtype=torch.int32, device=_dev()),
               status=torch.empty(1, dtype=torch.int32, device=_dev()))
    S.mh_step_noalloc(M, y, x, w.delta, w.order, xi, un, out["x_out"], out["log_ratio"],
                      out["accepted"], out["logZ_fwd"], out["logZ_rev"], out["status"],
                      block=block)
    torch.cuda.synchronize()
    return ref, out


def _agree(ref, out, label):
    assert int(out["status"].item()) == int(ref["status"].item()) == 0, label
    assert int(out["accepted"].item()) == int(ref["accepted"].item()), label
    for k in ("log_ratio", "logZ_fwd", "logZ_rev"):
        a, b = float(out[k].item()), float(ref[k].item())
        assert abs(a - b) <= REL * max(1.0, abs(b)), (label, k, a, b)
    np.testing.assert_allclose(out["x_out"].cpu().numpy(), ref["x_out"].cpu().numpy(),
                               rtol=REL, atol=REL, err_msg=label)


def test_noalloc_matches_workspace_step_twice_second_smaller(S):
    # first call: latent field d = 64, N = 96 (about 16 MiB of scratch)
    big = W.latent_field(N=96, d=64, n_sites=32)
    print("noalloc: latent_field N=96 d=64", flush=True)
    ref, out = _both(S, big)
    _agree(ref, out, "latent_field N=96 d=64")
    # second call, smaller, on the array the first one left behind
    small = W.poisson_ar1(N=200, d=8)
    print("noalloc: poisson_ar1 N=200 d=8", flush=True)
    ref, out = _both(S, small, block=8)
    _agree(ref, out, "poisson_ar1 N=200 d=8")


def test_noalloc_rejects_a_problem_beyond_its_array(S):
    from paper_2303_00301_amd import _lib
    w = W.latent_field(N=4096, d=64, n_sites=32)
    M = S.DeviceModel.from_workload(w, device=_dev())
    xi = torch.zeros((2, w.N, w.dx), dtype=torch.float64, device=_dev())
    un = torch.full((1,), 0.5, dtype=torch.float64, device=_dev())
    y, x = _T(w.y), _T(w.x_init())
    o = [torch.empty(1, dtype=torch.float64, device=_dev()) for _ in range(3)]
    i = [torch.empty(1, dtype=torch.int32, device=_dev()) for _ in range(2)]
    with pytest.raises(_lib.AkfError, match="AKF_ERR_SHAPE"):
        S.mh_step_noalloc(M, y, x, w.delta, w.order, xi, un, torch.empty_like(x), o[0], i[0],
                          o[1], o[2], i[1])
    lib = _lib.load()
    ms = M.cstruct()
    assert lib.akf_mh_workspace_bytes(C.byref(ms), w.order, 0) > _lib.NOALLOC_SCRATCH_BYTES
