"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/akf.h declares, sizes workspaces, and rejects bad
arguments before touching device memory."""
import ctypes as C
import os
import re

import pytest

from paper_2303_00301_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "akf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(akf_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), (set(names) ^ set(_lib.SIGNATURES))


def _fake_model(N=16, dx=4, dy=4, emit=1):
    m = _lib.AkfModel()
    m.N, m.dx, m.dy = N, dx, dy
    fake = 0x1000
    m.m0 = m.P0 = m.F = m.Q = fake
    m.b = None
    m.emit = emit
    m.H = m.R = fake
    m.site = fake
    m.nu, m.scale = 3.0, 0.5
    return m


def test_workspace_sizes_grow_with_problem():
    lib = _lib.load()
    small = lib.akf_mh_workspace_bytes(C.byref(_fake_model(N=64, dx=8)), 2, 0)
    big = lib.akf_mh_workspace_bytes(C.byref(_fake_model(N=4096, dx=64)), 2, 0)
    assert 0 < small < big
    assert lib.akf_mh_workspace_bytes(C.byref(_fake_model(dx=65)), 2, 0) == 0
    assert lib.akf_mh_workspace_bytes(C.byref(_fake_model()), 3, 0) == 0
    assert lib.akf_filter_workspace_bytes(C.byref(_fake_model(N=100, dx=3)), 0) > 0
    assert lib.akf_sampler_workspace_bytes(C.byref(_fake_model(N=100, dx=3)), 7) > 0


@pytest.mark.parametrize("field,value,code", [
    ("N", 0, 2), ("dx", 0, 2), ("dx", 65, 2), ("dy", 0, 2), ("emit", 9, 1),
])
def test_mh_step_rejects_bad_model(field, value, code):
    lib = _lib.load()
    m = _fake_model()
    setattr(m, field, value)
    p = C.c_void_p(0x2000)
    rc = lib.akf_mh_step(C.byref(m), p, p, 0.5, 2, p, p, p, None, None, None, None, None,
                         C.c_void_p(0x10000), 1 << 30, 0, None)
    assert rc == code
    assert lib.akf_last_error()


def test_order3_validation():
    """Order 3 (the observation model's linearisation) is accepted for the
    Gaussian-around-a-mean families only, with a finite reference variance >= 0,
    and only by the plain step and run; the quadratic family needs a finite
    obs_beta and scale > 0."""
    lib = _lib.load()
    q = _fake_model(emit=6)
    q.scale, q.obs_beta, q.slr_var = 0.5, 0.3, 0.1
    assert lib.akf_mh_workspace_bytes(C.byref(q), 3, 0) > 0
    assert lib.akf_mh_workspace_bytes(C.byref(q), 2, 0) > 0
    g = _fake_model(emit=5)
    assert lib.akf_mh_workspace_bytes(C.byref(g), 3, 0) > 0
    for emit in (0, 1, 2, 3, 4):
        assert lib.akf_mh_workspace_bytes(C.byref(_fake_model(emit=emit)), 3, 0) == 0
    p = C.c_void_p(0x2000)
    ws = C.c_void_p(0x10000)
    step = lambda m, order=3: lib.akf_mh_step(C.byref(m), p, p, 0.5, order, p, p, p, None, None,
                                              None, None, None, ws, 1 << 30, 0, None)
    q.slr_var = -0.1
    assert step(q) == 1
    q.slr_var = float("inf")
    assert step(q) == 1
    q.slr_var, q.obs_beta = 0.1, float("nan")
    assert step(q) == 1
    q.obs_beta, q.scale = 0.3, 0.0
    assert step(q) == 1
    q.scale = 0.5
    assert lib.akf_mh_reuse_workspace_bytes(C.byref(q), 3, 0) == 0
    assert lib.akf_mh_factorised_workspace_bytes(C.byref(q), 3) == 0


def test_sqrt_filter_validation():
    """The square-root filter takes AKF_F32 and AKF_F64 (its FP32 workspace is
    smaller), dx <= 32 and linear dynamics; the covariance-form entry points
    still reject AKF_F32."""
    lib = _lib.load()
    m = _fake_model(N=250, dx=30, dy=30)
    m.dtype = _lib.AKF_F64
    b64 = lib.akf_sqrt_workspace_bytes(C.byref(m), 0)
    m.dtype = _lib.AKF_F32
    b32 = lib.akf_sqrt_workspace_bytes(C.byref(m), 0)
    assert 0 < b32 < b64
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) == 0
    assert lib.akf_filter_workspace_bytes(C.byref(m), 0) == 0
    m.dtype = 7
    assert lib.akf_sqrt_workspace_bytes(C.byref(m), 0) == 0
    m.dtype = _lib.AKF_F32
    m.dx = 33
    assert lib.akf_sqrt_workspace_bytes(C.byref(m), 0) == 0
    m.dx = 8
    m.dyn = 2
    m.dyn_par[1] = 0.01
    assert lib.akf_sqrt_workspace_bytes(C.byref(m), 0) == 0
    m.dyn = 0
    p = C.c_void_p(0x2000)
    ws = C.c_void_p(0x10000)
    call = lambda **kw: lib.akf_sqrt_filter_sample(
        C.byref(m), kw.get("om", p), p, kw.get("xi", p), kw.get("x", p), kw.get("mf", p), None,
        None, None, None, ws, kw.get("ws_bytes", 1 << 30), kw.get("block", 0), None)
    assert call(om=None) == 1
    assert call(mf=None) == 1
    assert call(xi=None) == 1       # a path sample needs normals
    assert call(block=-1) == 1
    assert call(ws_bytes=16) == 3


def test_mh_step_noalloc_rejects_problems_beyond_its_array():
    """The no-allocation step refuses, before any device call, a problem whose
    workspace exceeds the library's fixed scratch array."""
    lib = _lib.load()
    hdr = open(os.path.join(ROOT, "include", "akf.h")).read()
    mib = re.search(r"#define AKF_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << 20\)", hdr)
    assert mib and int(mib.group(1)) << 20 == _lib.NOALLOC_SCRATCH_BYTES
    m = _fake_model(N=4096, dx=64, dy=32)
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) > _lib.NOALLOC_SCRATCH_BYTES
    p = C.c_void_p(0x2000)
    rc = lib.akf_mh_step_noalloc(C.byref(m), p, p, 0.5, 2, p, p, p, None, None, None, None,
                                 None, 0, None)
    assert rc == 2
    assert b"scratch" in lib.akf_last_error()
    small = _fake_model(N=1024, dx=8, dy=8)
    assert 0 < lib.akf_mh_workspace_bytes(C.byref(small), 2, 0) <= _lib.NOALLOC_SCRATCH_BYTES


def test_mh_step_rejects_bad_arguments():
    lib = _lib.load()
    m = _fake_model()
    p = C.c_void_p(0x2000)
    ws = C.c_void_p(0x10000)
    call = lambda **kw: lib.akf_mh_step(
        C.byref(m), kw.get("y", p), p, kw.get("delta", 0.5), kw.get("order", 2), p, p, p, None,
        None, None, None, None, kw.get("ws", ws), kw.get("ws_bytes", 1 << 30), kw.get("block", 0),
        None)
    assert call(delta=0.0) == 1
    assert call(delta=float("nan")) == 1
    assert call(order=4) == 1
    assert call(order=3) == 5    # order 3 needs GAUSS_SITE or GAUSS_QUAD (this model is Poisson)
    assert call(y=None) == 1
    assert call(block=-1) == 1
    assert call(ws=C.c_void_p(0x10001)) == 3   # misaligned
    assert call(ws_bytes=100) == 3            # too small
    assert b"workspace" in lib.akf_last_error()


def test_student_t_needs_positive_parameters():
    lib = _lib.load()
    m = _fake_model(emit=2)
    m.nu = 0.0
    p = C.c_void_p(0x2000)
    rc = lib.akf_mh_step(C.byref(m), p, p, 0.5, 2, p, p, p, None, None, None, None, None,
                         C.c_void_p(0x10000), 1 << 30, 0, None)
    assert rc == 1


def test_multivariate_t_order_and_parameters():
    lib = _lib.load()
    p = C.c_void_p(0x2000)
    m = _fake_model(emit=4)
    # order 2 would need a dense time-varying Omega_t: rejected on both paths
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) == 0
    assert b"first-order" in lib.akf_last_error()
    assert lib.akf_mh_factorised_workspace_bytes(C.byref(m), 2) == 0
    rc = lib.akf_mh_step(C.byref(m), p, p, 0.5, 2, p, p, p, None, None, None, None, None,
                         C.c_void_p(0x10000), 1 << 30, 0, None)
    assert rc == 5
    assert lib.akf_mh_workspace_bytes(C.byref(m), 1, 0) > 0
    m.nu = 0.0
    assert lib.akf_mh_workspace_bytes(C.byref(m), 1, 0) == 0
    m = _fake_model(emit=4)
    m.R = None
    assert lib.akf_mh_factorised_workspace_bytes(C.byref(m), 1) == 0


def test_factorised_entry_points_reject_bad_requests():
    lib = _lib.load()
    p = C.c_void_p(0x2000)
    ws = C.c_void_p(0x10000)
    g = _fake_model(emit=0)
    assert lib.akf_mh_factorised_workspace_bytes(C.byref(g), 1) == 0
    assert b"Gaussian" in lib.akf_last_error()
    m = _fake_model(N=1024, dx=64, dy=64, emit=4)
    need = lib.akf_mh_factorised_workspace_bytes(C.byref(m), 1)
    # vectors only: far below the dense step's element storage
    assert 0 < need < lib.akf_mh_workspace_bytes(C.byref(m), 1, 0) // 4
    call = lambda **kw: lib.akf_mh_step_factorised(
        C.byref(m), kw.get("y", p), p, kw.get("delta", 0.5), kw.get("order", 1), p, p, p, None,
        None, None, None, None, kw.get("ws", ws), kw.get("ws_bytes", 1 << 30), None)
    assert call(delta=-1.0) == 1
    assert call(order=0) == 1
    assert call(y=None) == 1
    assert call(ws_bytes=need - 1) == 3
    assert lib.akf_mh_run_factorised(C.byref(m), p, p, 0.5, 1, -1, p, p, None, None, None, None,
                                     None, ws, 1 << 30, None) == 1


def test_nonlinear_dynamics_validation():
    lib = _lib.load()
    m = _fake_model(N=64, dx=3, dy=2, emit=5)
    m.scale = 1.0
    m.dyn = 1
    m.F = None
    m.dyn_par[3] = 2e-4
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) > 0
    # linear-only entry points refuse nonlinear dynamics
    assert lib.akf_filter_workspace_bytes(C.byref(m), 0) == 0
    assert b"linear dynamics" in lib.akf_last_error()
    assert lib.akf_sampler_workspace_bytes(C.byref(m), 0) == 0
    assert lib.akf_dnc_workspace_bytes(C.byref(m)) == 0
    assert lib.akf_mh_factorised_workspace_bytes(C.byref(m), 1) == 0
    m.dyn_par[3] = 0.0
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) == 0   # dt must be > 0
    m.dyn_par[3] = 2e-4
    m.dx = 4
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) == 0   # Lorenz-63 needs dx = 3
    m.dyn = 2
    m.dyn_par[1] = 0.01
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) > 0    # Lorenz-96, dx >= 4
    m.dx = 3
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) == 0
    m.dyn = 7
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) == 0
    # linear dynamics still need F
    m2 = _fake_model()
    m2.F = None
    assert lib.akf_mh_workspace_bytes(C.byref(m2), 2, 0) == 0


def test_gauss_site_and_dnc_workspace():
    lib = _lib.load()
    m = _fake_model(N=100, dx=5, dy=3, emit=5)
    m.scale = 0.0
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) == 0   # scale must be > 0
    m.scale = 2.0
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) > 0
    small = lib.akf_dnc_workspace_bytes(C.byref(_fake_model(N=100, dx=5)))
    big = lib.akf_dnc_workspace_bytes(C.byref(_fake_model(N=4096, dx=64)))
    assert 0 < small < big
    p = C.c_void_p(0x2000)
    rc = lib.akf_dnc_sample(C.byref(_fake_model(N=100, dx=5)), p, p, p, None, None,
                            C.c_void_p(0x10000), 1 << 30, None)
    assert rc == 1  # x is required


def test_first_order_run_validation():
    lib = _lib.load()
    m = _fake_model(N=128, dx=10)
    base = lib.akf_mh_workspace_bytes(C.byref(m), 1, 0)
    need = lib.akf_mh_first_order_workspace_bytes(C.byref(m), 0)
    # three more [N, D, D] matrices (D = 16 here) and log det S
    assert need >= base + 3 * 128 * 16 * 16 * 8 + 128 * 8
    assert lib.akf_mh_first_order_workspace_bytes(C.byref(m), -1) == 0
    p = C.c_void_p(0x2000)
    ws = C.c_void_p(0x100000)
    call = lambda model, n=1, delta=0.5, wsb=need, block=0: lib.akf_mh_run_first_order(
        C.byref(model), p, p, delta, n, p, p, None, None, None, None, None, ws, wsb, block, None)
    assert call(m, n=-1) == 1
    assert call(m, delta=0.0) == 1
    assert call(m, block=-2) == 1
    assert call(m, wsb=need - 1) == 3  # workspace too small
    # nonlinear dynamics: the auxiliary model's matrices change with the path
    nl = _fake_model(N=64, dx=3, dy=2, emit=5)
    nl.scale = 1.0
    nl.dyn = 1
    nl.F = None
    nl.dyn_par[3] = 2e-4
    assert lib.akf_mh_first_order_workspace_bytes(C.byref(nl), 0) == 0
    assert b"linear dynamics" in lib.akf_last_error()
    assert call(nl) == 5


def test_reuse_run_validation():
    lib = _lib.load()
    m = _fake_model(N=128, dx=10, emit=1)
    need2 = lib.akf_mh_reuse_workspace_bytes(C.byref(m), 2, 0)
    assert need2 == lib.akf_mh_first_order_workspace_bytes(C.byref(m), 0) > 0
    assert lib.akf_mh_reuse_workspace_bytes(C.byref(m), 1, 0) == need2
    assert lib.akf_mh_reuse_workspace_bytes(C.byref(m), 3, 0) == 0
    # GAUSSIAN has a dense Omega under order 2
    g = _fake_model(N=128, dx=10, dy=4, emit=0)
    assert lib.akf_mh_reuse_workspace_bytes(C.byref(g), 2, 0) == 0
    assert b"dense Omega" in lib.akf_last_error()
    assert lib.akf_mh_reuse_workspace_bytes(C.byref(g), 1, 0) > 0
    p = C.c_void_p(0x2000)
    ws = C.c_void_p(0x100000)
    call = lambda model, order=2, n=1, delta=0.5, wsb=need2: lib.akf_mh_run_reuse(
        C.byref(model), p, p, delta, order, n, p, p, None, None, None, None, None, ws, wsb, 0, None)
    assert call(g) == 5
    assert call(m, n=-1) == 1
    assert call(m, delta=-1.0) == 1
    assert call(m, wsb=need2 - 1) == 3
    nl = _fake_model(N=64, dx=3, dy=2, emit=5)
    nl.scale = 1.0
    nl.dyn = 1
    nl.F = None
    nl.dyn_par[3] = 2e-4
    assert lib.akf_mh_reuse_workspace_bytes(C.byref(nl), 2, 0) == 0
    assert call(nl) == 5


def test_dtype_selector():
    """The model's dtype field: AKF_F64 (0, the zero-initialised default) is the
    built path; AKF_F32 is a valid request the library does not implement
    (AKF_ERR_UNSUPPORTED from the calls, 0 from the workspace queries); any
    other value is invalid."""
    lib = _lib.load()
    p = C.c_void_p(0x2000)
    ws = C.c_void_p(0x10000)
    m = _fake_model()
    assert m.dtype == _lib.AKF_F64
    assert lib.akf_mh_workspace_bytes(C.byref(m), 2, 0) > 0
    step = lambda model: lib.akf_mh_step(C.byref(model), p, p, 0.5, 2, p, p, p, None, None, None,
                                         None, None, ws, 1 << 30, 0, None)
    m.dtype = _lib.AKF_F32
    assert step(m) == 5
    assert b"AKF_F32" in lib.akf_last_error()
    for q in (lib.akf_mh_workspace_bytes(C.byref(m), 2, 0),
              lib.akf_filter_workspace_bytes(C.byref(m), 0),
              lib.akf_sampler_workspace_bytes(C.byref(m), 0),
              lib.akf_mh_first_order_workspace_bytes(C.byref(m), 0),
              lib.akf_mh_reuse_workspace_bytes(C.byref(m), 2, 0),
              lib.akf_dnc_workspace_bytes(C.byref(m)),
              lib.akf_smoother_workspace_bytes(C.byref(m), 0)):
        assert q == 0
    assert lib.akf_mh_run(C.byref(m), p, p, 0.5, 2, 1, p, p, None, None, None, None, None, ws,
                          1 << 30, 0, None) == 5
    m.dtype = 7
    assert step(m) == 1
    # batched chains validate each chain's model the same way
    ch = (_lib.AkfChain * 1)()
    ch[0].model = _fake_model()
    ch[0].model.dtype = _lib.AKF_F32
    ch[0].y = ch[0].x = ch[0].xi = ch[0].unif = 0x2000
    ch[0].delta, ch[0].order = 0.5, 2
    h = C.c_void_p()
    assert lib.akf_batch_plan_create(C.byref(h), 1, ch, 1, 8, None, None) == 5
    assert not h.value
