"""Python front end of the auxiliary Kalman MCMC library.

Torch supplies device memory and the stream; the arithmetic happens in the HIP
kernels behind include/akf.h.  All tensors are float64 on a ROCm device.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib

EMIT_GAUSSIAN, EMIT_POISSON_LOG, EMIT_STUDENT_T, EMIT_STOCH_VOL, EMIT_MVT = 0, 1, 2, 3, 4
EMIT_GAUSS_SITE, EMIT_GAUSS_QUAD = 5, 6
DYN_LINEAR, DYN_LORENZ63, DYN_LORENZ96 = 0, 1, 2
ST_FWD_NOT_PD, ST_REV_NOT_PD, ST_NONFINITE = 1, 2, 4


def _dev(device=None) -> torch.device:
    if device is None:
        device = torch.device("cuda", torch.cuda.current_device())
    device = torch.device(device)
    if device.type != "cuda":
        raise _lib.AkfError("the auxiliary Kalman kernels need a ROCm device tensor")
    return device


def _t(a, device, dtype=torch.float64) -> Optional[torch.Tensor]:
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_f64(name, t: torch.Tensor, shape):
    if t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda":
        raise _lib.AkfError(f"{name} must be a contiguous float64 ROCm tensor")
    if tuple(t.shape) != tuple(shape):
        raise _lib.AkfError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


@dataclass
class DeviceModel:
    """Gaussian-dynamics state-space model resident on the device."""
    N: int
    m0: torch.Tensor
    P0: torch.Tensor
    F: torch.Tensor
    Q: torch.Tensor
    emit: int
    b: Optional[torch.Tensor] = None
    H: Optional[torch.Tensor] = None
    R: Optional[torch.Tensor] = None
    site: Optional[torch.Tensor] = None
    nu: float = 0.0
    scale: float = 0.0
    dyn: int = DYN_LINEAR
    dyn_par: tuple = (0.0, 0.0, 0.0, 0.0)
    obs_beta: float = 0.0
    slr_var: float = 0.0

    @classmethod
    def from_arrays(cls, N, m0, P0, F, Q, emit, b=None, H=None, R=None, site=None, nu=0.0,
                    scale=0.0, dyn=DYN_LINEAR, dyn_par=(0.0, 0.0, 0.0, 0.0), obs_beta=0.0,
                    slr_var=0.0, device=None):
        dev = _dev(device)
        return cls(N=int(N), m0=_t(m0, dev), P0=_t(P0, dev), F=_t(F, dev), Q=_t(Q, dev),
                   emit=int(emit), b=_t(b, dev), H=_t(H, dev), R=_t(R, dev),
                   site=_t(site, dev, torch.int32), nu=float(nu), scale=float(scale),
                   dyn=int(dyn), dyn_par=tuple(float(v) for v in dyn_par),
                   obs_beta=float(obs_beta), slr_var=float(slr_var))

    @classmethod
    def from_workload(cls, w, device=None):
        return cls.from_arrays(w.N, w.m0, w.P0, w.F, w.Q, w.emit, b=w.b, H=w.H, R=w.R,
                               site=w.site, nu=w.nu, scale=w.scale, dyn=w.dyn,
                               dyn_par=w.dyn_par, obs_beta=getattr(w, "obs_beta", 0.0),
                               slr_var=getattr(w, "slr_var", 0.0), device=device)

    @property
    def dx(self) -> int:
        return int(self.m0.shape[0])

    @property
    def dy(self) -> int:
        if self.emit == EMIT_GAUSSIAN:
            return int(self.H.shape[0]) if self.H is not None else 0
        return int(self.site.shape[0]) if self.site is not None else 0

    @property
    def device(self) -> torch.device:
        return self.m0.device

    @property
    def is_diagonal_form(self) -> bool:
        """True when P0, F and Q hold diagonals [dx] (the factorised entry points)."""
        return self.Q.dim() == 1

    def diagonal(self) -> "DeviceModel":
        """The model with P0, F and Q replaced by their diagonals, as the
        factorised entry points take it.  Raises if any of them is not diagonal."""
        out = {}
        for k in ("P0", "F", "Q"):
            a = getattr(self, k)
            dg = torch.diagonal(a).contiguous()
            if not torch.equal(a, torch.diag(dg)):
                raise _lib.AkfError(f"{k} is not diagonal: the prior does not factorise")
            out[k] = dg
        return DeviceModel(N=self.N, m0=self.m0, P0=out["P0"], F=out["F"], Q=out["Q"],
                           emit=self.emit, b=self.b, H=self.H, R=self.R, site=self.site,
                           nu=self.nu, scale=self.scale, obs_beta=self.obs_beta,
                           slr_var=self.slr_var)

    def cstruct(self) -> _lib.AkfModel:
        s = _lib.AkfModel()
        s.N, s.dx, s.dy = self.N, self.dx, self.dy
        s.m0, s.P0, s.Q = self.m0.data_ptr(), self.P0.data_ptr(), self.Q.data_ptr()
        s.F = self.F.data_ptr() if self.F is not None else None
        s.b = self.b.data_ptr() if self.b is not None else None
        s.emit = self.emit
        s.H = self.H.data_ptr() if self.H is not None else None
        s.R = self.R.data_ptr() if self.R is not None else None
        s.site = self.site.data_ptr() if self.site is not None else None
        s.nu, s.scale = self.nu, self.scale
        s.dyn = self.dyn
        par = list(self.dyn_par) + [0.0] * (4 - len(self.dyn_par))
        for i in range(4):
            s.dyn_par[i] = par[i]
        s.obs_beta, s.slr_var = self.obs_beta, self.slr_var
        return s


class Workspace:
    """Caller-owned scratch buffer reused across calls (grown on demand)."""

    def __init__(self, device=None):
        self.device = _dev(device)
        self.buf: Optional[torch.Tensor] = None

    def get(self, nbytes: int) -> torch.Tensor:
        if nbytes <= 0:
            raise _lib.AkfError("unsupported problem size (workspace query returned 0)")
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        return self.buf

    def ptr_bytes(self, nbytes: int):
        b = self.get(nbytes)
        p = b.data_ptr()
        off = (-p) % 256
        return C.c_void_p(p + off), C.c_size_t(b.numel() - off)


_default_ws = {}


def _ws_for(device) -> Workspace:
    key = (device.type, device.index)
    if key not in _default_ws:
        _default_ws[key] = Workspace(device)
    return _default_ws[key]


def _need(nbytes: int, what: str) -> int:
    """A workspace size from a *_workspace_bytes query; 0 means the request was
    rejected, and the library's last error says why."""
    if nbytes == 0:
        msg = _lib.load().akf_last_error()
        raise _lib.AkfError(f"{what} rejected the request: {msg.decode() if msg else ''}")
    return nbytes


def _check_form(model: DeviceModel, factorised: bool):
    if factorised != model.is_diagonal_form:
        raise _lib.AkfError("the factorised step takes P0, F and Q as diagonals "
                            "(DeviceModel.diagonal()); the dense step takes matrices")


def mh_step(model: DeviceModel, y, x, delta: float, order: int, xi, unif, x_out=None,
            block: int = 0, ws: Optional[Workspace] = None, factorised: bool = False) -> dict:
    """One auxiliary Kalman MH step.  xi [2,N,dx], unif [1] (device tensors).
    factorised=True runs the step for a prior that factorises over coordinates
    (akf_mh_step_factorised; `model` from DeviceModel.diagonal(), block unused).
    Returns device tensors: x_out, log_ratio, accepted, logZ_fwd, logZ_rev, status."""
    lib = _lib.load()
    _check_form(model, factorised)
    dev = model.device
    N, dx = model.N, model.dx
    _check_f64("y", y, (N, model.dy))
    _check_f64("x", x, (N, dx))
    _check_f64("xi", xi, (2, N, dx))
    _check_f64("unif", unif, (1,))
    if x_out is None:
        x_out = torch.empty_like(x)
    lr = torch.empty(1, dtype=torch.float64, device=dev)
    lzf = torch.empty(1, dtype=torch.float64, device=dev)
    lzr = torch.empty(1, dtype=torch.float64, device=dev)
    acc = torch.empty(1, dtype=torch.int32, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    ms = model.cstruct()
    if factorised:
        need = _need(lib.akf_mh_factorised_workspace_bytes(C.byref(ms), order),
                     "akf_mh_factorised_workspace_bytes")
        wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
        rc = lib.akf_mh_step_factorised(C.byref(ms), _ptr(y), _ptr(x), float(delta), int(order),
                                        _ptr(xi), _ptr(unif), _ptr(x_out), _ptr(lr), _ptr(acc),
                                        _ptr(lzf), _ptr(lzr), _ptr(st), wsp, wsb, _stream(dev))
        _lib.check(rc, "akf_mh_step_factorised")
    else:
        need = _need(lib.akf_mh_workspace_bytes(C.byref(ms), order, block),
                     "akf_mh_workspace_bytes")
        wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
        rc = lib.akf_mh_step(C.byref(ms), _ptr(y), _ptr(x), float(delta), int(order), _ptr(xi),
                             _ptr(unif), _ptr(x_out), _ptr(lr), _ptr(acc), _ptr(lzf), _ptr(lzr),
                             _ptr(st), wsp, wsb, int(block), _stream(dev))
        _lib.check(rc, "akf_mh_step")
    return dict(x_out=x_out, log_ratio=lr, accepted=acc, logZ_fwd=lzf, logZ_rev=lzr, status=st)


def mh_step_noalloc(model: DeviceModel, y, x, delta: float, order: int, xi, unif, x_out,
                    log_ratio, accepted, logZ_fwd, logZ_rev, status, block: int = 0) -> None:
    """akf_mh_step_noalloc: mh_step with the library's fixed scratch array in
    place of a workspace.  Every output is a caller tensor (x_out [N,dx]
    float64; log_ratio, logZ_fwd, logZ_rev [1] float64; accepted, status [1]
    int32), so this call allocates nothing on the device."""
    lib = _lib.load()
    _check_form(model, False)
    N, dx = model.N, model.dx
    _check_f64("y", y, (N, model.dy))
    _check_f64("x", x, (N, dx))
    _check_f64("xi", xi, (2, N, dx))
    _check_f64("unif", unif, (1,))
    _check_f64("x_out", x_out, (N, dx))
    for name, t in (("log_ratio", log_ratio), ("logZ_fwd", logZ_fwd), ("logZ_rev", logZ_rev)):
        _check_f64(name, t, (1,))
    for name, t in (("accepted", accepted), ("status", status)):
        if t.dtype != torch.int32 or tuple(t.shape) != (1,) or t.device != model.device:
            raise _lib.AkfError(f"{name} must be an int32 tensor of shape (1,) on {model.device}")
    ms = model.cstruct()
    rc = lib.akf_mh_step_noalloc(C.byref(ms), _ptr(y), _ptr(x), float(delta), int(order),
                                 _ptr(xi), _ptr(unif), _ptr(x_out), _ptr(log_ratio),
                                 _ptr(accepted), _ptr(logZ_fwd), _ptr(logZ_rev), _ptr(status),
                                 int(block), _stream(model.device))
    _lib.check(rc, "akf_mh_step_noalloc")


def mh_run(model: DeviceModel, y, x, delta: float, order: int, xi, unif, block: int = 0,
           ws: Optional[Workspace] = None, outputs: bool = True, factorised: bool = False,
           reuse_matrices: bool = False) -> dict:
    """n_steps MH steps, x updated in place.  xi [n_steps,2,N,dx], unif [n_steps].
    factorised as in mh_step.  reuse_matrices (dense prior): the auxiliary
    model's matrices are reused wherever unchanged -- order 1: formed once for
    the whole call (akf_mh_run_first_order); order 2: kept from a forward
    proposal for the next one after a rejection (akf_mh_run_reuse, the branch
    decided on the device, so the call can be captured in a graph).  The chain
    is the same up to rounding."""
    lib = _lib.load()
    _check_form(model, factorised)
    if reuse_matrices and factorised:
        raise ValueError("reuse_matrices takes the dense prior")
    dev = model.device
    N, dx = model.N, model.dx
    n = int(xi.shape[0])
    _check_f64("y", y, (N, model.dy))
    _check_f64("x", x, (N, dx))
    _check_f64("xi", xi, (n, 2, N, dx))
    _check_f64("unif", unif, (n,))
    out = {}
    if outputs:
        out = dict(log_ratio=torch.empty(n, dtype=torch.float64, device=dev),
                   accepted=torch.empty(n, dtype=torch.int32, device=dev),
                   logZ_fwd=torch.empty(n, dtype=torch.float64, device=dev),
                   logZ_rev=torch.empty(n, dtype=torch.float64, device=dev),
                   status=torch.empty(n, dtype=torch.int32, device=dev))
    ms = model.cstruct()
    outs = [_ptr(out.get(k)) for k in ("log_ratio", "accepted", "logZ_fwd", "logZ_rev", "status")]
    if factorised:
        need = _need(lib.akf_mh_factorised_workspace_bytes(C.byref(ms), order),
                     "akf_mh_factorised_workspace_bytes")
        wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
        rc = lib.akf_mh_run_factorised(C.byref(ms), _ptr(y), _ptr(x), float(delta), int(order), n,
                                       _ptr(xi), _ptr(unif), *outs, wsp, wsb, _stream(dev))
        _lib.check(rc, "akf_mh_run_factorised")
    elif reuse_matrices and order == 1:
        need = _need(lib.akf_mh_first_order_workspace_bytes(C.byref(ms), block),
                     "akf_mh_first_order_workspace_bytes")
        wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
        rc = lib.akf_mh_run_first_order(C.byref(ms), _ptr(y), _ptr(x), float(delta), n, _ptr(xi),
                                        _ptr(unif), *outs, wsp, wsb, int(block), _stream(dev))
        _lib.check(rc, "akf_mh_run_first_order")
    elif reuse_matrices:
        need = _need(lib.akf_mh_reuse_workspace_bytes(C.byref(ms), int(order), block),
                     "akf_mh_reuse_workspace_bytes")
        wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
        rc = lib.akf_mh_run_reuse(C.byref(ms), _ptr(y), _ptr(x), float(delta), int(order), n,
                                  _ptr(xi), _ptr(unif), *outs, wsp, wsb, int(block), _stream(dev))
        _lib.check(rc, "akf_mh_run_reuse")
    else:
        need = _need(lib.akf_mh_workspace_bytes(C.byref(ms), order, block),
                     "akf_mh_workspace_bytes")
        wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
        rc = lib.akf_mh_run(C.byref(ms), _ptr(y), _ptr(x), float(delta), int(order), n, _ptr(xi),
                            _ptr(unif), *outs, wsp, wsb, int(block), _stream(dev))
        _lib.check(rc, "akf_mh_run")
    out["x"] = x
    return out


def aux_filter(model: DeviceModel, omega, Omega, block: int = 0, moments: bool = True,
               ws: Optional[Workspace] = None):
    """Parallel-in-time filter of x_t = F x_{t-1} + b + N(0,Q), omega_t = x_t + N(0, diag Omega_t).
    Returns (mf [N,dx] | None, Pf [N,dx,dx] | None, ell [N], status [1])."""
    lib = _lib.load()
    dev = model.device
    N, dx = model.N, model.dx
    _check_f64("omega", omega, (N, dx))
    _check_f64("Omega", Omega, (N, dx))
    mf = torch.empty((N, dx), dtype=torch.float64, device=dev) if moments else None
    Pf = torch.empty((N, dx, dx), dtype=torch.float64, device=dev) if moments else None
    ell = torch.empty(N, dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    ms = model.cstruct()
    need = _need(lib.akf_filter_workspace_bytes(C.byref(ms), block), "akf_filter_workspace_bytes")
    wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
    rc = lib.akf_aux_filter(C.byref(ms), _ptr(omega), _ptr(Omega), _ptr(mf), _ptr(Pf), _ptr(ell),
                            _ptr(st), wsp, wsb, int(block), _stream(dev))
    _lib.check(rc, "akf_aux_filter")
    return mf, Pf, ell, st


def rts_sample(model: DeviceModel, mf, Pf, xi, block: int = 0, ws: Optional[Workspace] = None):
    """Pathwise RTS sample from filtering moments.  Returns (x [N,dx], status [1])."""
    lib = _lib.load()
    dev = model.device
    N, dx = model.N, model.dx
    _check_f64("mf", mf, (N, dx))
    _check_f64("Pf", Pf, (N, dx, dx))
    _check_f64("xi", xi, (N, dx))
    x = torch.empty((N, dx), dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    ms = model.cstruct()
    need = _need(lib.akf_sampler_workspace_bytes(C.byref(ms), block), "akf_sampler_workspace_bytes")
    wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
    rc = lib.akf_rts_sample(C.byref(ms), _ptr(mf), _ptr(Pf), _ptr(xi), _ptr(x), _ptr(st), wsp,
                            wsb, int(block), _stream(dev))
    _lib.check(rc, "akf_rts_sample")
    return x, st


def sqrt_filter_sample(model: DeviceModel, omega, Omega, xi=None, dtype: str = "f32",
                       block: int = 0, factors: bool = True, ws: Optional[Workspace] = None):
    """Square-root parallel filter (and, with xi [N,dx], the pathwise sample) of
    x_t = F x_{t-1} + b + N(0,Q), omega_t = x_t + N(0, diag Omega_t), computed in
    FP32 (dtype "f32") or FP64 ("f64") with the triangularisations in FP64
    (akf_sqrt_filter_sample; dx <= 32).  Returns a dict of device tensors: mf
    [N,dx], Uf [N,dx,dx] (lower factors of P^f; None unless factors), ell [N],
    logZ [1], x [N,dx] (None without xi), status [1]."""
    lib = _lib.load()
    dev = model.device
    N, dx = model.N, model.dx
    _check_f64("omega", omega, (N, dx))
    _check_f64("Omega", Omega, (N, dx))
    if xi is not None:
        _check_f64("xi", xi, (N, dx))
    if dtype not in ("f32", "f64"):
        raise ValueError("dtype must be 'f32' or 'f64'")
    f = dict(dtype=torch.float64, device=dev)
    mf = torch.empty((N, dx), **f)
    Uf = torch.empty((N, dx, dx), **f) if factors else None
    ell = torch.empty(N, **f)
    lz = torch.empty(1, **f)
    x = torch.empty((N, dx), **f) if xi is not None else None
    st = torch.empty(1, dtype=torch.int32, device=dev)
    ms = model.cstruct()
    ms.dtype = _lib.AKF_F32 if dtype == "f32" else _lib.AKF_F64
    need = _need(lib.akf_sqrt_workspace_bytes(C.byref(ms), block), "akf_sqrt_workspace_bytes")
    wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
    rc = lib.akf_sqrt_filter_sample(C.byref(ms), _ptr(omega), _ptr(Omega), _ptr(xi), _ptr(x),
                                    _ptr(mf), _ptr(Uf), _ptr(ell), _ptr(lz), _ptr(st), wsp, wsb,
                                    int(block), _stream(dev))
    _lib.check(rc, "akf_sqrt_filter_sample")
    return dict(mf=mf, Uf=Uf, ell=ell, logZ=lz, x=x, status=st)


def dnc_sample(model: DeviceModel, mf, Pf, xi, ws: Optional[Workspace] = None):
    """Divide-and-conquer path sample from filtering moments (same law as
    rts_sample, its own noise map).  Returns (x [N,dx], status [1])."""
    lib = _lib.load()
    dev = model.device
    N, dx = model.N, model.dx
    _check_f64("mf", mf, (N, dx))
    _check_f64("Pf", Pf, (N, dx, dx))
    _check_f64("xi", xi, (N, dx))
    x = torch.empty((N, dx), dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    ms = model.cstruct()
    need = _need(lib.akf_dnc_workspace_bytes(C.byref(ms)), "akf_dnc_workspace_bytes")
    wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
    rc = lib.akf_dnc_sample(C.byref(ms), _ptr(mf), _ptr(Pf), _ptr(xi), _ptr(x), _ptr(st), wsp,
                            wsb, _stream(dev))
    _lib.check(rc, "akf_dnc_sample")
    return x, st


def smoother(model: DeviceModel, mf, Pf, block: int = 0, ws: Optional[Workspace] = None):
    """RTS smoothing moments from filtering moments (parallel (E, g, L) suffix scan).
    Returns (ms [N,dx], Ps [N,dx,dx], status [1])."""
    lib = _lib.load()
    dev = model.device
    N, dx = model.N, model.dx
    _check_f64("mf", mf, (N, dx))
    _check_f64("Pf", Pf, (N, dx, dx))
    ms = torch.empty((N, dx), dtype=torch.float64, device=dev)
    Ps = torch.empty((N, dx, dx), dtype=torch.float64, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    ms_ = model.cstruct()
    need = _need(lib.akf_smoother_workspace_bytes(C.byref(ms_), block),
                 "akf_smoother_workspace_bytes")
    wsp, wsb = (ws or _ws_for(dev)).ptr_bytes(need)
    rc = lib.akf_smoother(C.byref(ms_), _ptr(mf), _ptr(Pf), _ptr(ms), _ptr(Ps), _ptr(st), wsp, wsb,
                          int(block), _stream(dev))
    _lib.check(rc, "akf_smoother")
    return ms, Ps, st


class LGSSM:
    """Linear-Gaussian model with theta = (F, log diag Q, H, log diag R) on the device."""

    def __init__(self, m0, P0, y, device=None):
        dev = _dev(device)
        self.m0 = _t(m0, dev)
        self.P0 = _t(P0, dev)
        self.y = _t(y, dev)
        self.N, self.dy = self.y.shape
        self.dx = self.m0.shape[0]
        self.device = dev

    def cstruct(self, F, logq, H, logr) -> _lib.AkfLgssm:
        for name, t, shp in (("F", F, (self.dx, self.dx)), ("logq", logq, (self.dx,)),
                             ("H", H, (self.dy, self.dx)), ("logr", logr, (self.dy,))):
            _check_f64(name, t, shp)
        s = _lib.AkfLgssm()
        s.N, s.dx, s.dy = self.N, self.dx, self.dy
        s.m0, s.P0 = self.m0.data_ptr(), self.P0.data_ptr()
        s.F, s.logq, s.H, s.logr = F.data_ptr(), logq.data_ptr(), H.data_ptr(), logr.data_ptr()
        s.y = self.y.data_ptr()
        return s


def lgssm_loglik(model: LGSSM, F, logq, H, logr, block: int = 0,
                 ws: Optional[Workspace] = None, ell: bool = False):
    """log p(y | theta).  Returns (ll [1], ell [N] | None, status [1], ws).  The
    returned workspace holds the checkpoint used by lgssm_loglik_grad."""
    lib = _lib.load()
    dev = model.device
    s = model.cstruct(F, logq, H, logr)
    need = _need(lib.akf_lgssm_workspace_bytes(C.byref(s), block), "akf_lgssm_workspace_bytes")
    ws = ws or Workspace(dev)
    wsp, wsb = ws.ptr_bytes(need)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    el = torch.empty(model.N, dtype=torch.float64, device=dev) if ell else None
    st = torch.empty(1, dtype=torch.int32, device=dev)
    rc = lib.akf_lgssm_loglik(C.byref(s), _ptr(ll), _ptr(el), _ptr(st), wsp, wsb, int(block),
                              _stream(dev))
    _lib.check(rc, "akf_lgssm_loglik")
    return ll, el, st, ws


def lgssm_loglik_grad(model: LGSSM, F, logq, H, logr, ws: Workspace, ll_bar=None,
                      block: int = 0):
    """Adjoint of lgssm_loglik (same workspace, called after it).  Returns
    (dF, dlogq, dH, dlogr, status)."""
    lib = _lib.load()
    dev = model.device
    s = model.cstruct(F, logq, H, logr)
    need = _need(lib.akf_lgssm_workspace_bytes(C.byref(s), block), "akf_lgssm_workspace_bytes")
    wsp, wsb = ws.ptr_bytes(need)
    dF = torch.empty_like(F)
    dq = torch.empty_like(logq)
    dH = torch.empty_like(H)
    dr = torch.empty_like(logr)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    if ll_bar is not None:
        _check_f64("ll_bar", ll_bar, (1,))
    rc = lib.akf_lgssm_loglik_grad(C.byref(s), _ptr(ll_bar), _ptr(dF), _ptr(dq), _ptr(dH),
                                   _ptr(dr), _ptr(st), wsp, wsb, int(block), _stream(dev))
    _lib.check(rc, "akf_lgssm_loglik_grad")
    return dF, dq, dH, dr, st


class KalmanLogLik(torch.autograd.Function):
    """log p(y | F, log diag Q, H, log diag R) with a hand-written reverse-mode
    adjoint.  forward keeps the workspace (the filtering-moment checkpoint) on
    ctx; backward runs the adjoint scans on it."""

    @staticmethod
    def forward(ctx, F, logq, H, logr, model: LGSSM, block: int = 0):
        F, logq, H, logr = (a.detach().contiguous() for a in (F, logq, H, logr))
        ll, _, st, ws = lgssm_loglik(model, F, logq, H, logr, block=block)
        ctx.model, ctx.ws, ctx.block = model, ws, block
        ctx.save_for_backward(F, logq, H, logr)
        return ll.reshape(())

    @staticmethod
    def backward(ctx, g):
        F, logq, H, logr = ctx.saved_tensors
        gb = g.reshape(1).to(torch.float64).contiguous()
        dF, dq, dH, dr, _ = lgssm_loglik_grad(ctx.model, F, logq, H, logr, ctx.ws, ll_bar=gb,
                                              block=ctx.block)
        return dF, dq, dH, dr, None, None


class GibbsState:
    """State of a Gibbs sampler over (theta, x) of an LGSSM (akf_gibbs_*):
    theta [p] (flat F, logq, H, logr), its log posterior and gradient, the
    path x [N,dx] and the library's per-theta state buffer.  All device
    tensors, updated in place by gibbs_sweep."""

    def __init__(self, model: "LGSSM", theta, logpost, grad, x, state, ws, prior_sd, block):
        self.model, self.theta, self.logpost, self.grad, self.x = model, theta, logpost, grad, x
        self.state, self.ws, self.prior_sd, self.block = state, ws, float(prior_sd), int(block)
        self.status = torch.zeros(2, dtype=torch.int32, device=model.device)


def n_theta(dx: int, dy: int) -> int:
    return dx * dx + dx + dy * dx + dy


def _lgssm_shape(model: "LGSSM") -> _lib.AkfLgssm:
    s = _lib.AkfLgssm()
    s.N, s.dx, s.dy = model.N, model.dx, model.dy
    s.m0, s.P0, s.y = model.m0.data_ptr(), model.P0.data_ptr(), model.y.data_ptr()
    return s


def gibbs_init(model: "LGSSM", theta, x, prior_sd: float = 10.0, block: int = 0) -> GibbsState:
    """Starts a Gibbs sampler at theta [p] (copied) and path x [N,dx] (copied):
    log posterior, gradient and the per-theta state (akf_gibbs_init)."""
    lib = _lib.load()
    dev = model.device
    p = n_theta(model.dx, model.dy)
    _check_f64("theta", theta, (p,))
    _check_f64("x", x, (model.N, model.dx))
    s = _lgssm_shape(model)
    nst = _need(lib.akf_gibbs_state_bytes(C.byref(s)), "akf_gibbs_state_bytes")
    nws = _need(lib.akf_gibbs_workspace_bytes(C.byref(s), int(block)), "akf_gibbs_workspace_bytes")
    state, ws = Workspace(dev), Workspace(dev)
    stp, stb = state.ptr_bytes(nst)
    wsp, wsb = ws.ptr_bytes(nws)
    G = GibbsState(model, theta.clone(), torch.empty(1, dtype=torch.float64, device=dev),
                   torch.empty(p, dtype=torch.float64, device=dev), x.clone(), state, ws,
                   prior_sd, block)
    rc = lib.akf_gibbs_init(C.byref(s), _ptr(G.theta), float(prior_sd), _ptr(G.logpost),
                            _ptr(G.grad), stp, stb, _ptr(G.status), wsp, wsb, int(block),
                            _stream(dev))
    _lib.check(rc, "akf_gibbs_init")
    return G


def gibbs_sweep(G: GibbsState, eps: float, xi_theta, u_theta, xi_x, delta: float = 1.0,
                xi_path=None, u_path=None, outputs: bool = True) -> dict:
    """One sweep (akf_gibbs_sweep): MALA on theta, exact refresh of x, then
    len(u_path) auxiliary Kalman path steps.  xi_theta [p], u_theta [1],
    xi_x [N,dx], xi_path [k,2,N,dx], u_path [k] (device tensors; k may be 0).
    Updates G in place; returns device tensors accepted_theta, log_alpha,
    path_log_ratio, path_accepted, path_status and status [2]."""
    lib = _lib.load()
    model = G.model
    dev = model.device
    N, dx = model.N, model.dx
    p = G.theta.numel()
    _check_f64("xi_theta", xi_theta, (p,))
    _check_f64("u_theta", u_theta, (1,))
    _check_f64("xi_x", xi_x, (N, dx))
    k = 0 if u_path is None else int(u_path.shape[0])
    if k:
        _check_f64("xi_path", xi_path, (k, 2, N, dx))
        _check_f64("u_path", u_path, (k,))
    out = {}
    if outputs:
        out = dict(accepted_theta=torch.empty(1, dtype=torch.int32, device=dev),
                   log_alpha=torch.empty(1, dtype=torch.float64, device=dev),
                   path_log_ratio=torch.empty(k, dtype=torch.float64, device=dev),
                   path_accepted=torch.empty(k, dtype=torch.int32, device=dev),
                   path_status=torch.empty(k, dtype=torch.int32, device=dev))
    s = _lgssm_shape(model)
    nst = _need(lib.akf_gibbs_state_bytes(C.byref(s)), "akf_gibbs_state_bytes")
    nws = _need(lib.akf_gibbs_workspace_bytes(C.byref(s), G.block), "akf_gibbs_workspace_bytes")
    stp, stb = G.state.ptr_bytes(nst)
    wsp, wsb = G.ws.ptr_bytes(nws)
    o = [_ptr(out.get(n)) if k or not n.startswith("path") else None
         for n in ("accepted_theta", "log_alpha", "path_log_ratio", "path_accepted",
                   "path_status")]
    rc = lib.akf_gibbs_sweep(C.byref(s), _ptr(G.theta), _ptr(G.logpost), _ptr(G.grad),
                             _ptr(G.x), stp, stb, G.prior_sd, float(eps), _ptr(xi_theta),
                             _ptr(u_theta), _ptr(xi_x), float(delta), k,
                             _ptr(xi_path) if k else None, _ptr(u_path) if k else None, *o,
                             _ptr(G.status), wsp, wsb, G.block, _stream(dev))
    _lib.check(rc, "akf_gibbs_sweep")
    out["status"] = G.status
    return out


class BatchPlan:
    """Many independent chains advanced together by batched persistent kernels
    (include/akf.h, akf_batch_*).  `chains` is a list of dicts with keys model
    (DeviceModel), y, x (updated in place), xi [n_steps,2,N,dx], unif [n_steps],
    delta, order and optional per-step outputs log_ratio, accepted, logZ_fwd,
    logZ_rev, status (device tensors).  The plan keeps references to every
    tensor it points at."""

    def __init__(self, chains, n_steps: int, block: int = 0, tune_cache: Optional[str] = None,
                 device=None):
        lib = _lib.load()
        self.device = _dev(device)
        self.stream = torch.cuda.Stream(device=self.device)  # default priority
        self.chains = chains
        self.n_steps = int(n_steps)
        arr = (_lib.AkfChain * len(chains))()
        for k, c in enumerate(chains):
            m = c["model"]
            N, dx = m.N, m.dx
            _check_f64("y", c["y"], (N, m.dy))
            _check_f64("x", c["x"], (N, dx))
            _check_f64("xi", c["xi"], (n_steps, 2, N, dx))
            _check_f64("unif", c["unif"], (n_steps,))
            a = arr[k]
            a.model = m.cstruct()
            a.y, a.x, a.xi, a.unif = (c["y"].data_ptr(), c["x"].data_ptr(), c["xi"].data_ptr(),
                                      c["unif"].data_ptr())
            a.delta, a.order = float(c["delta"]), int(c["order"])
            for f in ("log_ratio", "accepted", "logZ_fwd", "logZ_rev", "status"):
                t = c.get(f)
                setattr(a, f, t.data_ptr() if t is not None else None)
        self._arr = arr
        self.handle = C.c_void_p()
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        rc = lib.akf_batch_plan_create(C.byref(self.handle), len(chains), arr, self.n_steps,
                                       int(block), tune_cache.encode() if tune_cache else None,
                                       C.c_void_p(self.stream.cuda_stream))
        _lib.check(rc, "akf_batch_plan_create")
        cur.wait_stream(self.stream)

    def run(self, use_graph: bool = True):
        lib = _lib.load()
        cur = torch.cuda.current_stream(self.device)
        self.stream.wait_stream(cur)
        rc = lib.akf_batch_mh_run(self.handle, 1 if use_graph else 0,
                                  C.c_void_p(self.stream.cuda_stream))
        _lib.check(rc, "akf_batch_mh_run")
        cur.wait_stream(self.stream)

    def info(self) -> dict:
        lib = _lib.load()
        n = C.c_int32()
        D = (C.c_int32 * 4)()
        B = (C.c_int32 * 4)()
        nc = (C.c_int32 * 4)()
        sb = (C.c_int32 * 4)()
        nbytes = C.c_size_t()
        _lib.check(lib.akf_batch_plan_info(self.handle, 4, C.byref(n), D, B, nc, sb,
                                           C.byref(nbytes)), "akf_batch_plan_info")
        return dict(classes=[dict(D=D[i], block=B[i], chains=nc[i], sbuild_teams_per_simd=sb[i])
                             for i in range(n.value)],
                    device_bytes=nbytes.value)

    def close(self):
        if self.handle:
            _lib.load().akf_batch_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
