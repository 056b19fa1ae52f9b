"""FP64 oracle of one Gibbs sweep over (theta, x) for the linear-Gaussian model.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP library and never imports it.

Model (App. A, eq. lgssm-app with b = c = 0; the parametric form of eq.
parametric-ssm): x_0 ~ N(m0, P0), x_t = F x_{t-1} + N(0, diag exp(logq)),
y_t = H x_t + N(0, diag exp(logr)); theta = (F, log diag Q, H, log diag R),
flattened in that order (F and H row-major), p = dx^2 + dx + dy*dx + dy.

The paper estimates parameters by alternating a theta update with the
auxiliary Kalman path update inside a Gibbs sampler (Sec. "Parameter
estimation in a continuous-discrete diffusion smoothing problem").  Its own
theta step is conjugate; here theta moves by a gradient step, and a gradient
step on the MARGINAL posterior p(theta | y) changes theta without regard to x,
so x must be re-drawn from p(x | theta', y) before any path step that
conditions on it.  One sweep is therefore, in this order:

  1. MALA on log pi(theta) = log p(theta) + log p(y | theta), prior N(0, sd^2)
     on every coordinate: theta' = theta + (eps^2/2) g(theta) + eps xi,
     log alpha = log pi(theta') - log pi(theta) + log q(theta | theta')
     - log q(theta' | theta), q(a | b) = N(a; b + (eps^2/2) g(b), eps^2 I);
     accept iff log u < log alpha (a non-finite log alpha rejects);
  2. x ~ p(x | theta, y) exactly, by forward filtering and backward sampling
     (the Kalman filter and the RTS sampler of the oracle) with the supplied
     normals;
  3. k auxiliary Kalman MH steps on x at the new theta (second order: the
     emission is Gaussian, so every step accepts).

Each sub-step leaves the joint posterior p(theta, x | y) invariant: 1 is an MH
kernel on the theta-marginal, 2 draws x from its full conditional (together a
valid collapsed-Gibbs pair), 3 is a p(x | theta, y)-invariant kernel.

The arithmetic here is numpy on top of the oracle's C functions
(``fisher_score`` for log p(y | theta) and its gradient by Fisher's identity,
``kf``, ``rts_sample``, ``mh_chain``).  Pins: tests/test_oracle_gibbs.py (a long
chain's theta and x moments against quadrature of the posterior over theta with
the dense joint Gaussian; the same check fails with the MALA Hastings term
removed; the log-posterior gradient against central differences).
"""
from __future__ import annotations

import numpy as np

from . import EMIT_GAUSSIAN, Model, fisher_score, kf, mh_chain, rts_sample


def n_params(dx: int, dy: int) -> int:
    return dx * dx + dx + dy * dx + dy


def split(theta, dx: int, dy: int):
    """(F [dx,dx], logq [dx], H [dy,dx], logr [dy]) views of a flat theta."""
    theta = np.asarray(theta, dtype=np.float64)
    i = 0
    F = theta[i:i + dx * dx].reshape(dx, dx)
    i += dx * dx
    logq = theta[i:i + dx]
    i += dx
    H = theta[i:i + dy * dx].reshape(dy, dx)
    i += dy * dx
    logr = theta[i:i + dy]
    return F, logq, H, logr


def flat(F, logq, H, logr) -> np.ndarray:
    return np.concatenate([np.ravel(F), np.ravel(logq), np.ravel(H), np.ravel(logr)]).astype(
        np.float64)


def log_prior(theta, sd: float) -> float:
    theta = np.asarray(theta, dtype=np.float64)
    return float(-0.5 * (theta @ theta) / sd ** 2
                 - 0.5 * theta.size * np.log(2.0 * np.pi * sd ** 2))


def log_post_grad(m0, P0, y, theta, sd: float, dx: int, dy: int):
    """(log p(theta) + log p(y | theta), its gradient [p], log p(y | theta)).
    A failed filter gives NaN for all three."""
    F, logq, H, logr = split(theta, dx, dy)
    ll, dF, dq, dH, dr = fisher_score(m0, P0, F, logq, H, logr, y)
    theta = np.asarray(theta, dtype=np.float64)
    g = flat(dF, dq, dH, dr) - theta / sd ** 2
    return ll + log_prior(theta, sd), g, ll


def mala_log_q(to, frm, grad_frm, eps: float) -> float:
    """log density (up to its constant) of proposing `to` from `frm`."""
    r = np.asarray(to) - np.asarray(frm) - 0.5 * eps ** 2 * np.asarray(grad_frm)
    return float(-0.5 * (r @ r) / eps ** 2)


def gibbs_sweep(m0, P0, y, theta, logpost, grad, x, prior_sd: float, eps: float, xi_theta,
                u_theta: float, xi_x, delta: float, xi_path, u_path):
    """One sweep.  theta [p], logpost, grad [p]: the current point and its
    cached log posterior and gradient; x [N,dx]; xi_theta [p]; u_theta in
    (0,1); xi_x [N,dx] (refresh); xi_path [k,2,N,dx], u_path [k] (k may be 0).
    Returns a dict with the new state and every intermediate that the sweep
    decides on."""
    y = np.asarray(y, dtype=np.float64)
    N, dy = y.shape
    dx = len(m0)
    theta = np.asarray(theta, dtype=np.float64)
    grad = np.asarray(grad, dtype=np.float64)
    # 1. MALA on the theta-marginal
    prop = theta + 0.5 * eps ** 2 * grad + eps * np.asarray(xi_theta, dtype=np.float64)
    lp_p, g_p, ll_p = log_post_grad(m0, P0, y, prop, prior_sd, dx, dy)
    log_alpha = (lp_p - logpost + mala_log_q(theta, prop, g_p, eps)
                 - mala_log_q(prop, theta, grad, eps))
    acc = bool(np.isfinite(log_alpha) and np.log(u_theta) < log_alpha)
    if acc:
        theta, logpost, grad = prop, lp_p, g_p
    # 2. exact refresh of x given theta
    F, logq, H, logr = split(theta, dx, dy)
    Q = np.diag(np.exp(logq))
    R = np.diag(np.exp(logr))
    f = kf(m0, P0, F, Q, H, R, y)
    x_ref, rc = rts_sample(F, f["mf"], f["Pf"], f["mp"], f["Pp"], xi_x)
    out = dict(theta=theta.copy(), logpost=float(logpost), grad=grad.copy(), accepted_theta=acc,
               log_alpha=float(log_alpha), theta_prop=prop, logpost_prop=float(lp_p),
               loglik_prop=float(ll_p), x_refresh=x_ref, refresh_status=int(f["rc"] or rc))
    # 3. auxiliary Kalman path steps at theta
    xi_path = np.asarray(xi_path, dtype=np.float64)
    k = xi_path.shape[0] if xi_path.ndim == 4 else 0
    if k:
        M = Model(m0=np.asarray(m0, float), P0=np.asarray(P0, float), F=F.copy(), Q=Q,
                  emit=EMIT_GAUSSIAN, H=H.copy(), R=R)
        ch = mh_chain(M, y, x_ref, delta, 2, xi_path, np.asarray(u_path, dtype=np.float64),
                      keep_samples=False)
        out.update(x=ch["x"], path_log_ratio=ch["log_ratio"], path_accepted=ch["accepted"],
                   path_status=ch["status"])
    else:
        out.update(x=x_ref.copy(), path_log_ratio=np.zeros(0), path_accepted=np.zeros(0, int),
                   path_status=np.zeros(0, int))
    return out


def gibbs_init(m0, P0, y, theta, prior_sd: float):
    """(log posterior, gradient) at a starting theta."""
    y = np.asarray(y, dtype=np.float64)
    lp, g, _ = log_post_grad(m0, P0, y, theta, prior_sd, len(m0), y.shape[1])
    return lp, g
