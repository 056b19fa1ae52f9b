"""Seeded synthetic workloads shaped like the paper's experiments.

This module holds no part of the sampler's arithmetic: it only builds model
parameters, simulates observations from the model and draws the standard
normals / uniforms that the MCMC step consumes.  Both the GPU path and the CPU
oracle are fed from here.  Pure numpy; importing it does not load the HIP
library.

Seeds: model/data from ``default_rng(data_seed)``, step normals from
``default_rng(100 + cfg)``, uniforms from ``default_rng(200 + cfg)``.

Emission codes match the C-ABI: 0 Gaussian (H, R), 1 Poisson with log link,
2 Student-t at observation sites, 3 stochastic volatility (y ~ N(0, exp(x))),
4 multivariate t with a precision matrix, 5 Gaussian at observation sites (NaN =
not observed), 6 Gaussian around a quadratic mean at observation sites.  Dynamics: 0 linear (F, b), 1 Lorenz-63 and 2 Lorenz-96 Euler
steps.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

EMIT_GAUSSIAN, EMIT_POISSON_LOG, EMIT_STUDENT_T, EMIT_STOCH_VOL, EMIT_MVT = 0, 1, 2, 3, 4
EMIT_GAUSS_SITE, EMIT_GAUSS_QUAD = 5, 6
DYN_LINEAR, DYN_LORENZ63, DYN_LORENZ96 = 0, 1, 2


@dataclass
class Workload:
    """A state-space model with Gaussian dynamics and a chosen emission family,
    its observations y [N, dy], an initial path x0 [N, dx] and step settings."""
    name: str
    N: int
    m0: np.ndarray
    P0: np.ndarray
    F: np.ndarray
    Q: np.ndarray
    emit: int
    y: np.ndarray
    b: Optional[np.ndarray] = None
    H: Optional[np.ndarray] = None
    R: Optional[np.ndarray] = None
    site: Optional[np.ndarray] = None
    nu: float = 0.0
    scale: float = 0.0
    delta: float = 0.5
    order: int = 2
    seed: int = 0
    x_true: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)
    dyn: int = DYN_LINEAR
    dyn_par: tuple = (0.0, 0.0, 0.0, 0.0)
    obs_beta: float = 0.0
    slr_var: float = 0.0

    @property
    def dx(self) -> int:
        return int(self.m0.shape[0])

    @property
    def dy(self) -> int:
        return int(self.y.shape[1])

    def x_init(self) -> np.ndarray:
        """Initial chain state: the zero path (warm-up steps are not scored)."""
        return np.zeros((self.N, self.dx))

    def normals(self, n_steps: int, seed: Optional[int] = None) -> np.ndarray:
        """Standard normals [n_steps, 2, N, dx]: [:,0] for u, [:,1] for the path."""
        rng = np.random.default_rng(100 + self.seed if seed is None else seed)
        return rng.standard_normal((n_steps, 2, self.N, self.dx))

    def uniforms(self, n_steps: int, seed: Optional[int] = None) -> np.ndarray:
        """MH uniforms in (0, 1), [n_steps]."""
        rng = np.random.default_rng(200 + self.seed if seed is None else seed)
        u = rng.random(n_steps)
        return np.where(u <= 0.0, np.nextafter(0.0, 1.0), u)

    def oracle_kwargs(self) -> dict:
        return dict(m0=self.m0, P0=self.P0, F=self.F, Q=self.Q, emit=self.emit, b=self.b,
                    H=self.H, R=self.R, site=self.site, nu=self.nu, scale=self.scale,
                    dyn=self.dyn, dyn_par=tuple(self.dyn_par), obs_beta=self.obs_beta,
                    slr_var=self.slr_var)


def _simulate(rng, N, m0, P0, F, Q, b=None):
    """x_0 ~ N(m0, P0), x_t = F x_{t-1} + b + N(0, Q): all noise drawn at once."""
    d = len(m0)
    z = rng.standard_normal((N, d))
    e = z @ np.linalg.cholesky(Q).T
    if b is not None:
        e = e + b
    x = np.empty((N, d))
    x[0] = m0 + np.linalg.cholesky(P0) @ z[0]
    for t in range(1, N):
        x[t] = F @ x[t - 1] + e[t]
    return x


def rotation(theta: float) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    return np.array([[c, -s], [s, c]])


def random_stable_F(rng, d: int, rho: float) -> np.ndarray:
    """F = rho * G / spectral_radius(G), G with i.i.d. N(0,1) entries."""
    G = rng.standard_normal((d, d))
    return rho * G / np.max(np.abs(np.linalg.eigvals(G)))


def linear_gaussian_tiny(N: int = 64, seed: int = 0) -> Workload:
    """d_x = d_y = 2 linear-Gaussian SSM: F = 0.9 R(pi/8), Q = 0.1 I, H = I,
    R = 0.5 I, x0 ~ N(0, I); delta = 0.5, second-order proposal (exact)."""
    rng = np.random.default_rng(seed)
    d = 2
    m0, P0 = np.zeros(d), np.eye(d)
    F, Q = 0.9 * rotation(np.pi / 8), 0.1 * np.eye(d)
    H, R = np.eye(d), 0.5 * np.eye(d)
    x = _simulate(rng, N, m0, P0, F, Q)
    y = x @ H.T + rng.standard_normal((N, d)) @ np.linalg.cholesky(R).T
    return Workload("linear_gaussian_d2_N64", N, m0, P0, F, Q, EMIT_GAUSSIAN, y, H=H, R=R,
                    delta=0.5, order=2, seed=seed, x_true=x)


def poisson_ar1(N: int = 1024, d: int = 8, seed: int = 2) -> Workload:
    """d_x = d_y = 8 AR(1) latent (F = 0.95 I, Q = 0.2 I, x0 ~ N(0, I)) with
    y_{t,i} ~ Poisson(exp(x_{t,i})); delta = 0.2."""
    rng = np.random.default_rng(seed)
    m0, P0 = np.zeros(d), np.eye(d)
    F, Q = 0.95 * np.eye(d), 0.2 * np.eye(d)
    x = _simulate(rng, N, m0, P0, F, Q)
    y = rng.poisson(np.exp(x)).astype(np.float64)
    return Workload(f"poisson_ar1_d{d}_N{N}", N, m0, P0, F, Q, EMIT_POISSON_LOG, y,
                    site=np.arange(d, dtype=np.int32), delta=0.2, order=2, seed=seed, x_true=x)


def periodic_grid_F_Q(d: int = 64):
    """F = 0.9 I + 0.04 (P + P^T), P the cyclic shift; Q the squared-exponential
    kernel on the periodic grid, lengthscale 4, variance 0.1, plus 1e-6 I."""
    P = np.roll(np.eye(d), 1, axis=1)
    F = 0.9 * np.eye(d) + 0.04 * (P + P.T)
    i = np.arange(d)
    dist = np.abs(i[:, None] - i[None, :])
    dist = np.minimum(dist, d - dist)
    Q = 0.1 * np.exp(-dist.astype(float) ** 2 / (2 * 4.0 ** 2)) + 1e-6 * np.eye(d)
    return F, Q


# Step size for the latent-field workload, frozen after a 400-step Robbins-Monro warm-up
# toward 30% acceptance (paper_2303_00301_amd.mcmc.tune_delta, seed 7); 300 frozen steps
# then accepted 30.0%.
LATENT_FIELD_DELTA = 0.057


def latent_field(N: int = 4096, d: int = 64, n_sites: int = 32, nu: float = 3.0,
                 scale: float = 0.5, seed: int = 3, delta: Optional[float] = None) -> Workload:
    """d_x = 64 latent field on a 1-D periodic grid (periodic_grid_F_Q), observed
    at n_sites evenly spaced sites through Student-t(nu, scale) noise."""
    rng = np.random.default_rng(seed)
    m0, P0 = np.zeros(d), np.eye(d)
    F, Q = periodic_grid_F_Q(d)
    x = _simulate(rng, N, m0, P0, F, Q)
    site = (np.arange(n_sites) * (d // n_sites)).astype(np.int32)
    y = x[:, site] + scale * rng.standard_t(nu, size=(N, n_sites))
    return Workload(f"latent_field_d{d}_N{N}", N, m0, P0, F, Q, EMIT_STUDENT_T, y, site=site,
                    nu=nu, scale=scale, delta=LATENT_FIELD_DELTA if delta is None else delta,
                    order=2, seed=seed, x_true=x)


# Step size of the quadratic-observation field under order 3 (the latent field's
# order-2 value; the proposal's curvature here comes from the fitted Gaussian).
QUAD_FIELD_DELTA = 0.057


def quadratic_obs_field(N: int = 4096, d: int = 64, n_sites: int = 32, beta: float = 0.2,
                        scale: float = 0.5, slr_var: float = 0.05, seed: int = 9,
                        delta: Optional[float] = None, repeat_sites: int = 0) -> Workload:
    """The latent field's dynamics (periodic_grid_F_Q) observed through a
    nonlinear mean: y_{t,k} = z + beta z^2 + N(0, scale^2), z = x_t[site[k]], at
    n_sites evenly spaced sites, the first `repeat_sites` of them observed by a
    second site as well.  Sampled with order 3: the observation model is
    replaced, around the path, by the Gaussian of the statistical linear
    regression with reference variance slr_var."""
    rng = np.random.default_rng(seed)
    m0, P0 = np.zeros(d), np.eye(d)
    F, Q = periodic_grid_F_Q(d)
    x = _simulate(rng, N, m0, P0, F, Q)
    base = (np.arange(n_sites) * (d // n_sites)).astype(np.int32)
    site = np.concatenate([base, base[:repeat_sites]]).astype(np.int32)
    z = x[:, site]
    y = np.ascontiguousarray(z + beta * z * z + scale * rng.standard_normal(z.shape))
    return Workload(f"quadratic_obs_field_d{d}_N{N}", N, m0, P0, F, Q, EMIT_GAUSS_QUAD, y,
                    site=site, scale=scale, delta=QUAD_FIELD_DELTA if delta is None else delta,
                    order=3, seed=seed, x_true=x, obs_beta=beta, slr_var=slr_var)


# Step sizes of the stochastic-volatility workload (d = 30, T = 250, seed 6) toward
# the paper's 50% acceptance: a 600-step Robbins-Monro warm-up on log delta (gain
# k^-0.6, the recursion of paper_2303_00301_amd.mcmc.tune_delta) started at the
# simulated path, then frozen; 400 frozen steps accepted 47% (order 1) and 49%
# (order 2).
STOCH_VOL_DELTA = {1: 0.039, 2: 0.091}


def stoch_vol(N: int = 250, d: int = 30, order: int = 2, seed: int = 6,
              delta: Optional[float] = None) -> Workload:
    """Multivariate stochastic volatility (Sec. "Multivariate stochastic
    volatility model"): F = phi I, Q_ij = tau (1 if i = j else rho) with
    phi = 0.9, tau = 2, rho = 0.25, x_0 from the stationary law
    N(0, Q / (1 - phi^2)), and y_t(k) ~ N(0, exp(x_t(k))) for every coordinate."""
    rng = np.random.default_rng(seed)
    phi, tau, rho = 0.9, 2.0, 0.25
    F = phi * np.eye(d)
    Q = tau * (rho * np.ones((d, d)) + (1.0 - rho) * np.eye(d))
    m0, P0 = np.zeros(d), Q / (1.0 - phi * phi)
    x = _simulate(rng, N, m0, P0, F, Q)
    y = np.exp(0.5 * x) * rng.standard_normal((N, d))
    return Workload(f"stoch_vol_d{d}_N{N}", N, m0, P0, F, Q, EMIT_STOCH_VOL, y,
                    site=np.arange(d, dtype=np.int32),
                    delta=STOCH_VOL_DELTA[order] if delta is None else delta, order=order,
                    seed=seed, x_true=x)


def lattice_precision(side: int = 8, tau: float = -0.25, r: int = 1) -> np.ndarray:
    """Precision of the spatio-temporal observation noise on a side x side
    lattice (node k = i * side + j): tau ** D for a Manhattan distance D <= r,
    else 0 (so 1 on the diagonal)."""
    ij = np.array([(i, j) for i in range(side) for j in range(side)])
    D = np.abs(ij[:, None, :] - ij[None, :, :]).sum(-1)
    return np.where(D <= r, np.power(tau, D.astype(np.float64)), 0.0)


# Step size of the spatio-temporal workload (side 8, T = 1024, seed 8), first order,
# toward the paper's 50% acceptance: a 600-step Robbins-Monro warm-up on log delta
# (gain k^-0.6, the recursion of paper_2303_00301_amd.mcmc.tune_delta) started at the
# simulated path on the oracle's factorised step, then frozen; 400 frozen steps
# accepted 55%.
SPATIO_TEMPORAL_DELTA = 0.0051


def spatio_temporal(N: int = 1024, side: int = 8, nu: float = 1.0, tau: float = -0.25,
                    sigma_x: float = 1.0, seed: int = 8, delta: Optional[float] = None) -> Workload:
    """Spatio-temporal model (Sec. "Spatio-temporal model"): independent random
    walks X_t(i, j) = X_{t-1}(i, j) + N(0, sigma_x^2) on a side x side lattice,
    observed as Y_t = X_t + V_t with V_t multivariate t (nu degrees of freedom)
    whose precision is lattice_precision(side, tau, 1).  x_0 ~ N(0, sigma_x^2 I).
    First-order proposals: the auxiliary model factorises over the lattice."""
    rng = np.random.default_rng(seed)
    d = side * side
    m0, P0 = np.zeros(d), sigma_x ** 2 * np.eye(d)
    F, Q = np.eye(d), sigma_x ** 2 * np.eye(d)
    x = _simulate(rng, N, m0, P0, F, Q)
    R = lattice_precision(side, tau, 1)
    Lc = np.linalg.cholesky(np.linalg.inv(R))
    z = rng.standard_normal((N, d)) @ Lc.T
    w = rng.chisquare(nu, size=(N, 1))
    y = x + z * np.sqrt(nu / w)
    return Workload(f"spatio_temporal_{side}x{side}_N{N}", N, m0, P0, F, Q, EMIT_MVT, y, R=R,
                    site=np.arange(d, dtype=np.int32), nu=nu,
                    delta=SPATIO_TEMPORAL_DELTA if delta is None else delta, order=1,
                    seed=seed, x_true=x)


def euler_drift(dyn: int, par, x: np.ndarray) -> np.ndarray:
    """beta(x) of the Lorenz-63 (dyn 1) or Lorenz-96 (dyn 2) SDE, for simulating
    data; the samplers evaluate the dynamics themselves."""
    if dyn == DYN_LORENZ63:
        t1, t2, t3 = par[:3]
        return np.array([t1 * (x[1] - x[0]), t2 * x[0] - x[1] - x[0] * x[2],
                         x[0] * x[1] - t3 * x[2]])
    return (np.roll(x, -1) - np.roll(x, 2)) * np.roll(x, 1) - x + par[0]


def _simulate_sde(rng, N, m0, P0, dyn, par, dt, sigma):
    d = len(m0)
    x = np.zeros((N, d))
    x[0] = m0 + np.linalg.cholesky(P0) @ rng.standard_normal(d)
    for t in range(1, N):
        x[t] = x[t - 1] + dt * euler_drift(dyn, par, x[t - 1]) + \
            sigma * np.sqrt(dt) * rng.standard_normal(d)
    return x


# Step size of the Lorenz-63 workload (seed 9), second order.  On the oracle, 60
# steps from the prior-simulated start accepted 95% at this delta and 2.5% at
# delta = 100; from the simulated path, 77% at delta = 1e6, where the u_t carry
# almost no information, matching the paper's report that its adaptation drove
# delta to very large values at about 70% acceptance.
LORENZ63_DELTA = 1.0


def lorenz63(N: int = 10001, dt: float = 2e-4, obs_every: int = 50, sigma: float = 3.0,
             seed: int = 9, delta: Optional[float] = None) -> Workload:
    """Lorenz-63 SDE dx = beta_theta(x) dt + sigma dW with theta = (10, 28, 8/3)
    (Sec. "Parameter estimation in a continuous-discrete diffusion smoothing
    problem"), Euler-Maruyama on a fine grid of step dt over [0, (N-1) dt],
    x_2 and x_3 observed every obs_every steps with N(0, 5) noise (NaN
    elsewhere).  x_0 ~ N((1.5, -1.5, 25), I).  The chain starts from a path
    simulated from the prior dynamics (another seed), as in that experiment."""
    rng = np.random.default_rng(seed)
    par = (10.0, 28.0, 8.0 / 3.0, dt)
    m0, P0 = np.array([1.5, -1.5, 25.0]), np.eye(3)
    Q = sigma ** 2 * dt * np.eye(3)
    x = _simulate_sde(rng, N, m0, P0, DYN_LORENZ63, par, dt, sigma)
    y = np.full((N, 2), np.nan)
    obs = np.arange(0, N, obs_every)
    y[obs] = x[obs][:, 1:] + np.sqrt(5.0) * rng.standard_normal((len(obs), 2))
    x_start = _simulate_sde(np.random.default_rng(seed + 1000), N, m0, P0, DYN_LORENZ63, par, dt,
                            sigma)
    return Workload(f"lorenz63_dt{dt:g}_N{N}", N, m0, P0, None, Q, EMIT_GAUSS_SITE, y,
                    site=np.array([1, 2], np.int32), scale=np.sqrt(5.0),
                    delta=LORENZ63_DELTA if delta is None else delta, order=2, seed=seed,
                    x_true=x, dyn=DYN_LORENZ63, dyn_par=par, extra={"x_start": x_start})


def lorenz96(N: int = 2048, d: int = 40, dt: float = 0.005, forcing: float = 8.0,
             sigma: float = 0.5, n_sites: int = 20, seed: int = 10,
             delta: Optional[float] = None) -> Workload:
    """Lorenz-96 SDE (d coordinates on a ring, forcing 8), Euler-Maruyama with
    step dt and noise sigma dW, every other coordinate observed with Student-t
    noise (nu = 3, scale 0.5) at every step; second order."""
    rng = np.random.default_rng(seed)
    par = (forcing, dt, 0.0, 0.0)
    m0, P0 = forcing * np.ones(d), np.eye(d)
    x = _simulate_sde(rng, N, m0, P0, DYN_LORENZ96, par, dt, sigma)
    site = (np.arange(n_sites) * (d // n_sites)).astype(np.int32)
    y = x[:, site] + 0.5 * rng.standard_t(3.0, size=(N, n_sites))
    return Workload(f"lorenz96_d{d}_N{N}", N, m0, P0, None, sigma ** 2 * dt * np.eye(d),
                    EMIT_STUDENT_T, y, site=site, nu=3.0, scale=0.5,
                    delta=0.05 if delta is None else delta, order=2, seed=seed, x_true=x,
                    dyn=DYN_LORENZ96, dyn_par=par)


def ragged_poisson_batch(n_chains: int = 512, n_min: int = 128, n_max: int = 8192,
                         dims=(4, 16, 32), seed: int = 4, delta: float = 0.1) -> List[Workload]:
    """Independent chains with N_i ~ U{n_min..n_max}, d_i ~ U(dims), random stable
    F_i (spectral radius ~ U(0.5, 0.95)), Q = 0.1 I, P0 = I, Poisson log-link
    emissions with d_y = d_x."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_chains):
        N = int(rng.integers(n_min, n_max + 1))
        d = int(rng.choice(dims))
        rho = float(rng.uniform(0.5, 0.95))
        F = random_stable_F(rng, d, rho)
        Q = 0.1 * np.eye(d)
        m0, P0 = np.zeros(d), np.eye(d)
        x = _simulate(rng, N, m0, P0, F, Q)
        y = rng.poisson(np.exp(np.clip(x, -30, 10))).astype(np.float64)
        out.append(Workload(f"chain{c}_d{d}_N{N}", N, m0, P0, F, Q, EMIT_POISSON_LOG, y,
                            site=np.arange(d, dtype=np.int32), delta=delta, order=2,
                            seed=1000 * seed + c, x_true=x))
    return out


@dataclass
class LGSSMTheta:
    F: np.ndarray
    logq: np.ndarray
    H: np.ndarray
    logr: np.ndarray

    def flat(self) -> np.ndarray:
        return np.concatenate([self.F.ravel(), self.logq, self.H.ravel(), self.logr])


@dataclass
class ParamWorkload:
    name: str
    N: int
    m0: np.ndarray
    P0: np.ndarray
    y: np.ndarray
    theta_true: LGSSMTheta
    theta0: LGSSMTheta


def lgssm_params(N: int = 16384, dx: int = 32, dy: int = 16, seed: int = 5) -> ParamWorkload:
    """Linear-Gaussian SSM for parameter gradients: theta = (F, log diag Q, H,
    log diag R).  True: F (spectral radius 0.9), Q = 0.1 I, H ~ N(0, 1/32),
    R = 0.5 I; y simulated from seed.  Evaluation point theta0 drawn fresh."""
    rng = np.random.default_rng(seed)
    m0, P0 = np.zeros(dx), np.eye(dx)
    Ft = random_stable_F(rng, dx, 0.9)
    Ht = rng.normal(0.0, np.sqrt(1.0 / 32), size=(dy, dx))
    tt = LGSSMTheta(Ft, np.full(dx, np.log(0.1)), Ht, np.full(dy, np.log(0.5)))
    x = _simulate(rng, N, m0, P0, Ft, 0.1 * np.eye(dx))
    y = x @ Ht.T + np.sqrt(0.5) * rng.standard_normal((N, dy))
    rng0 = np.random.default_rng(seed + 1000)
    t0 = LGSSMTheta(random_stable_F(rng0, dx, 0.9),
                    np.log(0.1) + 0.1 * rng0.standard_normal(dx),
                    rng0.normal(0.0, np.sqrt(1.0 / 32), size=(dy, dx)),
                    np.log(0.5) + 0.1 * rng0.standard_normal(dy))
    return ParamWorkload(f"lgssm_params_dx{dx}_dy{dy}_N{N}", N, m0, P0, y, tt, t0)
