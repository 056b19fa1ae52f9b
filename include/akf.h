/*
 * akf.h -- C ABI of the MI355X auxiliary Kalman MCMC library (libauxkf.so).
 *
 * Method: Corenflos & Sarkka, "Auxiliary MCMC samplers for parallelisable
 * inference in high-dimensional latent dynamical systems" (arXiv 2303.00301).
 * A state-space model has Gaussian dynamics p_0 = N(m0, P0),
 * p_t(x_t | x_{t-1}) = N(F x_{t-1} + b, Q) and emission densities h_t(y_t | x_t)
 * (Sec. 2.2, eq. gaussian-FK).  One MCMC step (Alg. "General Auxiliary Kalman
 * sampler" with Sigma_t = I) draws u_t = x_t + sqrt(delta/2) xi^u_t, linearises
 * log h_t at the current path (first order, eq. gaussian-FK-proposal, or second
 * order, eq. second-order), samples a proposal x* from the resulting auxiliary
 * linear-Gaussian model with a parallel-in-time Kalman filter and pathwise
 * backward sampler (App. A, "Prefix-sums and the parallel Kalman filter",
 * "Parallel Rauch--Tung--Striebel sampler"), and accepts it with the Hastings
 * ratio of the augmented target pi(x, u).
 *
 * Conventions for every entry point:
 *   - Arrays are DEVICE pointers to row-major float64 data, owned by the caller;
 *     the library never allocates, frees or retains them.  Every call is
 *     enqueued on `stream` (a hipStream_t; NULL = the default stream) and is
 *     asynchronous with respect to the host.
 *   - Scratch memory is the caller's `ws` buffer of `ws_bytes` bytes (device,
 *     256-byte aligned); query its size with the matching *_workspace_bytes
 *     call.  A workspace must not be shared by calls that may overlap.
 *   - Synchronous errors (bad arguments, unsupported sizes, launch failures)
 *     are returned as akf_status; akf_last_error() describes the last one on
 *     the calling thread.  Numerical failures are asynchronous and reported
 *     in the per-step device status word (AKF_ST_* bits); a step with a
 *     non-zero status rejects (x_out = x_in).
 *   - Sizes: 1 <= dx <= 64, 1 <= dy <= 64, N >= 1.
 */
#ifndef AKF_H
#define AKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AKF_OK = 0,
  AKF_ERR_INVALID = 1,     /* null pointer, bad enum, delta <= 0, ... */
  AKF_ERR_SHAPE = 2,       /* sizes outside the supported range */
  AKF_ERR_WORKSPACE = 3,   /* ws_bytes smaller than required, or misaligned */
  AKF_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
  AKF_ERR_UNSUPPORTED = 5  /* valid request the library does not implement */
} akf_status;

typedef enum {
  AKF_EMIT_GAUSSIAN = 0,    /* y_t = H x_t + N(0, R): H [dy,dx], R [dy,dy] SPD */
  AKF_EMIT_POISSON_LOG = 1, /* y_{t,k} ~ Poisson(exp(x_{t,site[k]})) */
  AKF_EMIT_STUDENT_T = 2,   /* y_{t,k} = x_{t,site[k]} + scale * t_nu */
  AKF_EMIT_STOCH_VOL = 3,   /* y_{t,k} ~ N(0, exp(x_{t,site[k]})) (stochastic volatility) */
  AKF_EMIT_MVT = 4,         /* y_t = x_t[site] + V_t, V_t multivariate t with nu degrees of
                               freedom and precision R [dy,dy] (Sec. "Spatio-temporal model");
                               first-order proposals only */
  AKF_EMIT_GAUSS_SITE = 5,  /* y_{t,k} = x_{t,site[k]} + N(0, scale^2) */
  AKF_EMIT_GAUSS_QUAD = 6   /* y_{t,k} = z + obs_beta z^2 + N(0, scale^2), z = x_{t,site[k]}
                               (a nonlinear observation mean, for order 3) */
} akf_emit;

/* Dynamics families: x_t = F x_{t-1} + b + N(0, Q), or x_t = f(x_{t-1}) + N(0, Q)
 * with f one Euler-Maruyama step of an SDE dx = beta(x) dt + noise. */
typedef enum {
  AKF_DYN_LINEAR = 0,    /* F, b */
  AKF_DYN_LORENZ63 = 1,  /* dx = 3; beta = (p0 (x1 - x0), p1 x0 - x1 - x0 x2, x0 x1 - p2 x2),
                            dt = p3 (Sec. "Parameter estimation in a continuous-discrete
                            diffusion smoothing problem") */
  AKF_DYN_LORENZ96 = 2   /* dx >= 4; beta_i = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + p0 (cyclic),
                            dt = p1 */
} akf_dyn;

/* Arithmetic and storage type of the path's internals (the boundary arrays
 * are float64 whatever the selection).  The MH step and every covariance-form
 * entry point compute in FP64: on gfx950 plain FP32 vector arithmetic has the
 * FP64 rate and FP32 matrix cores twice the FP64 rate, and the paper reports
 * its parallel Kalman sampler diverging in FP32 (Sec. "Multivariate stochastic
 * volatility model"), so they reject AKF_F32 with AKF_ERR_UNSUPPORTED.  The
 * square-root filter and sampler (akf_sqrt_filter_sample), the form built for
 * FP32, take either. */
typedef enum {
  AKF_F64 = 0, /* default: a zero-initialised model selects it */
  AKF_F32 = 1
} akf_dtype;

/* Per-step device status bits. */
enum {
  AKF_ST_FWD_NOT_PD = 1, /* forward proposal undefined: 2/delta - Lambda_t not PD,
                            or a Cholesky pivot <= 0 in the forward filter/sampler */
  AKF_ST_REV_NOT_PD = 2, /* same for the reverse proposal at x* */
  AKF_ST_NONFINITE = 4   /* the log ratio is not finite */
};
/* When the forward proposal fails only AKF_ST_FWD_NOT_PD is reported, since x*
 * and everything derived from it are then undefined. */

/*
 * Model description (eq. ssm with Gaussian dynamics).  m0 [dx], P0 [dx,dx],
 * F [dx,dx], b [dx] or NULL (zero), Q [dx,dx].  Emission per `emit`:
 * GAUSSIAN uses H, R; POISSON_LOG, STUDENT_T, STOCH_VOL, MVT, GAUSS_SITE and
 * GAUSS_QUAD use site [dy] (int32, each in [0, dx); several sites may observe
 * the same coordinate); STUDENT_T also nu > 0 and scale > 0; GAUSS_SITE and
 * GAUSS_QUAD scale > 0 (GAUSS_QUAD also obs_beta); MVT also the precision
 * R [dy,dy] (symmetric positive definite) and nu > 0.  In the site-wise
 * families (POISSON_LOG, STUDENT_T, STOCH_VOL, GAUSS_SITE, GAUSS_QUAD) a NaN
 * y_{t,k} marks an unobserved site.  All pointers are device pointers.
 * MVT with order 2 is rejected with AKF_ERR_UNSUPPORTED (its Hessian would
 * make Omega_t dense and time-varying).
 *
 * dyn selects the dynamics (akf_dyn; zero-initialise the struct for linear
 * dynamics).  With a nonlinear family F and b are ignored (may be NULL), Q is
 * the per-step noise covariance and dyn_par holds the family's parameters;
 * each step linearises f around the current path (x for the forward proposal,
 * x* for the reverse one; Example "gslr-example") and adds the mismatch
 * between the true and the linearised transition densities to log r.
 * Nonlinear dynamics are accepted by akf_mh_step / akf_mh_run only.
 *
 * dtype (akf_dtype) selects the internal arithmetic; every entry point taking
 * a model but akf_sqrt_filter_sample returns AKF_ERR_UNSUPPORTED for AKF_F32
 * (and AKF_ERR_INVALID for an unknown value), the workspace queries return 0.
 */
typedef struct akf_model {
  int32_t N, dx, dy;
  const double *m0, *P0, *F, *b, *Q;
  int32_t emit;
  const double *H, *R;
  const int32_t* site;
  double nu, scale;
  int32_t dyn;
  double dyn_par[4];
  int32_t dtype;
  double obs_beta; /* GAUSS_QUAD: coefficient of the quadratic term of the observation mean */
  double slr_var;  /* order 3: reference variance gamma^2 >= 0 of the observation-model
                      linearisation (0 = the Taylor limit) */
} akf_model;

/* Description of the last synchronous error on this thread (static storage). */
const char* akf_last_error(void);

/*
 * Workspace bytes for akf_mh_step / akf_mh_run on this model.  `block` is the
 * number of time steps per scan block (0 = automatic); pass the same value to
 * the step call.  Returns 0 when the model sizes are unsupported.
 */
size_t akf_mh_workspace_bytes(const akf_model* model, int32_t order, int32_t block);

/*
 * One auxiliary Kalman MH step (Alg. "General Auxiliary Kalman sampler").
 *   y      [N,dy]     observations
 *   x_in   [N,dx]     current path
 *   delta  > 0        auxiliary step size (u_t ~ N(x_t, delta/2 I))
 *   order  1, 2 or 3  linearisation of log h_t: 1 and 2 take log h_t's own
 *                     gradient (and Hessian) at the path (eq. gaussian-FK-proposal,
 *                     eq. second-order); 3 replaces h_t by a Gaussian
 *                     N(H_t z + c_t, R_t) fitted around the path by statistical
 *                     linear regression with reference variable N(x_t, slr_var I)
 *                     (eq. observation-approx, eq. coeffs, eq. general-GSLR-coeffs)
 *                     and takes that Gaussian's gradient and Hessian
 *                     (eq. two-lin-prop); order 3 needs GAUSS_SITE or GAUSS_QUAD
 *                     (AKF_ERR_UNSUPPORTED otherwise) and slr_var >= 0.  The
 *                     target keeps the true h_t in every order.
 *   xi     [2,N,dx]   standard normals: xi[0] for u, xi[1] for the path sample
 *   unif   [1]        uniform in (0,1) for the accept test (accept iff log unif < log r)
 *   x_out  [N,dx]     new path (x* if accepted, else x_in); may alias x_in
 *   log_ratio, logZ_fwd, logZ_rev [1] double, accepted, status [1] int32: optional
 *                     (NULL = not written).  logZ_* are the log marginal
 *                     likelihoods of the pseudo-observations under the forward
 *                     (at x) and reverse (at x*) auxiliary models; log_ratio is
 *                     -inf when status != 0.
 */
akf_status akf_mh_step(const akf_model* model, const double* y, const double* x_in, double delta,
                       int32_t order, const double* xi, const double* unif, double* x_out,
                       double* log_ratio, int32_t* accepted, double* logZ_fwd, double* logZ_rev,
                       int32_t* status, void* ws, size_t ws_bytes, int32_t block, void* stream);

/*
 * n_steps MH steps on one chain, x updated in place.  xi [n_steps,2,N,dx],
 * unif [n_steps]; per-step outputs are arrays of n_steps (each may be NULL).
 * Same workspace as akf_mh_step.
 */
akf_status akf_mh_run(const akf_model* model, const double* y, double* x, double delta,
                      int32_t order, int32_t n_steps, const double* xi, const double* unif,
                      double* log_ratio, int32_t* accepted, double* logZ_fwd, double* logZ_rev,
                      int32_t* status, void* ws, size_t ws_bytes, int32_t block, void* stream);

/*
 * akf_mh_step without a workspace, for callers that cannot allocate device
 * memory (work under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments and outputs are akf_mh_step's; the scratch memory is a
 * fixed array of AKF_NOALLOC_SCRATCH_BYTES bytes inside the library, one per
 * device (each device holds it until the process ends).  The call allocates
 * and frees nothing.
 *   - Limit: a problem whose akf_mh_workspace_bytes(model, order, block)
 *     exceeds AKF_NOALLOC_SCRATCH_BYTES returns AKF_ERR_SHAPE (64 MiB covers,
 *     e.g., dx = 8 at N = 1024, dx = 30 at N = 250, dx = 64 at N = 96).
 *   - Every call on one device shares that device's array: calls that may
 *     overlap on one device (other streams, other host threads) race; order
 *     them on one stream.  The array keeps the last call's contents; the step
 *     initialises everything it reads, so no clearing is needed between calls.
 *   - `stream` must belong to the current device (AKF_ERR_INVALID otherwise).
 */
#define AKF_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
akf_status akf_mh_step_noalloc(const akf_model* model, const double* y, const double* x_in,
                               double delta, int32_t order, const double* xi, const double* unif,
                               double* x_out, double* log_ratio, int32_t* accepted,
                               double* logZ_fwd, double* logZ_rev, int32_t* status, int32_t block,
                               void* stream);

/*
 * n_steps first-order MH steps (Sec. "Auxiliary Kalman sampler", eq.
 * gaussian-FK-proposal, order fixed at 1) on one chain, with the auxiliary
 * model's matrices formed once per call.  Under order 1, Omega_t = delta/2 I
 * whatever the path, so the forward and reverse auxiliary models of every
 * step share their covariances (P^p_t, S_t, P^f_t, E_t, L_t); only the means
 * depend on the path.  The first step runs the full filter and sampler and
 * keeps S_t^{-1}, log det S_t, E_t and chol(L_t); every later proposal is
 * matrix-vector work.  Arguments, outputs, normals and status bits as
 * akf_mh_run with order = 1; the chain is the same up to rounding.
 *   - model: linear dynamics (AKF_ERR_UNSUPPORTED otherwise); any emission.
 *   - workspace: akf_mh_first_order_workspace_bytes (that of akf_mh_run plus
 *     three [N, D, D] matrices, D the padded width 16, 32 or 64); its
 *     contents do not carry over between calls.
 */
size_t akf_mh_first_order_workspace_bytes(const akf_model* model, int32_t block);
akf_status akf_mh_run_first_order(const akf_model* model, const double* y, double* x,
                                  double delta, int32_t n_steps, const double* xi,
                                  const double* unif, double* log_ratio, int32_t* accepted,
                                  double* logZ_fwd, double* logZ_rev, int32_t* status, void* ws,
                                  size_t ws_bytes, int32_t block, void* stream);

/*
 * n_steps MH steps of order 1 or 2 on one chain reusing the auxiliary model's
 * matrices wherever they are unchanged (the matrix parts A, C, J of the filter
 * elements, and everything built from them, depend on x only through
 * Omega_t, never on u).  Order 1: as akf_mh_run_first_order.  Order 2:
 * Omega_t depends on x, so a forward proposal after a rejected step (same x,
 * new u) reuses the covariances of the forward proposal before it and is
 * matrix-vector work; after an accepted or failed step, and at step 0, the
 * forward proposal runs in full and keeps its matrices; the reverse proposal
 * (a new x* every step) always runs in full.  The branch is decided on the
 * device: each step issues the launches of both forward branches, gated on a
 * workspace word that the step's decision updates, so the call never
 * synchronises with the host, returns once the steps are enqueued, and can be
 * captured in a graph (the first step initialises the word; a replay must
 * start from step 0 of its own capture).  Arguments, outputs, normals and
 * status bits as akf_mh_run; the chain equals akf_mh_run's up to rounding.
 *   - model: linear dynamics; order 2 takes the diagonal-Omega families
 *     (POISSON_LOG, STUDENT_T, STOCH_VOL, GAUSS_SITE), AKF_ERR_UNSUPPORTED
 *     for GAUSSIAN; MVT needs order 1 as everywhere.
 *   - workspace: akf_mh_reuse_workspace_bytes (that of
 *     akf_mh_run_first_order).
 */
size_t akf_mh_reuse_workspace_bytes(const akf_model* model, int32_t order, int32_t block);
akf_status akf_mh_run_reuse(const akf_model* model, const double* y, double* x, double delta,
                            int32_t order, int32_t n_steps, const double* xi, const double* unif,
                            double* log_ratio, int32_t* accepted, double* logZ_fwd,
                            double* logZ_rev, int32_t* status, void* ws, size_t ws_bytes,
                            int32_t block, void* stream);

/*
 * Factorised step (Sec. "Spatio-temporal model").  When P0, F and Q are
 * diagonal the prior is a product over coordinates; with a diagonal Omega_t
 * (first order, or second order with the POISSON_LOG, STUDENT_T or STOCH_VOL
 * families, whose Hessians are diagonal) the auxiliary linear-Gaussian model
 * is then dx independent scalar models, while the target stays coupled
 * through h_t.  These entry points run the same MH step as akf_mh_step /
 * akf_mh_run (same arguments, outputs, status bits and normals) with dx scalar
 * filters and samplers in place of the dense ones.
 *   - model->P0, model->F and model->Q point to the DIAGONALS, [dx] each;
 *     m0 [dx] and b [dx] (or NULL) as usual.
 *   - emission: any family but GAUSSIAN (AKF_ERR_UNSUPPORTED); MVT needs
 *     order 1.
 *   - no scan-block argument: one workgroup per coordinate walks time in
 *     chunks of at most 2048 steps.
 */
size_t akf_mh_factorised_workspace_bytes(const akf_model* model, int32_t order);
akf_status akf_mh_step_factorised(const akf_model* model, const double* y, const double* x_in,
                                  double delta, int32_t order, const double* xi,
                                  const double* unif, double* x_out, double* log_ratio,
                                  int32_t* accepted, double* logZ_fwd, double* logZ_rev,
                                  int32_t* status, void* ws, size_t ws_bytes, void* stream);
akf_status akf_mh_run_factorised(const akf_model* model, const double* y, double* x, double delta,
                                 int32_t order, int32_t n_steps, const double* xi,
                                 const double* unif, double* log_ratio, int32_t* accepted,
                                 double* logZ_fwd, double* logZ_rev, int32_t* status, void* ws,
                                 size_t ws_bytes, void* stream);

/*
 * Parallel-in-time Kalman filter of the auxiliary linear-Gaussian model
 * x_t = F x_{t-1} + b + N(0,Q), omega_t = x_t + N(0, diag(Omega_t))
 * (App. A, "Prefix-sums and the parallel Kalman filter"; likelihood in the
 * predictive form of eq. marginal-likelihood).  The model's emission fields
 * are ignored.  omega, Omega [N,dx]; outputs mf [N,dx], Pf [N,dx,dx] (each may
 * be NULL), ell [N] per-step log-likelihood terms.  *status (device int32, may
 * be NULL) receives AKF_ST_FWD_NOT_PD when a matrix that must be positive
 * definite is not (a non-positive pivot), else 0.
 */
size_t akf_filter_workspace_bytes(const akf_model* model, int32_t block);
akf_status akf_aux_filter(const akf_model* model, const double* omega, const double* Omega,
                          double* mf, double* Pf, double* ell, int32_t* status, void* ws,
                          size_t ws_bytes, int32_t block, void* stream);

/*
 * Pathwise sampler (App. A, "Parallel Rauch--Tung--Striebel sampler"): from the
 * filtering moments mf [N,dx], Pf [N,dx,dx] of the model's dynamics, returns
 * x [N,dx] with x_{N-1} = mf + chol(Pf) xi_{N-1} and
 * x_t = mf_t + G_t (x_{t+1} - F mf_t - b) + chol(Sigma_t) xi_t (chol = lower
 * Cholesky factor with positive diagonal), xi [N,dx] standard normals.
 */
size_t akf_sampler_workspace_bytes(const akf_model* model, int32_t block);
akf_status akf_rts_sample(const akf_model* model, const double* mf, const double* Pf,
                          const double* xi, double* x, int32_t* status, void* ws,
                          size_t ws_bytes, int32_t block, void* stream);

/*
 * Square-root form of the parallel filter and of the pathwise sampler, the
 * form the paper points to for FP32 robustness (Sec. "Multivariate stochastic
 * volatility model": its parallel Kalman sampler diverged in FP32).  Same
 * auxiliary model as akf_aux_filter (x_t = F x_{t-1} + b + N(0, Q),
 * omega_t = x_t + N(0, diag(Omega_t)); emission fields ignored) and the same
 * results up to rounding, with every covariance carried as a lower-triangular
 * factor and every covariance update a triangularisation (Householder, in
 * double): filtering elements (A, b, U, eta, Z) with C = U U^T, J = Z Z^T
 * (App. A, "Prefix-sums and the parallel Kalman filter", in factor form),
 * sampling elements E_t and chol(L_t) from one triangularisation per step
 * (App. A, "Parallel Rauch--Tung--Striebel sampler").
 *   - model->dtype selects the storage and arithmetic of every matrix and
 *     vector: AKF_F32 or AKF_F64 (the triangularisations and the likelihood
 *     sums accumulate in double either way).  1 <= dx <= 32; linear dynamics.
 *   - omega, Omega [N,dx] (Omega: the diagonal variances, > 0);
 *     mf [N,dx] filtering means (required); Uf [N,dx,dx] the lower factors of
 *     the filtering covariances (P^f_t = Uf_t Uf_t^T) or NULL; ell [N] the
 *     per-step predictive log-likelihood terms or NULL; logZ [1] their sum or
 *     NULL (NaN when *status != 0).
 *   - xi [N,dx] standard normals and x_out [N,dx]: the path sample, with
 *     x_{N-1} = mf + Uf xi_{N-1}, x_t = mf_t + E_t (x_{t+1} - F mf_t - b) +
 *     chol(L_t) xi_t (the noise map of akf_rts_sample); x_out NULL skips the
 *     sampler (xi may then be NULL).
 *   - *status (device int32, may be NULL): AKF_ST_FWD_NOT_PD when Q or P0 is
 *     not positive definite or a factor has a non-positive pivot, else 0.
 *   - workspace: akf_sqrt_workspace_bytes(model, block); block = time steps
 *     per scan block (0 = automatic).
 */
size_t akf_sqrt_workspace_bytes(const akf_model* model, int32_t block);
akf_status akf_sqrt_filter_sample(const akf_model* model, const double* omega,
                                  const double* Omega, const double* xi, double* x_out,
                                  double* mf, double* Uf, double* ell, double* logZ,
                                  int32_t* status, void* ws, size_t ws_bytes, int32_t block,
                                  void* stream);

/*
 * Divide-and-conquer pathwise sampler (App. A, "Divide-and-conquer
 * strategies"): same inputs and law as akf_rts_sample, drawn top-down on the
 * bisection tree of [0, T] (T = N-1; [k, m] with m - k >= 2 splits at
 * l = (k + m) / 2) from the bridges p(x_l | x_k, x_m) (eq. recursive_params)
 * built bottom-up from the elements of eq. init-dnc and eq. EgL_comb.  Noise
 * map: x_T = mf_T + chol(Pf_T) xi_T, x_0 = E_{0:T} x_T + g_{0:T} +
 * chol(L_{0:T}) xi_0, x_l = G x_k + Gamma x_m + w + chol(V) xi_l, so for the
 * same xi the path differs from akf_rts_sample's (same distribution).
 * mf [N,dx], Pf [N,dx,dx], xi [N,dx], x [N,dx]; linear dynamics only.
 */
size_t akf_dnc_workspace_bytes(const akf_model* model);
akf_status akf_dnc_sample(const akf_model* model, const double* mf, const double* Pf,
                          const double* xi, double* x, int32_t* status, void* ws,
                          size_t ws_bytes, void* stream);

/*
 * RTS smoother (eq. init-dnc, eq. EgL_comb): from the filtering moments
 * mf [N,dx], Pf [N,dx,dx] of the model's dynamics, the smoothing moments
 * ms [N,dx], Ps [N,dx,dx] by a parallel suffix scan of (E, g, L) elements.
 */
size_t akf_smoother_workspace_bytes(const akf_model* model, int32_t block);
akf_status akf_smoother(const akf_model* model, const double* mf, const double* Pf, double* ms,
                        double* Ps, int32_t* status, void* ws, size_t ws_bytes, int32_t block,
                        void* stream);

/*
 * Linear-Gaussian state-space model with parameters theta = (F, log diag Q,
 * H, log diag R) (App. A, eq. lgssm-app with b = c = 0):
 *   x_0 ~ N(m0, P0), x_t = F x_{t-1} + N(0, diag exp(logq)),
 *   y_t = H x_t + N(0, diag exp(logr)).
 * m0 [dx], P0 [dx,dx], F [dx,dx], logq [dx], H [dy,dx], logr [dy], y [N,dy];
 * 1 <= dx, dy <= 32.
 */
typedef struct akf_lgssm {
  int32_t N, dx, dy;
  const double *m0, *P0;
  const double *F, *logq;
  const double *H, *logr;
  const double* y;
} akf_lgssm;

/*
 * log p(y_{0:T} | theta) by the parallel filter (predictive form of eq.
 * marginal-likelihood): ll [1] device double, ell [N] per-step terms (may be
 * NULL).  When a matrix that must be positive definite is not (status != 0),
 * ll is NaN.  The filtering moments stay in `ws` as the checkpoint of the
 * adjoint; akf_lgssm_loglik_grad must be called with the same model, block
 * and workspace, after this call and before any other use of the workspace.
 */
size_t akf_lgssm_workspace_bytes(const akf_lgssm* m, int32_t block);
akf_status akf_lgssm_loglik(const akf_lgssm* m, double* ll, double* ell, int32_t* status, void* ws,
                            size_t ws_bytes, int32_t block, void* stream);

/*
 * Reverse-mode adjoint of akf_lgssm_loglik: ll_bar [1] (device, NULL = 1)
 * times d log p / d theta, written to dF [dx,dx], dlogq [dx], dH [dy,dx],
 * dlogr [dy].  Two suffix scans over time (mean and covariance adjoints) from
 * the checkpointed filtering moments, then per-step gradient terms.  When the
 * forward pass or the adjoint met a matrix that is not positive definite
 * (status != 0) every gradient entry is NaN.
 */
akf_status akf_lgssm_loglik_grad(const akf_lgssm* m, const double* ll_bar, double* dF,
                                 double* dlogq, double* dH, double* dlogr, int32_t* status,
                                 void* ws, size_t ws_bytes, int32_t block, void* stream);

/*
 * Gibbs sampler over (theta, x) of the linear-Gaussian model above (the
 * parametric model of eq. parametric-ssm; parameters and path updated in
 * turn as in Sec. "Parameter estimation in a continuous-discrete diffusion
 * smoothing problem").  theta is one flat device array of
 * p = dx*dx + dx + dy*dx + dy doubles: F (row-major), logq, H (row-major),
 * logr.  The prior is N(0, prior_sd^2) on every coordinate.  The fields
 * F, logq, H and logr of `m` are ignored (theta replaces them); N, dx, dy, m0,
 * P0 and y are used.  1 <= dx, dy <= 32.
 *
 * One sweep, all on the device (no host synchronisation):
 *   1. MALA on log pi(theta) = log p(theta) + log p(y | theta):
 *      theta' = theta + (eps^2/2) grad(theta) + eps xi_theta, with
 *      log p(y | theta') and its gradient from the parallel filter and the
 *      adjoint; log alpha = log pi(theta') - log pi(theta)
 *      + log q(theta | theta') - log q(theta' | theta),
 *      q(a | b) = N(a; b + (eps^2/2) grad(b), eps^2 I); accept iff the
 *      proposal's filter succeeded, log alpha is finite and
 *      log u_theta < log alpha.  theta, logpost and grad are replaced on
 *      acceptance.
 *   2. x ~ p(x | theta, y) exactly (parallel filter + RTS sampler, normals
 *      xi_x [N,dx]), overwriting x: the theta move targets the theta-marginal,
 *      so x is re-drawn from its full conditional;
 *   3. n_path auxiliary Kalman MH steps (order 2; the emission is Gaussian,
 *      so every step accepts) on x at theta, with xi_path [n_path,2,N,dx] and
 *      u_path [n_path] as in akf_mh_run.
 * Arguments: theta [p], logpost [1], grad [p] (log posterior and its gradient
 * at theta, kept by the caller between sweeps), x [N,dx] (all in/out);
 * state: `akf_gibbs_state_bytes` bytes (256-aligned) holding the filtering
 * moments and dense Q, R of theta between sweeps; eps > 0; u_theta [1] in
 * (0,1).  Outputs (device, each may be NULL): accepted_theta [1],
 * log_alpha [1], path_log_ratio / path_accepted / path_status [n_path],
 * status [2]: [0] the proposal's filter/adjoint status (non-zero = the
 * proposal was rejected as undefined), [1] the refresh sampler's status.
 * akf_gibbs_init fills logpost, grad and the state for a starting theta
 * (status [1]; logpost NaN if its filter fails).  Workspace:
 * akf_gibbs_workspace_bytes (contents not kept between calls).
 */
size_t akf_gibbs_state_bytes(const akf_lgssm* m);
size_t akf_gibbs_workspace_bytes(const akf_lgssm* m, int32_t block);
akf_status akf_gibbs_init(const akf_lgssm* m, const double* theta, double prior_sd,
                          double* logpost, double* grad, void* state, size_t state_bytes,
                          int32_t* status, void* ws, size_t ws_bytes, int32_t block,
                          void* stream);
akf_status akf_gibbs_sweep(const akf_lgssm* m, double* theta, double* logpost, double* grad,
                           double* x, void* state, size_t state_bytes, double prior_sd, double eps,
                           const double* xi_theta, const double* u_theta, const double* xi_x,
                           double delta, int32_t n_path, const double* xi_path,
                           const double* u_path, int32_t* accepted_theta, double* log_alpha,
                           double* path_log_ratio, int32_t* path_accepted, int32_t* path_status,
                           int32_t* status, void* ws, size_t ws_bytes, int32_t block,
                           void* stream);

/*
 * Batched chains: many independent chains (each its own model, length N and
 * dimension dx) advanced together.  All chains are grouped by team size
 * (dx <= 16, <= 32, <= 64); every phase of a step is one persistent launch per
 * group that walks a table of (chain, block / tree node / time step) work
 * items, so the whole batch needs a few dozen launches per step instead of a
 * few dozen per chain.  One step is captured in a hipGraph and replayed; a
 * device step counter selects each step's normals and outputs.  Emissions:
 * Poisson log-link, Student-t and stochastic volatility.
 *
 * Per chain (device pointers): model, y [N,dy], x [N,dx] (updated in place),
 * xi [n_steps,2,N,dx], unif [n_steps], delta, order, and optional per-step
 * outputs [n_steps] (NULL = not written).
 */
typedef struct akf_chain {
  akf_model model;
  const double* y;
  double* x;
  const double* xi;
  const double* unif;
  double delta;
  int32_t order;
  double* log_ratio;
  int32_t* accepted;
  double* logZ_fwd;
  double* logZ_rev;
  int32_t* status;
} akf_chain;

typedef struct akf_batch_plan akf_batch_plan;

/*
 * Builds a plan (library-owned; the only object this library allocates):
 * validates the chains (host array, copied), allocates the device descriptors,
 * work tables and per-chain workspaces, and picks the scan block per group.
 * block = 0 autotunes: each candidate block size is timed on one step of the
 * real batch (on scratch copies of x; no state changes), and the choice is
 * appended to the text cache `tune_cache` (one JSON object per line; NULL =
 * no cache) and reused when the same group shape is seen again.
 */
akf_status akf_batch_plan_create(akf_batch_plan** plan, int32_t n_chains, const akf_chain* chains,
                                 int32_t n_steps, int32_t block, const char* tune_cache,
                                 void* stream);

/* Runs n_steps steps on every chain; use_graph = 1 captures one step in a
 * hipGraph on `stream` (which must not be the legacy default stream) at the
 * first call and replays it, use_graph = 0 launches eagerly. */
akf_status akf_batch_mh_run(akf_batch_plan* plan, int32_t use_graph, void* stream);

/* Plan diagnostics: number of groups and, per group (up to max_classes), its
 * team size D, scan block, chain count and, at D = 32, the sampler build's
 * one-wave teams per SIMD (2, or 1 with the whole register file; 0 at the
 * widths with a single layout); total device bytes.  Any output pointer
 * except n_classes may be NULL. */
akf_status akf_batch_plan_info(const akf_batch_plan* plan, int32_t max_classes,
                               int32_t* n_classes, int32_t* D, int32_t* block,
                               int32_t* n_chains_in_class, int32_t* sbuild_teams_per_simd,
                               size_t* device_bytes);
void akf_batch_plan_destroy(akf_batch_plan* plan);

/*
 * Kernel timing, for diagnostics and benchmarks.  While enabled for `family`
 * (0 filter fold, 1 filter scan levels (Hillis-Steele levels for one chain,
 * up-sweep levels for batched chains), 2 filter down-sweep, 3 filter final,
 * 4 sampler element build, 5 sampler fold, 6 sampler up-sweep, 7 sampler
 * down-sweep, 8 sampler final, 9 factorised scalar filter/sampler,
 * 10 emission and dynamics linearisation, 11 the whole divide-and-conquer
 * sampler, 12 and 13 the block folds of akf_mh_run_first_order's filtering
 * means and sampled path, 14 the adjoint's per-step gradient contractions,
 * 15 the adjoint's element build, 16 / 17 / 18 the batched filter folds of
 * team width 16 / 32 / 64, 19 / 20 / 21 the batched sampler element builds of
 * those widths, 22 the MH bookkeeping kernels (step initialisation and the
 * accept decision); every launch of akf_mh_step / akf_mh_run on a model with
 * linear dynamics belongs to one family), every
 * launch of that kernel on any stream is
 * bracketed by a pair of hipEvents recorded on the launch stream; at most
 * `capacity` launches are kept.  akf_timing_collect waits for the recorded
 * events and returns the number of launches and their summed duration in
 * milliseconds, then clears the record.  family < 0 disables timing.  The
 * events are created by akf_timing_enable (not under graph capture); launches
 * enqueued while their stream is being captured are not timed.
 */
akf_status akf_timing_enable(int32_t family, int32_t capacity);
akf_status akf_timing_collect(int32_t* n_launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* AKF_H */
