/*
 * akf_oracle.c -- sequential FP64 CPU oracle for the auxiliary Kalman MCMC step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  It shares no code, header, table or helper with
 * the HIP library (paper_2303_00301_amd/csrc); only tests/, the smoke check and
 * the CPU-baseline leg of bench.py may load it.
 *
 * Everything is double precision, row-major, one chain, textbook loops.
 * Paper: Corenflos & Sarkka, "Auxiliary MCMC samplers for parallelisable
 * inference in high-dimensional latent dynamical systems" (arXiv 2303.00301).
 *
 *   or_kf            Kalman filter with predictive-form marginal likelihood
 *                    (App. A.1, Alg. "Kalman filter"; eq. marginal-likelihood).
 *   or_rts_sample    Rauch-Tung-Striebel *sampler* with a fixed noise map
 *                    (App. A.1, Alg. "Rauch-Tung-Striebel sampler", eq. backward).
 *   or_dnc_sample    divide-and-conquer pathwise sampler on the bisection tree
 *                    (App. A, "Divide-and-conquer strategies").
 *   or_rts_smooth    RTS smoother marginals and the backward gains, used for the
 *                    Fisher-identity score and moment checks.
 *   or_emission      log h_t, its gradient v_t and Hessian Lambda_t for the
 *                    Gaussian / Poisson-log / Student-t / stochastic-volatility /
 *                    multivariate-t / Gaussian-at-sites families (Sec. 2.2, eq.
 *                    linearised-log-potential-second).
 *   or_dyn, or_dyn_linearise  Euler steps of the Lorenz-63 / Lorenz-96 SDEs and
 *                    their extended linearisation (Example "gslr-example").
 *   or_obs_linearise the observation model's Gaussian approximation
 *                    N(H z + c, R) around x_t by statistical linear regression
 *                    (eq. observation-approx, eq. coeffs; Taylor limit at a zero
 *                    reference variance).
 *   or_linearise     pseudo-observations (omega_t, Omega_t) of the auxiliary
 *                    LGSSM: first order (eq. gaussian-FK-proposal), second
 *                    order (eq. second-order), or the linearised observation
 *                    model (order 3: eq. two-lin-prop), with Sigma_t = I.
 *   or_mh_step       one step of the general auxiliary Kalman sampler
 *                    (Alg. "General Auxiliary Kalman sampler"), Hastings-within-
 *                    Gibbs on x | u.
 *   or_mh_step_factorised  the same step when the prior and Omega_t are
 *                    diagonal, as dx one-dimensional filters and samplers
 *                    (Sec. "Spatio-temporal model").
 *   or_fisher_score  gradient of log p(y | theta) by Fisher's identity for an
 *                    LGSSM with theta = (F, log diag Q, H, log diag R).
 *
 * Parity status: every function here is pinned by tests/test_oracle_*.py against
 * dense joint-Gaussian brute force, closed forms, quadrature and finite
 * differences (see the test files for which pin covers which function).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define LOG2PI 1.8378770664093454835606594728112

/* ------------------------------------------------------------------ */
/* small dense helpers (row-major)                                      */
/* ------------------------------------------------------------------ */

/* C[m,n] = A[m,k] * B[k,n] */
static void mm(int m, int n, int k, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[i * k + l] * B[l * n + j];
      C[i * n + j] = s;
    }
}

/* C[m,n] = A[m,k] * B[n,k]^T */
static void mm_nt(int m, int n, int k, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[i * k + l] * B[j * k + l];
      C[i * n + j] = s;
    }
}

/* C[m,n] = A[k,m]^T * B[k,n] */
static void mm_tn(int m, int n, int k, const double* A, const double* B, double* C) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += A[l * m + i] * B[l * n + j];
      C[i * n + j] = s;
    }
}

static void mv(int m, int n, const double* A, const double* x, double* y) {
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += A[i * n + j] * x[j];
    y[i] = s;
  }
}

static void symmetrise(int n, double* A) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      double s = 0.5 * (A[i * n + j] + A[j * n + i]);
      A[i * n + j] = s;
      A[j * n + i] = s;
    }
}

/* Lower Cholesky factor L (positive diagonal) of a symmetric matrix A.
 * Returns 0 on success, 1 when A is not numerically positive definite. */
static int chol(int n, const double* A, double* L) {
  memset(L, 0, sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0) || !isfinite(s)) return 1;
    double d = sqrt(s);
    L[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / d;
    }
  }
  return 0;
}

/* Solve L z = b in place (forward substitution). */
static void fwd_sub(int n, const double* L, double* b) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
    b[i] = s / L[i * n + i];
  }
}

/* Solve L^T z = b in place (backward substitution). */
static void bwd_sub(int n, const double* L, double* b) {
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
    b[i] = s / L[i * n + i];
  }
}

/* X = A^{-1} B for SPD A given its Cholesky factor L; B is [n, nrhs], in place. */
static void chol_solve(int n, int nrhs, const double* L, double* B, double* col) {
  for (int j = 0; j < nrhs; ++j) {
    for (int i = 0; i < n; ++i) col[i] = B[i * nrhs + j];
    fwd_sub(n, L, col);
    bwd_sub(n, L, col);
    for (int i = 0; i < n; ++i) B[i * nrhs + j] = col[i];
  }
}

static double chol_logdet(int n, const double* L) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += log(L[i * n + i]);
  return 2.0 * s;
}

/* log N(x; mu, S) with S given by its Cholesky factor L. */
static double gauss_logpdf_chol(int n, const double* x, const double* mu, const double* L, double* tmp) {
  for (int i = 0; i < n; ++i) tmp[i] = x[i] - mu[i];
  fwd_sub(n, L, tmp);
  double q = 0.0;
  for (int i = 0; i < n; ++i) q += tmp[i] * tmp[i];
  return -0.5 * (n * LOG2PI + chol_logdet(n, L) + q);
}

/* ------------------------------------------------------------------ */
/* Kalman filter                                                        */
/* ------------------------------------------------------------------ */

/*
 * Kalman filter for  x_0 ~ N(m0,P0),  x_t = F_t x_{t-1} + b_t + N(0,Q),
 * y_t = H_t x_t + N(0, R_t),  t = 0..N-1.
 * F_t = F + t*F_stride, b_t = b + t*b_stride, H_t = H + t*H_stride,
 * R_t = R + t*R_stride (stride 0: time-invariant; F_0, b_0 are not used).
 * The likelihood uses the predictive moments, log p(y_t | y_{0:t-1}) =
 * log N(y_t; H m^p_t, H P^p_t H^T + R_t) (the printed filtered-moment form is a
 * typo; the algorithm's update line uses the predictive one).
 * Outputs mf/Pf/mp/Pp may be NULL.  ell[t] receives the per-step term.
 * Returns 0, or 1 + t when S_t was not positive definite at step t.
 */
int or_kf(int N, int dx, int dy, const double* m0, const double* P0, const double* F,
          long F_stride, const double* b, long b_stride, const double* Q, const double* H,
          long H_stride, const double* R, long R_stride, const double* y, double* mf, double* Pf,
          double* mp, double* Pp, double* ell) {
  const int n = dx, p = dy;
  double* m_p = malloc(sizeof(double) * n);
  double* P_p = malloc(sizeof(double) * n * n);
  double* m_f = malloc(sizeof(double) * n);
  double* P_f = malloc(sizeof(double) * n * n);
  double* T = malloc(sizeof(double) * n * n);
  double* HP = malloc(sizeof(double) * p * n);
  double* S = malloc(sizeof(double) * p * p);
  double* L = malloc(sizeof(double) * p * p);
  double* v = malloc(sizeof(double) * p);
  double* Kt = malloc(sizeof(double) * p * n); /* K^T = S^{-1} H P */
  double* col = malloc(sizeof(double) * (p > n ? p : n));
  double* tmp = malloc(sizeof(double) * (p > n ? p : n));
  int rc = 0;
  for (int t = 0; t < N && rc == 0; ++t) {
    const double* Ht = H + (long)t * H_stride;
    const double* Rt = R + (long)t * R_stride;
    if (t == 0) {
      memcpy(m_p, m0, sizeof(double) * n);
      memcpy(P_p, P0, sizeof(double) * n * n);
    } else {
      const double* Ft = F + (long)t * F_stride;
      mv(n, n, Ft, m_f, m_p);
      if (b)
        for (int i = 0; i < n; ++i) m_p[i] += b[(long)t * b_stride + i];
      mm(n, n, n, Ft, P_f, T);
      mm_nt(n, n, n, T, Ft, P_p);
      for (int i = 0; i < n * n; ++i) P_p[i] += Q[i];
      symmetrise(n, P_p);
    }
    if (mp) memcpy(mp + (long)t * n, m_p, sizeof(double) * n);
    if (Pp) memcpy(Pp + (long)t * n * n, P_p, sizeof(double) * n * n);
    /* innovation */
    mm(p, n, n, Ht, P_p, HP);
    mm_nt(p, p, n, HP, Ht, S);
    for (int i = 0; i < p * p; ++i) S[i] += Rt[i];
    symmetrise(p, S);
    if (chol(p, S, L)) {
      rc = 1 + t;
      break;
    }
    mv(p, n, Ht, m_p, v);
    for (int i = 0; i < p; ++i) v[i] = y[(long)t * p + i] - v[i];
    for (int i = 0; i < p; ++i) tmp[i] = v[i];
    fwd_sub(p, L, tmp);
    double q = 0.0;
    for (int i = 0; i < p; ++i) q += tmp[i] * tmp[i];
    ell[t] = -0.5 * (p * LOG2PI + chol_logdet(p, L) + q);
    /* gain: K^T = S^{-1} (H P) */
    memcpy(Kt, HP, sizeof(double) * p * n);
    chol_solve(p, n, L, Kt, col);
    /* m_f = m_p + K v */
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += Kt[k * n + i] * v[k];
      m_f[i] = m_p[i] + s;
    }
    /* P_f = P_p - K H P_p = P_p - (HP)^T S^{-1} (HP) */
    mm_tn(n, n, p, HP, Kt, T);
    for (int i = 0; i < n * n; ++i) P_f[i] = P_p[i] - T[i];
    symmetrise(n, P_f);
    if (mf) memcpy(mf + (long)t * n, m_f, sizeof(double) * n);
    if (Pf) memcpy(Pf + (long)t * n * n, P_f, sizeof(double) * n * n);
  }
  free(m_p); free(P_p); free(m_f); free(P_f); free(T); free(HP); free(S); free(L);
  free(v); free(Kt); free(col); free(tmp);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Backward gains shared by the sampler and smoother                    */
/* ------------------------------------------------------------------ */

/*
 * G_t = P^f_t F^T (P^p_{t+1})^{-1} and Sigma_t = P^f_t - G_t P^p_{t+1} G_t^T,
 * the moments of p(x_t | x_{t+1}, y_{0:t}) (eq. backward).  Returns 0 or 1.
 */
static int backward_gain(int n, const double* F, const double* Pf, const double* Pp1, double* G,
                         double* Sig, double* work) {
  double* Lp = work;             /* n*n */
  double* FP = work + n * n;     /* n*n : F P^f  (so G^T = Pp1^{-1} F P^f) */
  double* col = work + 2 * n * n;
  double* T = work + 2 * n * n + n;
  if (chol(n, Pp1, Lp)) return 1;
  mm(n, n, n, F, Pf, FP);
  memcpy(T, FP, sizeof(double) * n * n);
  chol_solve(n, n, Lp, T, col); /* T = Pp1^{-1} F Pf = G^T */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) G[i * n + j] = T[j * n + i];
  /* Sigma = Pf - G Pp1 G^T = Pf - G (F Pf) */
  mm(n, n, n, G, FP, T);
  for (int i = 0; i < n * n; ++i) Sig[i] = Pf[i] - T[i];
  symmetrise(n, Sig);
  return 0;
}

/*
 * RTS sampler with a fixed noise map (eq. backward): x_{N-1} = m^f + chol(P^f) xi,
 * x_t = m^f_t + G_t (x_{t+1} - m^p_{t+1}) + chol(Sigma_t) xi_t, chol = lower
 * Cholesky factor with positive diagonal; G_t uses F_{t+1} = F + (t+1)*F_stride,
 * the transition into step t+1.  Returns 0, or 1 + t on a non-PD covariance at
 * step t.
 */
int or_rts_sample(int N, int dx, const double* F, long F_stride, const double* mf,
                  const double* Pf, const double* mp, const double* Pp, const double* xi,
                  double* x) {
  const int n = dx;
  double* G = malloc(sizeof(double) * n * n);
  double* Sig = malloc(sizeof(double) * n * n);
  double* L = malloc(sizeof(double) * n * n);
  double* d = malloc(sizeof(double) * n);
  double* work = malloc(sizeof(double) * (3 * n * n + n));
  int rc = 0;
  const long t1 = N - 1;
  if (chol(n, Pf + t1 * n * n, L)) rc = N;
  else {
    mv(n, n, L, xi + t1 * n, d);
    for (int i = 0; i < n; ++i) x[t1 * n + i] = mf[t1 * n + i] + d[i];
  }
  for (long t = N - 2; t >= 0 && rc == 0; --t) {
    if (backward_gain(n, F + (t + 1) * F_stride, Pf + t * n * n, Pp + (t + 1) * n * n, G, Sig,
                      work) ||
        chol(n, Sig, L)) {
      rc = 1 + (int)t;
      break;
    }
    for (int i = 0; i < n; ++i) d[i] = x[(t + 1) * n + i] - mp[(t + 1) * n + i];
    double* e = work;
    mv(n, n, G, d, e);
    double* z = work + n;
    mv(n, n, L, xi + t * n, z);
    for (int i = 0; i < n; ++i) x[t * n + i] = mf[t * n + i] + e[i] + z[i];
  }
  free(G); free(Sig); free(L); free(d); free(work);
  return rc;
}

/*
 * Divide-and-conquer pathwise sampler (App. A, "Divide-and-conquer
 * strategies"): the same law as or_rts_sample, drawn top-down on the bisection
 * tree of [0, T] (T = N-1; an interval [k, m] with m - k >= 2 splits at
 * l = (k + m) / 2).  Elements (E, g, L)_{k:m} of p(x_k | x_m) start from
 * eq. init-dnc on [t, t+1] (F_{t+1}, b_{t+1} the transition into t+1) and
 * compose by eq. EgL_comb; the bridge p(x_l | x_k, x_m) has the parameters of
 * eq. recursive_params.  Noise map: x_T = m^f_T + chol(P^f_T) xi_T,
 * x_0 = E_{0:T} x_T + g_{0:T} + chol(L_{0:T}) xi_0, and each midpoint
 * x_l = G x_k + Gamma x_m + w + chol(V) xi_l (chol = lower factor, positive
 * diagonal).  F [dx,dx] with F_stride = 0, or per step; b NULL, [dx] with
 * b_stride = 0, or per step.  Returns 0, or 1 on a non-PD matrix.
 */
typedef struct {
  int n;
  const double *F, *b, *Q, *mf, *Pf;
  long F_stride, b_stride;
  const double* xi;
  double* x;
} dnc_ctx;

/* (E, g, L) of [t, t+1] (eq. init-dnc) */
static int dnc_leaf(const dnc_ctx* c, int t, double* E, double* g, double* L) {
  const int n = c->n;
  const double* F = c->F + (long)(t + 1) * c->F_stride;
  const double* Pf = c->Pf + (long)t * n * n;
  double* Pp = malloc(sizeof(double) * n * n);
  double* FP = malloc(sizeof(double) * n * n);
  double* Lp = malloc(sizeof(double) * n * n);
  double* T = malloc(sizeof(double) * n * n);
  double* col = malloc(sizeof(double) * n);
  double* mp = malloc(sizeof(double) * n);
  int rc = 0;
  mm(n, n, n, F, Pf, FP);           /* F P^f */
  mm_nt(n, n, n, FP, F, Pp);        /* F P^f F' */
  for (int i = 0; i < n * n; ++i) Pp[i] += c->Q[i];
  symmetrise(n, Pp);
  if (chol(n, Pp, Lp)) rc = 1;
  else {
    memcpy(T, FP, sizeof(double) * n * n);
    chol_solve(n, n, Lp, T, col);   /* T = Pp^{-1} F P^f = E' */
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) E[i * n + j] = T[j * n + i];
    mv(n, n, F, c->mf + (long)t * n, mp);
    if (c->b)
      for (int i = 0; i < n; ++i) mp[i] += c->b[(long)(t + 1) * c->b_stride + i];
    mv(n, n, E, mp, col);
    for (int i = 0; i < n; ++i) g[i] = c->mf[(long)t * n + i] - col[i];
    mm(n, n, n, E, FP, T);          /* E F P^f */
    for (int i = 0; i < n * n; ++i) L[i] = Pf[i] - T[i];
    symmetrise(n, L);
  }
  free(Pp); free(FP); free(Lp); free(T); free(col); free(mp);
  return rc;
}

/*
 * (E, g, L)_{k:m} of the interval; for m - k >= 2 also samples the subtree
 * below it once x_k and x_m are known (bridges are formed on the way down,
 * samples drawn after both endpoints are fixed by the caller).  Here: builds
 * the element only; dnc_down draws.
 */
static int dnc_elem(const dnc_ctx* c, int k, int m, double* E, double* g, double* L) {
  const int n = c->n;
  if (m - k == 1) return dnc_leaf(c, k, E, g, L);
  const int l = (k + m) / 2;
  double* E1 = malloc(sizeof(double) * n * n);
  double* g1 = malloc(sizeof(double) * n);
  double* L1 = malloc(sizeof(double) * n * n);
  double* E2 = malloc(sizeof(double) * n * n);
  double* g2 = malloc(sizeof(double) * n);
  double* L2 = malloc(sizeof(double) * n * n);
  double* T = malloc(sizeof(double) * n * n);
  int rc = dnc_elem(c, k, l, E1, g1, L1) || dnc_elem(c, l, m, E2, g2, L2);
  if (!rc) {
    /* eq. EgL_comb with [k,l] on the left and [l,m] on the right */
    mm(n, n, n, E1, E2, E);
    mv(n, n, E1, g2, g);
    for (int i = 0; i < n; ++i) g[i] += g1[i];
    mm(n, n, n, E1, L2, T);
    mm_nt(n, n, n, T, E1, L);
    for (int i = 0; i < n * n; ++i) L[i] += L1[i];
    symmetrise(n, L);
  }
  free(E1); free(g1); free(L1); free(E2); free(g2); free(L2); free(T);
  return rc;
}

/* draws x_l for the midpoint of [k, m] from p(x_l | x_k, x_m), then recurses */
static int dnc_down(const dnc_ctx* c, int k, int m) {
  const int n = c->n;
  if (m - k < 2) return 0;
  const int l = (k + m) / 2;
  double* E1 = malloc(sizeof(double) * n * n);
  double* g1 = malloc(sizeof(double) * n);
  double* L1 = malloc(sizeof(double) * n * n);
  double* E2 = malloc(sizeof(double) * n * n);
  double* g2 = malloc(sizeof(double) * n);
  double* L2 = malloc(sizeof(double) * n * n);
  double* E = malloc(sizeof(double) * n * n);
  double* g = malloc(sizeof(double) * n);
  double* L = malloc(sizeof(double) * n * n);
  double* G = malloc(sizeof(double) * n * n);
  double* T = malloc(sizeof(double) * n * n);
  double* V = malloc(sizeof(double) * n * n);
  double* Lc = malloc(sizeof(double) * n * n);
  double* col = malloc(sizeof(double) * n);
  double* v = malloc(sizeof(double) * n);
  int rc = dnc_elem(c, k, l, E1, g1, L1) || dnc_elem(c, l, m, E2, g2, L2);
  if (!rc) {
    mm(n, n, n, E1, E2, E);
    mv(n, n, E1, g2, g);
    for (int i = 0; i < n; ++i) g[i] += g1[i];
    mm(n, n, n, E1, L2, T);
    mm_nt(n, n, n, T, E1, L);
    for (int i = 0; i < n * n; ++i) L[i] += L1[i];
    symmetrise(n, L);
    /* eq. recursive_params: G = L2 E1' L^{-1} (G' = L^{-1} E1 L2) */
    if (chol(n, L, Lc)) rc = 1;
  }
  if (!rc) {
    mm(n, n, n, E1, L2, T);       /* E1 L2 */
    chol_solve(n, n, Lc, T, col); /* T = L^{-1} E1 L2 = G' */
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) G[i * n + j] = T[j * n + i];
    /* mean: G x_k + (E2 - G E) x_m + (g2 - G g) */
    const double* xk = c->x + (long)k * n;
    const double* xm = c->x + (long)m * n;
    double* xl = c->x + (long)l * n;
    for (int i = 0; i < n; ++i) {
      double s = g2[i];
      for (int j = 0; j < n; ++j) s += E2[i * n + j] * xm[j];
      v[i] = s;
    }
    for (int i = 0; i < n; ++i) col[i] = xk[i] - g[i];
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += E[i * n + j] * xm[j];
      col[i] -= s;                 /* x_k - E x_m - g */
    }
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += G[i * n + j] * col[j];
      v[i] += s;
    }
    /* V = L2 - G L G' = L2 - G E1 L2 */
    mm(n, n, n, E1, L2, T);
    double* GT = malloc(sizeof(double) * n * n);
    mm(n, n, n, G, T, GT);
    for (int i = 0; i < n * n; ++i) V[i] = L2[i] - GT[i];
    free(GT);
    symmetrise(n, V);
    if (chol(n, V, Lc)) rc = 1;
    else {
      mv(n, n, Lc, c->xi + (long)l * n, col);
      for (int i = 0; i < n; ++i) xl[i] = v[i] + col[i];
    }
  }
  free(E1); free(g1); free(L1); free(E2); free(g2); free(L2); free(E); free(g); free(L); free(G);
  free(T); free(V); free(Lc); free(col); free(v);
  if (rc) return rc;
  return dnc_down(c, k, l) || dnc_down(c, l, m);
}

int or_dnc_sample(int N, int dx, const double* F, long F_stride, const double* b, long b_stride,
                  const double* Q, const double* mf, const double* Pf, const double* xi,
                  double* x) {
  const int n = dx, T = N - 1;
  dnc_ctx c = {n, F, b, Q, mf, Pf, F_stride, b_stride, xi, x};
  double* L = malloc(sizeof(double) * n * n);
  double* E = malloc(sizeof(double) * n * n);
  double* g = malloc(sizeof(double) * n);
  double* Lk = malloc(sizeof(double) * n * n);
  double* d = malloc(sizeof(double) * n);
  int rc = 0;
  if (chol(n, Pf + (long)T * n * n, L)) rc = 1;
  else {
    mv(n, n, L, xi + (long)T * n, d);
    for (int i = 0; i < n; ++i) x[(long)T * n + i] = mf[(long)T * n + i] + d[i];
  }
  if (!rc && T >= 1) {
    rc = dnc_elem(&c, 0, T, E, g, Lk);
    if (!rc && chol(n, Lk, L)) rc = 1;
    if (!rc) {
      mv(n, n, E, x + (long)T * n, d);
      for (int i = 0; i < n; ++i) x[i] = d[i] + g[i];
      mv(n, n, L, xi, d);
      for (int i = 0; i < n; ++i) x[i] += d[i];
      rc = dnc_down(&c, 0, T);
    }
  }
  free(L); free(E); free(g); free(Lk); free(d);
  return rc;
}

/*
 * RTS smoother: smoothed means/covariances and the gains G_t (t < N-1;
 * G_{N-1} is set to zero).  Cov(x_{t+1}, x_t | y) = P^s_{t+1} G_t^T.
 */
int or_rts_smooth(int N, int dx, const double* F, long F_stride, const double* mf,
                  const double* Pf, const double* mp, const double* Pp, double* ms, double* Ps,
                  double* Gout) {
  const int n = dx;
  double* G = malloc(sizeof(double) * n * n);
  double* Sig = malloc(sizeof(double) * n * n);
  double* D = malloc(sizeof(double) * n * n);
  double* T = malloc(sizeof(double) * n * n);
  double* d = malloc(sizeof(double) * n);
  double* work = malloc(sizeof(double) * (3 * n * n + n));
  int rc = 0;
  const long t1 = N - 1;
  memcpy(ms + t1 * n, mf + t1 * n, sizeof(double) * n);
  memcpy(Ps + t1 * n * n, Pf + t1 * n * n, sizeof(double) * n * n);
  if (Gout) memset(Gout + t1 * n * n, 0, sizeof(double) * n * n);
  for (long t = N - 2; t >= 0; --t) {
    if (backward_gain(n, F + (t + 1) * F_stride, Pf + t * n * n, Pp + (t + 1) * n * n, G, Sig,
                      work)) {
      rc = 1 + (int)t;
      break;
    }
    for (int i = 0; i < n; ++i) d[i] = ms[(t + 1) * n + i] - mp[(t + 1) * n + i];
    mv(n, n, G, d, ms + t * n);
    for (int i = 0; i < n; ++i) ms[t * n + i] += mf[t * n + i];
    /* Ps_t = Sigma_t + G Ps_{t+1} G^T */
    mm(n, n, n, G, Ps + (t + 1) * n * n, T);
    mm_nt(n, n, n, T, G, D);
    for (int i = 0; i < n * n; ++i) Ps[t * n * n + i] = Sig[i] + D[i];
    symmetrise(n, Ps + t * n * n);
    if (Gout) memcpy(Gout + t * n * n, G, sizeof(double) * n * n);
  }
  free(G); free(Sig); free(D); free(T); free(d); free(work);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Emission families                                                    */
/* ------------------------------------------------------------------ */

enum { OR_EMIT_GAUSSIAN = 0, OR_EMIT_POISSON_LOG = 1, OR_EMIT_STUDENT_T = 2, OR_EMIT_STOCH_VOL = 3,
       OR_EMIT_MVT = 4, OR_EMIT_GAUSS_SITE = 5, OR_EMIT_GAUSS_QUAD = 6 };
enum { OR_DYN_LINEAR = 0, OR_DYN_LORENZ63 = 1, OR_DYN_LORENZ96 = 2 };

typedef struct {
  int N, dx, dy;
  const double *m0, *P0, *F, *b, *Q;
  int emit;
  const double *H, *R;  /* Gaussian: [dy,dx], [dy,dy]; multivariate t: R = precision [dy,dy] */
  const int* site;      /* non-Gaussian families: y_k observes x[site[k]] */
  double nu, scale;     /* Student-t (nu, scale); multivariate t (nu); Gaussian at sites (scale) */
  int dyn;              /* OR_DYN_*: linear (F, b) or x_t = f(x_{t-1}) + N(0, Q) */
  double dyn_par[4];    /* Lorenz-63: theta1, theta2, theta3, dt; Lorenz-96: forcing, dt */
  double obs_beta;      /* quadratic observation mean x + beta x^2 (Gaussian, quadratic mean) */
  double slr_var;       /* reference variance gamma^2 of the observation-model linearisation */
} or_model;

/*
 * log h(y_t | x_t) up to an additive constant that does not depend on x,
 * together with v = grad_x log h and Lambda = Hessian (dense [dx,dx]).
 * Constants dropped: Gaussian -(dy log 2pi + logdet R)/2, Poisson -log y!,
 * Student-t log Gamma terms and -log s, multivariate t log Gamma terms,
 * -(dy/2) log(nu pi) and +(1/2) logdet R, Gaussian at sites -(log 2pi)/2 - log s
 * per site.  They cancel in the MH ratio.  In the site-wise families
 * (Poisson, Student-t, stochastic volatility, Gaussian at sites) an entry
 * y_{t,k} that is NaN is not observed and contributes nothing.
 * v and Lam may be NULL.  Returns log h (may be +-inf / nan on overflow).
 */
double or_emission(const or_model* M, const double* yt, const double* xt, double* v, double* Lam) {
  const int n = M->dx, p = M->dy;
  double lh = 0.0;
  if (v) memset(v, 0, sizeof(double) * n);
  if (Lam) memset(Lam, 0, sizeof(double) * n * n);
  if (M->emit == OR_EMIT_GAUSSIAN) {
    double* r = malloc(sizeof(double) * p);
    double* w = malloc(sizeof(double) * p);
    double* L = malloc(sizeof(double) * p * p);
    double* RiH = malloc(sizeof(double) * p * n);
    double* col = malloc(sizeof(double) * p);
    chol(p, M->R, L);
    mv(p, n, M->H, xt, r);
    for (int k = 0; k < p; ++k) r[k] = yt[k] - r[k];
    memcpy(w, r, sizeof(double) * p);
    fwd_sub(p, L, w);
    double q = 0.0;
    for (int k = 0; k < p; ++k) q += w[k] * w[k];
    lh = -0.5 * q;
    /* w = R^{-1} r */
    memcpy(w, r, sizeof(double) * p);
    fwd_sub(p, L, w);
    bwd_sub(p, L, w);
    if (v)
      for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < p; ++k) s += M->H[k * n + i] * w[k];
        v[i] = s;
      }
    if (Lam) {
      memcpy(RiH, M->H, sizeof(double) * p * n);
      chol_solve(p, n, L, RiH, col);
      mm_tn(n, n, p, M->H, RiH, Lam);
      for (int i = 0; i < n * n; ++i) Lam[i] = -Lam[i];
      symmetrise(n, Lam);
    }
    free(r); free(w); free(L); free(RiH); free(col);
  } else if (M->emit == OR_EMIT_POISSON_LOG) {
    for (int k = 0; k < p; ++k) {
      if (isnan(yt[k])) continue;
      int i = M->site[k];
      double e = exp(xt[i]);
      lh += yt[k] * xt[i] - e;
      if (v) v[i] += yt[k] - e;
      if (Lam) Lam[i * n + i] -= e;
    }
  } else if (M->emit == OR_EMIT_MVT) {
    /* y = x[site] + V, V multivariate t (nu degrees of freedom) with precision
       matrix R [p, p] (Sec. "Spatio-temporal model"):
       log h = -(nu + p)/2 log(1 + r'R r / nu), r = y - x[site] (constants dropped);
       v_i = (nu + p)/(nu + q) s_i,  s_i = sum_{k: site[k] = i} (R r)_k,
       Lambda_ij = (nu + p) [2 s_i s_j / (nu + q)^2 - Rt_ij / (nu + q)],
       Rt_ij = sum_{k: site[k] = i, l: site[l] = j} R_kl. */
    double* r = malloc(sizeof(double) * p);
    double* Rr = malloc(sizeof(double) * p);
    double* sv = calloc(n, sizeof(double));
    for (int k = 0; k < p; ++k) r[k] = yt[k] - xt[M->site[k]];
    mv(p, p, M->R, r, Rr);
    double q = 0.0;
    for (int k = 0; k < p; ++k) q += r[k] * Rr[k];
    const double a = M->nu + p;
    lh = -0.5 * a * log1p(q / M->nu);
    for (int k = 0; k < p; ++k) sv[M->site[k]] += Rr[k];
    if (v)
      for (int i = 0; i < n; ++i) v[i] = a / (M->nu + q) * sv[i];
    if (Lam) {
      const double c1 = a / (M->nu + q), c2 = 2.0 * a / ((M->nu + q) * (M->nu + q));
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Lam[i * n + j] = c2 * sv[i] * sv[j];
      for (int k = 0; k < p; ++k)
        for (int l = 0; l < p; ++l) Lam[M->site[k] * n + M->site[l]] -= c1 * M->R[k * p + l];
      symmetrise(n, Lam);
    }
    free(r); free(Rr); free(sv);
  } else if (M->emit == OR_EMIT_STOCH_VOL) {
    /* y_k ~ N(0, exp(x_i)) (Sec. "Multivariate stochastic volatility model"):
       log h = -x_i/2 - y_k^2 exp(-x_i)/2 (the -log(2 pi)/2 constant dropped) */
    for (int k = 0; k < p; ++k) {
      if (isnan(yt[k])) continue;
      int i = M->site[k];
      double q = yt[k] * yt[k] * exp(-xt[i]);
      lh += -0.5 * xt[i] - 0.5 * q;
      if (v) v[i] += -0.5 + 0.5 * q;
      if (Lam) Lam[i * n + i] -= 0.5 * q;
    }
  } else if (M->emit == OR_EMIT_GAUSS_QUAD) {
    /* y_k = x_i + beta x_i^2 + N(0, s^2): log h = -(y_k - m)^2 / (2 s^2),
       m = x_i + beta x_i^2, dm/dx = 1 + 2 beta x_i, d2m/dx2 = 2 beta */
    const double s2 = M->scale * M->scale, be = M->obs_beta;
    for (int k = 0; k < p; ++k) {
      if (isnan(yt[k])) continue;
      int i = M->site[k];
      double m = xt[i] + be * xt[i] * xt[i], g = 1.0 + 2.0 * be * xt[i], r = yt[k] - m;
      lh += -0.5 * r * r / s2;
      if (v) v[i] += g * r / s2;
      if (Lam) Lam[i * n + i] += (2.0 * be * r - g * g) / s2;
    }
  } else if (M->emit == OR_EMIT_GAUSS_SITE) {
    /* y_k = x_i + N(0, s^2): log h = -(y_k - x_i)^2 / (2 s^2) */
    const double s2 = M->scale * M->scale;
    for (int k = 0; k < p; ++k) {
      if (isnan(yt[k])) continue;
      int i = M->site[k];
      double r = yt[k] - xt[i];
      lh += -0.5 * r * r / s2;
      if (v) v[i] += r / s2;
      if (Lam) Lam[i * n + i] -= 1.0 / s2;
    }
  } else {
    const double a = M->nu * M->scale * M->scale;
    for (int k = 0; k < p; ++k) {
      if (isnan(yt[k])) continue;
      int i = M->site[k];
      double r = yt[k] - xt[i];
      double den = a + r * r;
      lh += -0.5 * (M->nu + 1.0) * log1p(r * r / a);
      if (v) v[i] += (M->nu + 1.0) * r / den;
      if (Lam) Lam[i * n + i] += (M->nu + 1.0) * (r * r - a) / (den * den);
    }
  }
  return lh;
}

/* ------------------------------------------------------------------ */
/* Nonlinear dynamics x_t = f(x_{t-1}) + N(0, Q)                        */
/* ------------------------------------------------------------------ */

/*
 * One Euler-Maruyama step of an SDE dx = beta(x) dt + noise:
 * f(x) = x + dt beta(x), J = df/dx = I + dt dbeta/dx (J may be NULL).
 *   Lorenz-63 (Sec. "Parameter estimation in a continuous-discrete diffusion
 *   smoothing problem"), d = 3: beta = (t1 (x1 - x0), t2 x0 - x1 - x0 x2,
 *   x0 x1 - t3 x2);
 *   Lorenz-96, d >= 4 (cyclic indices): beta_i = (x_{i+1} - x_{i-2}) x_{i-1} - x_i + forcing.
 */
void or_dyn(const or_model* M, const double* x, double* f, double* J) {
  const int n = M->dx;
  double* beta = malloc(sizeof(double) * n);
  double* Jb = calloc((size_t)n * n, sizeof(double));
  double dt;
  if (M->dyn == OR_DYN_LORENZ63) {
    const double t1 = M->dyn_par[0], t2 = M->dyn_par[1], t3 = M->dyn_par[2];
    dt = M->dyn_par[3];
    beta[0] = t1 * (x[1] - x[0]);
    beta[1] = t2 * x[0] - x[1] - x[0] * x[2];
    beta[2] = x[0] * x[1] - t3 * x[2];
    Jb[0] = -t1; Jb[1] = t1; Jb[2] = 0.0;
    Jb[3] = t2 - x[2]; Jb[4] = -1.0; Jb[5] = -x[0];
    Jb[6] = x[1]; Jb[7] = x[0]; Jb[8] = -t3;
  } else {
    const double forcing = M->dyn_par[0];
    dt = M->dyn_par[1];
    for (int i = 0; i < n; ++i) {
      const int ip = (i + 1) % n, im = (i + n - 1) % n, im2 = (i + n - 2) % n;
      beta[i] = (x[ip] - x[im2]) * x[im] - x[i] + forcing;
      Jb[i * n + ip] += x[im];
      Jb[i * n + im2] -= x[im];
      Jb[i * n + im] += x[ip] - x[im2];
      Jb[i * n + i] -= 1.0;
    }
  }
  for (int i = 0; i < n; ++i) f[i] = x[i] + dt * beta[i];
  if (J)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) J[i * n + j] = (i == j ? 1.0 : 0.0) + dt * Jb[i * n + j];
  free(beta); free(Jb);
}

/*
 * Extended linearisation of the dynamics around the path a (Example
 * "gslr-example"): for t >= 1, F_t = J(a_{t-1}) and b_t = f(a_{t-1}) - F_t a_{t-1},
 * so that N(z_t; F_t z_{t-1} + b_t, Q) approximates p_t(z_t | z_{t-1}).
 * F [N,dx,dx], b [N,dx]; entries t = 0 are set to zero (unused).
 */
void or_dyn_linearise(const or_model* M, const double* a, double* F, double* b) {
  const int n = M->dx;
  double* f = malloc(sizeof(double) * n);
  memset(F, 0, sizeof(double) * n * n);
  memset(b, 0, sizeof(double) * n);
  for (long t = 1; t < M->N; ++t) {
    double* Ft = F + t * n * n;
    or_dyn(M, a + (t - 1) * n, f, Ft);
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += Ft[i * n + j] * a[(t - 1) * n + j];
      b[t * n + i] = f[i] - s;
    }
  }
  free(f);
}

/*
 * sum_{t >= 1} [log N(z_t; f(z_{t-1}), Q) - log N(z_t; F_t z_{t-1} + b_t, Q)]:
 * the true transition density of the path z against the linearised one in the
 * proposal; the terms of p(z, u) / q(z | ...) that do not cancel once the
 * dynamics are linearised.
 */
static double dyn_mismatch(const or_model* M, const double* z, const double* F, const double* b) {
  const int n = M->dx;
  double* L = malloc(sizeof(double) * n * n);
  double* f = malloc(sizeof(double) * n);
  double* g = malloc(sizeof(double) * n);
  double* tmp = malloc(sizeof(double) * n);
  double s = 0.0;
  if (chol(n, M->Q, L)) s = NAN;
  for (long t = 1; t < M->N && !isnan(s); ++t) {
    or_dyn(M, z + (t - 1) * n, f, NULL);
    mv(n, n, F + t * n * n, z + (t - 1) * n, g);
    for (int i = 0; i < n; ++i) g[i] += b[t * n + i];
    s += gauss_logpdf_chol(n, z + t * n, f, L, tmp) - gauss_logpdf_chol(n, z + t * n, g, L, tmp);
  }
  free(L); free(f); free(g); free(tmp);
  return s;
}

/*
 * Pseudo-observations of the auxiliary LGSSM at linearisation point x:
 *   order 2 (eq. second-order): Omega_t = (2/delta I - Lambda_t)^{-1},
 *                                omega_t = Omega_t (2/delta u_t + v_t - Lambda_t x_t);
 *   order 1 (eq. gaussian-FK-proposal): Lambda_t = 0, so Omega_t = delta/2 I and
 *                                omega_t = u_t + delta/2 v_t.
 * Omega: [N,dx,dx] dense.  loghsum receives sum_t log h_t(y_t|x_t).
 * Returns 0, or 1 + t when 2/delta I - Lambda_t is not positive definite.
 */
/*
 * Linearisation of the observation model (eq. observation-approx):
 * h_t(y_t | z) ~ N(y_t; H_t z + c_t, R_t) around x_t, by the statistical
 * linear regression of App. "Generalised statistical linear regression"
 * (eq. coeffs with the moments of eq. general-GSLR-coeffs) for the reference
 * variable zeta ~ N(x_t, Gamma), Gamma = slr_var I:
 *   mu = E[m(zeta)], C = Cov[m(zeta), zeta], S = E[V(zeta)] + Var[m(zeta)],
 *   H = C Gamma^{-1}, c = mu - H x, R = S - H Gamma H^T,
 * over the observed sites (NaN entries dropped).  slr_var = 0 is the Taylor
 * (extended) limit: H = dm/dx at x, c = m(x) - H x, R = E[V].  Families with a
 * Gaussian observation around a mean: Gaussian at sites (m_k = x_i, V = s^2)
 * and quadratic mean (m_k = x_i + beta x_i^2, V = s^2); the moments of a
 * quadratic of a Gaussian are exact:
 *   E[zeta_i^2] = x_i^2 + g2, Cov(zeta_i^2, zeta_i) = 2 x_i g2,
 *   Var(zeta_i^2) = 4 x_i^2 g2 + 2 g2^2  (g2 = slr_var).
 * The proposal of eq. two-lin-prop then sees this Gaussian in place of h_t,
 * whose log density at z = x has gradient and Hessian
 *   v = H^T R^{-1} (y - c - H x),  Lambda = -H^T R^{-1} H,
 * written to v [dx], Lam [dx,dx].  Returns 0, or -1 for another family or a
 * non-positive-definite R.
 */
int or_obs_linearise(const or_model* M, const double* yt, const double* xt, double* v,
                     double* Lam) {
  const int n = M->dx, p = M->dy;
  const double s2 = M->scale * M->scale, g2 = M->slr_var;
  const double be = (M->emit == OR_EMIT_GAUSS_QUAD) ? M->obs_beta : 0.0;
  memset(v, 0, sizeof(double) * n);
  memset(Lam, 0, sizeof(double) * n * n);
  if (M->emit != OR_EMIT_GAUSS_SITE && M->emit != OR_EMIT_GAUSS_QUAD) return -1;
  int* ks = malloc(sizeof(int) * p);
  int po = 0;
  for (int k = 0; k < p; ++k)
    if (!isnan(yt[k])) ks[po++] = k;
  if (po == 0) {
    free(ks);
    return 0;
  }
  double* mu = malloc(sizeof(double) * po);
  double* H = calloc((size_t)po * n, sizeof(double));
  double* R = malloc(sizeof(double) * po * po);
  double* L = malloc(sizeof(double) * po * po);
  double* r = malloc(sizeof(double) * po);
  double* RiH = malloc(sizeof(double) * po * n);
  double* col = malloc(sizeof(double) * po);
  /* moments over zeta (coordinates independent under Gamma = g2 I) */
  for (int a = 0; a < po; ++a) {
    const int i = M->site[ks[a]];
    const double x = xt[i];
    const double Ez2 = x * x + g2;
    mu[a] = x + be * Ez2;
    /* C_a,i = Cov(zeta + beta zeta^2, zeta) = g2 + 2 beta x g2; H = C / g2, or
       dm/dx in the Taylor limit (the same value) */
    H[a * n + i] = 1.0 + 2.0 * be * x;
  }
  for (int a = 0; a < po; ++a)
    for (int b = 0; b < po; ++b) {
      const int i = M->site[ks[a]], j = M->site[ks[b]];
      double S = (a == b) ? s2 : 0.0;
      if (g2 > 0.0 && i == j) {
        const double x = xt[i];
        /* Var(zeta + beta zeta^2) = g2 + 4 beta x g2 + beta^2 (4 x^2 g2 + 2 g2^2) */
        S += g2 + 4.0 * be * x * g2 + be * be * (4.0 * x * x * g2 + 2.0 * g2 * g2);
      }
      /* R = S - H Gamma H^T */
      double hgh = 0.0;
      for (int q = 0; q < n; ++q) hgh += H[a * n + q] * g2 * H[b * n + q];
      R[a * po + b] = S - hgh;
    }
  int rc = chol(po, R, L);
  if (!rc) {
    /* residual y - c - H x = y - mu */
    for (int a = 0; a < po; ++a) r[a] = yt[ks[a]] - mu[a];
    fwd_sub(po, L, r);
    bwd_sub(po, L, r);
    for (int q = 0; q < n; ++q) {
      double sq = 0.0;
      for (int a = 0; a < po; ++a) sq += H[a * n + q] * r[a];
      v[q] = sq;
    }
    memcpy(RiH, H, sizeof(double) * po * n);
    chol_solve(po, n, L, RiH, col);
    mm_tn(n, n, po, H, RiH, Lam);
    for (int q = 0; q < n * n; ++q) Lam[q] = -Lam[q];
    symmetrise(n, Lam);
  }
  free(ks); free(mu); free(H); free(R); free(L); free(r); free(RiH); free(col);
  return rc ? -1 : 0;
}

int or_linearise(const or_model* M, const double* y, const double* x, const double* u, double delta,
                 int order, double* omega, double* Omega, double* loghsum) {
  const int n = M->dx, p = M->dy;
  double* v = malloc(sizeof(double) * n);
  double* Lam = malloc(sizeof(double) * n * n);
  double* Prec = malloc(sizeof(double) * n * n);
  double* L = malloc(sizeof(double) * n * n);
  double* rhs = malloc(sizeof(double) * n);
  double* col = malloc(sizeof(double) * n);
  double* I = malloc(sizeof(double) * n * n);
  double lhs = 0.0;
  int rc = 0;
  for (long t = 0; t < M->N; ++t) {
    const double* xt = x + t * n;
    if (order == 3) {
      /* the linearised observation model in place of log h's own derivatives */
      lhs += or_emission(M, y + t * p, xt, NULL, NULL);
      if (or_obs_linearise(M, y + t * p, xt, v, Lam)) {
        if (rc == 0) rc = 1 + (int)t;
        memset(omega + t * n, 0, sizeof(double) * n);
        memset(Omega + t * n * n, 0, sizeof(double) * n * n);
        continue;
      }
    } else {
      lhs += or_emission(M, y + t * p, xt, v, Lam);
    }
    if (order == 1) memset(Lam, 0, sizeof(double) * n * n);
    for (int i = 0; i < n * n; ++i) Prec[i] = -Lam[i];
    for (int i = 0; i < n; ++i) Prec[i * n + i] += 2.0 / delta;
    if (chol(n, Prec, L)) {
      if (rc == 0) rc = 1 + (int)t;
      memset(omega + t * n, 0, sizeof(double) * n);
      memset(Omega + t * n * n, 0, sizeof(double) * n * n);
      continue;
    }
    /* Omega = Prec^{-1} */
    memset(I, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
    chol_solve(n, n, L, I, col);
    symmetrise(n, I);
    memcpy(Omega + t * n * n, I, sizeof(double) * n * n);
    /* rhs = 2/delta u + v - Lam x */
    mv(n, n, Lam, xt, rhs);
    for (int i = 0; i < n; ++i) rhs[i] = 2.0 / delta * u[t * n + i] + v[i] - rhs[i];
    mv(n, n, I, rhs, omega + t * n);
  }
  if (loghsum) *loghsum = lhs;
  free(v); free(Lam); free(Prec); free(L); free(rhs); free(col); free(I);
  return rc;
}

/* ------------------------------------------------------------------ */
/* One auxiliary Kalman MH step                                         */
/* ------------------------------------------------------------------ */

enum { OR_ST_FWD_NOT_PD = 1, OR_ST_REV_NOT_PD = 2, OR_ST_NONFINITE = 4 };

/* sum_t log N(omega_t; z_t, Omega_t) */
static double pseudo_obs_loglik(int N, int n, const double* omega, const double* Omega,
                                const double* z, double* L, double* tmp) {
  double s = 0.0;
  for (long t = 0; t < N; ++t) {
    if (chol(n, Omega + t * n * n, L)) return NAN;
    s += gauss_logpdf_chol(n, omega + t * n, z + t * n, L, tmp);
  }
  return s;
}

/*
 * One step of the auxiliary Kalman sampler with Sigma_t = I (Alg. "General
 * Auxiliary Kalman sampler", Gaussian dynamics so the dynamics linearisation
 * is the identity).  Inputs: current path x [N,dx], xi_u, xi_x [N,dx] standard
 * normals, unif in (0,1).  u_t = x_t + sqrt(delta/2) xi_u_t.
 *
 * log r = sum_t [log h(y_t|x*_t) - log h(y_t|x_t)]
 *       + sum_t [|u_t - x_t|^2 - |u_t - x*_t|^2] / delta
 *       + sum_t [log N(omega*_t; x_t, Omega*_t) - log N(omega_t; x*_t, Omega_t)]
 *       + log Z(x) - log Z(x*),
 * the prior p0 prod p_t cancelling between target and both proposals; Z(.) is
 * the auxiliary LGSSM marginal likelihood (eq. marginal-likelihood).  With
 * nonlinear dynamics the proposals use the extended linearisation of f around
 * x and x* (Alg. "General Auxiliary Kalman sampler", eq. auxiliary-LGSSM) and
 * log r gains dyn_mismatch(x*; at x) - dyn_mismatch(x; at x*).  Accept iff
 * log(unif) < log r.  x_out may alias x.  Diagnostics (may be NULL):
 * xstar [N,dx], ell_f [N] per-step log-likelihood terms of the forward filter.
 * Returns the status bitmask (0 = all well-defined).
 */
int or_mh_step(const or_model* M, const double* y, const double* x, double delta, int order,
               const double* xi_u, const double* xi_x, double unif, double* x_out,
               double* log_ratio, int* accepted, double* logZ_fwd, double* logZ_rev,
               double* xstar_out, double* ell_f_out) {
  const int N = M->N, n = M->dx;
  const size_t vn = (size_t)N * n, mn = (size_t)N * n * n;
  double* u = malloc(sizeof(double) * vn);
  double* om = malloc(sizeof(double) * vn);
  double* Om = malloc(sizeof(double) * mn);
  double* om2 = malloc(sizeof(double) * vn);
  double* Om2 = malloc(sizeof(double) * mn);
  double* mf = malloc(sizeof(double) * vn);
  double* Pf = malloc(sizeof(double) * mn);
  double* mp = malloc(sizeof(double) * vn);
  double* Pp = malloc(sizeof(double) * mn);
  double* ell = malloc(sizeof(double) * N);
  double* xs = malloc(sizeof(double) * vn);
  double* I = malloc(sizeof(double) * n * n);
  double* L = malloc(sizeof(double) * n * n);
  double* tmp = malloc(sizeof(double) * n);
  int status = 0;
  double lr = -INFINITY, lzf = NAN, lzr = NAN;
  memset(I, 0, sizeof(double) * n * n);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  const double su = sqrt(0.5 * delta);
  for (size_t i = 0; i < vn; ++i) u[i] = x[i] + su * xi_u[i];

  double lh_x = 0.0, lh_s = 0.0;
  /* dynamics of the auxiliary LGSSM: the model's (F, b), or the extended
     linearisation of f around x (forward) and x* (reverse) */
  const int nl = M->dyn != OR_DYN_LINEAR;
  double* Fx = nl ? malloc(sizeof(double) * mn) : NULL;
  double* bx = nl ? malloc(sizeof(double) * vn) : NULL;
  double* Fs = nl ? malloc(sizeof(double) * mn) : NULL;
  double* bs = nl ? malloc(sizeof(double) * vn) : NULL;
  const long Fst = nl ? (long)n * n : 0, bst = nl ? n : 0;
  if (nl) or_dyn_linearise(M, x, Fx, bx);
  const double* Ff = nl ? Fx : M->F;
  const double* bf = nl ? bx : M->b;
  /* forward proposal at x */
  if (or_linearise(M, y, x, u, delta, order, om, Om, &lh_x)) status |= OR_ST_FWD_NOT_PD;
  if (!status) {
    if (or_kf(N, n, n, M->m0, M->P0, Ff, Fst, bf, bst, M->Q, I, 0, Om, (long)n * n, om, mf, Pf, mp,
              Pp, ell))
      status |= OR_ST_FWD_NOT_PD;
  }
  if (!status) {
    lzf = 0.0;
    for (int t = 0; t < N; ++t) lzf += ell[t];
    if (ell_f_out) memcpy(ell_f_out, ell, sizeof(double) * N);
    if (or_rts_sample(N, n, Ff, Fst, mf, Pf, mp, Pp, xi_x, xs)) status |= OR_ST_FWD_NOT_PD;
  }
  if (!status) {
    if (xstar_out) memcpy(xstar_out, xs, sizeof(double) * vn);
    /* reverse proposal at x*, same u */
    if (or_linearise(M, y, xs, u, delta, order, om2, Om2, &lh_s)) status |= OR_ST_REV_NOT_PD;
  }
  if (nl && !status) or_dyn_linearise(M, xs, Fs, bs);
  const double* Fr = nl ? Fs : M->F;
  const double* br = nl ? bs : M->b;
  if (!status) {
    if (or_kf(N, n, n, M->m0, M->P0, Fr, Fst, br, bst, M->Q, I, 0, Om2, (long)n * n, om2, NULL,
              NULL, NULL, NULL, ell))
      status |= OR_ST_REV_NOT_PD;
  }
  if (!status) {
    lzr = 0.0;
    for (int t = 0; t < N; ++t) lzr += ell[t];
    double aux = 0.0;
    for (size_t i = 0; i < vn; ++i) {
      double a = u[i] - x[i], c = u[i] - xs[i];
      aux += a * a - c * c;
    }
    aux /= delta;
    double q_rev = pseudo_obs_loglik(N, n, om2, Om2, x, L, tmp);
    double q_fwd = pseudo_obs_loglik(N, n, om, Om, xs, L, tmp);
    lr = (lh_s - lh_x) + aux + (q_rev - q_fwd) + (lzf - lzr);
    if (nl) lr += dyn_mismatch(M, xs, Fx, bx) - dyn_mismatch(M, x, Fs, bs);
    if (!isfinite(lr)) {
      status |= OR_ST_NONFINITE;
      lr = -INFINITY;
    }
  }
  int acc = (status == 0) && (log(unif) < lr);
  if (status) lr = -INFINITY;
  if (x_out != x) memcpy(x_out, x, sizeof(double) * vn);
  if (acc) memcpy(x_out, xs, sizeof(double) * vn);
  if (log_ratio) *log_ratio = lr;
  if (accepted) *accepted = acc;
  if (logZ_fwd) *logZ_fwd = lzf;
  if (logZ_rev) *logZ_rev = lzr;
  free(u); free(om); free(Om); free(om2); free(Om2); free(mf); free(Pf); free(mp); free(Pp);
  free(ell); free(xs); free(I); free(L); free(tmp);
  free(Fx); free(bx); free(Fs); free(bs);
  return status;
}

/*
 * A chain of n_steps MH steps.  xi: [n_steps, 2, N, dx] (u-noise then path
 * noise), unif: [n_steps].  x is updated in place; per-step log r, acceptance
 * and status are written when the arrays are non-NULL; samples (if non-NULL)
 * receives the path after every step, [n_steps, N, dx].
 */
int or_mh_chain(const or_model* M, const double* y, double* x, double delta, int order, int n_steps,
                const double* xi, const double* unif, double* log_ratio, int* accepted,
                int* status, double* samples) {
  const size_t vn = (size_t)M->N * M->dx;
  for (int s = 0; s < n_steps; ++s) {
    double lr;
    int acc;
    int st = or_mh_step(M, y, x, delta, order, xi + (size_t)s * 2 * vn, xi + ((size_t)s * 2 + 1) * vn,
                        unif[s], x, &lr, &acc, NULL, NULL, NULL, NULL);
    if (log_ratio) log_ratio[s] = lr;
    if (accepted) accepted[s] = acc;
    if (status) status[s] = st;
    if (samples) memcpy(samples + (size_t)s * vn, x, sizeof(double) * vn);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* The same step when the auxiliary LGSSM factorises over coordinates   */
/* ------------------------------------------------------------------ */

/*
 * Diagonal linearisation: Omega_t = diag(1 / (2/delta - Lambda_t,ii)) and
 * omega_t,i = Omega_t,i (2/delta u_t,i + v_t,i - Lambda_t,ii x_t,i) (eq.
 * second-order with Sigma_t = I; Lambda = 0 under order 1).  Omega [N,dx]
 * holds the diagonals.  Returns 0, 1 + t when a precision is not positive at
 * step t, or -1 when order 2 meets an off-diagonal Hessian entry.
 */
static int linearise_diag(const or_model* M, const double* y, const double* x, const double* u,
                          double delta, int order, double* omega, double* Omega, double* loghsum) {
  const int n = M->dx, p = M->dy;
  double* v = malloc(sizeof(double) * n);
  double* Lam = malloc(sizeof(double) * n * n);
  double lhs = 0.0;
  int rc = 0;
  for (long t = 0; t < M->N && rc >= 0; ++t) {
    const double* xt = x + t * n;
    lhs += or_emission(M, y + t * p, xt, v, Lam);
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j)
        if (order == 2 && i != j && Lam[i * n + j] != 0.0) rc = -1;
      const double lam = (order == 1) ? 0.0 : Lam[i * n + i];
      const double prec = 2.0 / delta - lam;
      if (!(prec > 0.0) || !isfinite(v[i])) {
        if (rc == 0) rc = 1 + (int)t;
        omega[t * n + i] = 0.0;
        Omega[t * n + i] = 1.0;
        continue;
      }
      Omega[t * n + i] = 1.0 / prec;
      omega[t * n + i] = Omega[t * n + i] * (2.0 / delta * u[t * n + i] + v[i] - lam * xt[i]);
    }
  }
  if (loghsum) *loghsum = lhs;
  free(v); free(Lam);
  return rc;
}

/*
 * Auxiliary LGSSM of a factorising prior (P0, F, Q diagonal) with diagonal
 * Omega_t: dx independent one-dimensional LGSSMs (Sec. "Spatio-temporal
 * model"), each filtered by or_kf and, when xi_x != NULL, sampled by
 * or_rts_sample with dx = dy = 1.  Returns the sum of the per-coordinate log
 * marginal likelihoods (NaN on a filter failure); xs [N,dx] receives the path.
 */
static double factorised_filter_sample(const or_model* M, const double* om, const double* Om,
                                       const double* xi_x, double* xs, int* fail) {
  const int N = M->N, n = M->dx;
  double* yi = malloc(sizeof(double) * N);
  double* Ri = malloc(sizeof(double) * N);
  double* xii = malloc(sizeof(double) * N);
  double* mf = malloc(sizeof(double) * N);
  double* Pf = malloc(sizeof(double) * N);
  double* mp = malloc(sizeof(double) * N);
  double* Pp = malloc(sizeof(double) * N);
  double* ell = malloc(sizeof(double) * N);
  double* xo = malloc(sizeof(double) * N);
  const double one = 1.0;
  double lz = 0.0;
  *fail = 0;
  for (int i = 0; i < n && !*fail; ++i) {
    for (int t = 0; t < N; ++t) {
      yi[t] = om[(long)t * n + i];
      Ri[t] = Om[(long)t * n + i];
    }
    const double F = M->F[i * n + i], Q = M->Q[i * n + i], P0 = M->P0[i * n + i];
    if (or_kf(N, 1, 1, M->m0 + i, &P0, &F, 0, M->b ? M->b + i : NULL, 0, &Q, &one, 0, Ri, 1, yi, mf,
              Pf, mp, Pp, ell)) {
      *fail = 1;
      break;
    }
    for (int t = 0; t < N; ++t) lz += ell[t];
    if (xi_x) {
      for (int t = 0; t < N; ++t) xii[t] = xi_x[(long)t * n + i];
      if (or_rts_sample(N, 1, &F, 0, mf, Pf, mp, Pp, xii, xo)) {
        *fail = 1;
        break;
      }
      for (int t = 0; t < N; ++t) xs[(long)t * n + i] = xo[t];
    }
  }
  free(yi); free(Ri); free(xii); free(mf); free(Pf); free(mp); free(Pp); free(ell); free(xo);
  return *fail ? NAN : lz;
}

/*
 * or_mh_step for a prior that factorises over coordinates (P0, F and Q
 * diagonal; b arbitrary) and a diagonal Omega_t (order 1, or order 2 with a
 * diagonal emission Hessian).  The auxiliary proposal is then a product of dx
 * one-dimensional LGSSMs while the target stays coupled through h_t (Sec.
 * "Spatio-temporal model").  Same inputs, outputs and status bits as
 * or_mh_step; returns -1 when the model does not factorise.
 */
int or_mh_step_factorised(const or_model* M, const double* y, const double* x, double delta,
                          int order, const double* xi_u, const double* xi_x, double unif,
                          double* x_out, double* log_ratio, int* accepted, double* logZ_fwd,
                          double* logZ_rev, double* xstar_out) {
  const int N = M->N, n = M->dx;
  if (M->dyn != OR_DYN_LINEAR || order == 3) return -1;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (i != j && (M->F[i * n + j] != 0.0 || M->Q[i * n + j] != 0.0 || M->P0[i * n + j] != 0.0))
        return -1;
  const size_t vn = (size_t)N * n;
  double* u = malloc(sizeof(double) * vn);
  double* om = malloc(sizeof(double) * vn);
  double* Om = malloc(sizeof(double) * vn);
  double* om2 = malloc(sizeof(double) * vn);
  double* Om2 = malloc(sizeof(double) * vn);
  double* xs = malloc(sizeof(double) * vn);
  int status = 0, rc, fail;
  double lr = -INFINITY, lzf = NAN, lzr = NAN, lh_x = 0.0, lh_s = 0.0;
  const double su = sqrt(0.5 * delta);
  for (size_t i = 0; i < vn; ++i) u[i] = x[i] + su * xi_u[i];

  rc = linearise_diag(M, y, x, u, delta, order, om, Om, &lh_x);
  if (rc < 0) goto unsupported;
  if (rc) status |= OR_ST_FWD_NOT_PD;
  if (!status) {
    lzf = factorised_filter_sample(M, om, Om, xi_x, xs, &fail);
    if (fail) status |= OR_ST_FWD_NOT_PD;
  }
  if (!status) {
    if (xstar_out) memcpy(xstar_out, xs, sizeof(double) * vn);
    rc = linearise_diag(M, y, xs, u, delta, order, om2, Om2, &lh_s);
    if (rc < 0) goto unsupported;
    if (rc) status |= OR_ST_REV_NOT_PD;
  }
  if (!status) {
    lzr = factorised_filter_sample(M, om2, Om2, NULL, NULL, &fail);
    if (fail) status |= OR_ST_REV_NOT_PD;
  }
  if (!status) {
    double aux = 0.0, q_rev = 0.0, q_fwd = 0.0;
    for (size_t i = 0; i < vn; ++i) {
      const double a = u[i] - x[i], c = u[i] - xs[i];
      aux += a * a - c * c;
      const double r2 = om2[i] - x[i], f2 = om[i] - xs[i];
      q_rev += -0.5 * (LOG2PI + log(Om2[i]) + r2 * r2 / Om2[i]);
      q_fwd += -0.5 * (LOG2PI + log(Om[i]) + f2 * f2 / Om[i]);
    }
    lr = (lh_s - lh_x) + aux / delta + (q_rev - q_fwd) + (lzf - lzr);
    if (!isfinite(lr)) {
      status |= OR_ST_NONFINITE;
      lr = -INFINITY;
    }
  }
  {
    const int acc = (status == 0) && (log(unif) < lr);
    if (status) lr = -INFINITY;
    if (x_out != x) memcpy(x_out, x, sizeof(double) * vn);
    if (acc) memcpy(x_out, xs, sizeof(double) * vn);
    if (log_ratio) *log_ratio = lr;
    if (accepted) *accepted = acc;
    if (logZ_fwd) *logZ_fwd = lzf;
    if (logZ_rev) *logZ_rev = lzr;
  }
  free(u); free(om); free(Om); free(om2); free(Om2); free(xs);
  return status;
unsupported:
  free(u); free(om); free(Om); free(om2); free(Om2); free(xs);
  return -1;
}

/* A chain of or_mh_step_factorised steps; arguments as or_mh_chain. */
int or_mh_chain_factorised(const or_model* M, const double* y, double* x, double delta, int order,
                           int n_steps, const double* xi, const double* unif, double* log_ratio,
                           int* accepted, int* status, double* samples) {
  const size_t vn = (size_t)M->N * M->dx;
  for (int s = 0; s < n_steps; ++s) {
    double lr;
    int acc;
    int st = or_mh_step_factorised(M, y, x, delta, order, xi + (size_t)s * 2 * vn,
                                   xi + ((size_t)s * 2 + 1) * vn, unif[s], x, &lr, &acc, NULL,
                                   NULL, NULL);
    if (st < 0) return -1;
    if (log_ratio) log_ratio[s] = lr;
    if (accepted) accepted[s] = acc;
    if (status) status[s] = st;
    if (samples) memcpy(samples + (size_t)s * vn, x, sizeof(double) * vn);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* LGSSM log-likelihood and its Fisher-identity score                   */
/* ------------------------------------------------------------------ */

/*
 * log p(y | theta) for  x_0 ~ N(m0,P0), x_t = F x_{t-1} + N(0, diag exp(logq)),
 * y_t = H x_t + N(0, diag exp(logr)).  Returns the log-likelihood (NaN on failure).
 */
double or_lgssm_loglik(int N, int dx, int dy, const double* m0, const double* P0, const double* F,
                       const double* logq, const double* H, const double* logr, const double* y) {
  double* Q = calloc((size_t)dx * dx, sizeof(double));
  double* R = calloc((size_t)dy * dy, sizeof(double));
  double* ell = malloc(sizeof(double) * N);
  for (int i = 0; i < dx; ++i) Q[i * dx + i] = exp(logq[i]);
  for (int i = 0; i < dy; ++i) R[i * dy + i] = exp(logr[i]);
  int rc = or_kf(N, dx, dy, m0, P0, F, 0, NULL, 0, Q, H, 0, R, 0, y, NULL, NULL, NULL, NULL, ell);
  double s = 0.0;
  for (int t = 0; t < N; ++t) s += ell[t];
  free(Q); free(R); free(ell);
  return rc ? NAN : s;
}

/*
 * Fisher's identity: grad log p(y|theta) = E[grad log p(x, y | theta) | y], with
 * the expectation taken from the RTS smoother (marginals m^s, P^s and lag-one
 * covariances Cov(x_t, x_{t-1} | y) = P^s_t G_{t-1}^T).  Complete-data
 * statistics (sums over t = 1..N-1):
 *   S00 = sum E[x_{t-1} x_{t-1}^T], S10 = sum E[x_t x_{t-1}^T], S11 = sum E[x_t x_t^T]
 *   dF        = Q^{-1} (S10 - F S00)
 *   dlogq_i   = -(N-1)/2 + exp(-logq_i) Psi_ii / 2,
 *               Psi = S11 - F S10^T - S10 F^T + F S00 F^T
 *   dH        = R^{-1} (sum_t y_t m_t^T - H sum_t E[x_t x_t^T])        (t = 0..N-1)
 *   dlogr_j   = -N/2 + exp(-logr_j) Phi_jj / 2,
 *               Phi = sum_t E[(y_t - H x_t)(y_t - H x_t)^T]
 * Returns the log-likelihood (NaN on failure).
 */
double or_fisher_score(int N, int dx, int dy, const double* m0, const double* P0, const double* F,
                       const double* logq, const double* H, const double* logr, const double* y,
                       double* dF, double* dlogq, double* dH, double* dlogr) {
  const int n = dx, p = dy;
  const size_t vn = (size_t)N * n, mn = (size_t)N * n * n;
  double* Q = calloc((size_t)n * n, sizeof(double));
  double* R = calloc((size_t)p * p, sizeof(double));
  for (int i = 0; i < n; ++i) Q[i * n + i] = exp(logq[i]);
  for (int i = 0; i < p; ++i) R[i * p + i] = exp(logr[i]);
  double* mf = malloc(sizeof(double) * vn);
  double* Pf = malloc(sizeof(double) * mn);
  double* mp = malloc(sizeof(double) * vn);
  double* Pp = malloc(sizeof(double) * mn);
  double* ms = malloc(sizeof(double) * vn);
  double* Ps = malloc(sizeof(double) * mn);
  double* G = malloc(sizeof(double) * mn);
  double* ell = malloc(sizeof(double) * N);
  double* S00 = calloc((size_t)n * n, sizeof(double));
  double* S10 = calloc((size_t)n * n, sizeof(double));
  double* S11 = calloc((size_t)n * n, sizeof(double));
  double* Sxx = calloc((size_t)n * n, sizeof(double));
  double* Syx = calloc((size_t)p * n, sizeof(double));
  double* Phi = calloc((size_t)p * p, sizeof(double));
  double* T = malloc(sizeof(double) * n * n);
  double* T2 = malloc(sizeof(double) * n * n);
  double* Psi = malloc(sizeof(double) * n * n);
  double* HM = malloc(sizeof(double) * p * n);
  double* HP = malloc(sizeof(double) * p * n);
  double* r = malloc(sizeof(double) * p);
  double ll = NAN;
  int rc = or_kf(N, n, p, m0, P0, F, 0, NULL, 0, Q, H, 0, R, 0, y, mf, Pf, mp, Pp, ell);
  if (!rc) rc = or_rts_smooth(N, n, F, 0, mf, Pf, mp, Pp, ms, Ps, G);
  if (!rc) {
    ll = 0.0;
    for (int t = 0; t < N; ++t) ll += ell[t];
    for (long t = 0; t < N; ++t) {
      const double* m = ms + t * n;
      const double* P = Ps + t * n * n;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Sxx[i * n + j] += P[i * n + j] + m[i] * m[j];
      for (int k = 0; k < p; ++k)
        for (int j = 0; j < n; ++j) Syx[k * n + j] += y[t * p + k] * m[j];
      /* E[(y - Hx)(y - Hx)^T] = (y - H m)(y - H m)^T + H P H^T */
      mv(p, n, H, m, r);
      for (int k = 0; k < p; ++k) r[k] = y[t * p + k] - r[k];
      mm(p, n, n, H, P, HP);
      for (int k = 0; k < p; ++k)
        for (int l = 0; l < p; ++l) {
          double s = 0.0;
          for (int j = 0; j < n; ++j) s += HP[k * n + j] * H[l * n + j];
          Phi[k * p + l] += r[k] * r[l] + s;
        }
      if (t >= 1) {
        const double* m0t = ms + (t - 1) * n;
        const double* P0t = Ps + (t - 1) * n * n;
        /* Cov(x_t, x_{t-1}) = P^s_t G_{t-1}^T */
        mm_nt(n, n, n, P, G + (t - 1) * n * n, T);
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) {
            S00[i * n + j] += P0t[i * n + j] + m0t[i] * m0t[j];
            S10[i * n + j] += T[i * n + j] + m[i] * m0t[j];
            S11[i * n + j] += P[i * n + j] + m[i] * m[j];
          }
      }
    }
    /* dF = Q^{-1}(S10 - F S00) */
    mm(n, n, n, F, S00, T);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) dF[i * n + j] = (S10[i * n + j] - T[i * n + j]) / Q[i * n + i];
    /* Psi = S11 - F S10^T - S10 F^T + F S00 F^T */
    mm_nt(n, n, n, F, S10, T2); /* F S10^T */
    mm_nt(n, n, n, T, F, Psi);  /* F S00 F^T */
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        Psi[i * n + j] += S11[i * n + j] - T2[i * n + j] - T2[j * n + i];
    for (int i = 0; i < n; ++i)
      dlogq[i] = -0.5 * (N - 1) + 0.5 * exp(-logq[i]) * Psi[i * n + i];
    /* dH = R^{-1}(Syx - H Sxx) */
    mm(p, n, n, H, Sxx, HM);
    for (int k = 0; k < p; ++k)
      for (int j = 0; j < n; ++j) dH[k * n + j] = (Syx[k * n + j] - HM[k * n + j]) / R[k * p + k];
    for (int k = 0; k < p; ++k) dlogr[k] = -0.5 * N + 0.5 * exp(-logr[k]) * Phi[k * p + k];
  }
  free(Q); free(R); free(mf); free(Pf); free(mp); free(Pp); free(ms); free(Ps); free(G); free(ell);
  free(S00); free(S10); free(S11); free(Sxx); free(Syx); free(Phi); free(T); free(T2); free(Psi);
  free(HM); free(HP); free(r);
  return ll;
}
