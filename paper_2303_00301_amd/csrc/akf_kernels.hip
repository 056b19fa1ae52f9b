// akf_kernels.hip -- gfx950 kernels for one auxiliary-Kalman MH step.
//
// Method: Corenflos & Sarkka, auxiliary Kalman sampler (Alg. "General
// Auxiliary Kalman sampler", eq. second-order / gaussian-FK-proposal) with the
// parallel-in-time filter (App. A, "Prefix-sums and the parallel Kalman
// filter") and the parallel pathwise RTS sampler (App. A, "Parallel
// Rauch--Tung--Striebel sampler", eq. backward, eq. EgL_comb).
//
// The auxiliary LGSSM of one step has the model's Gaussian dynamics and the
// pseudo-observation omega_t = x_t + N(0, Omega_t) (H = I).  Both scans are
// blocked, reduce-then-scan, with one team (workgroup) per block of B time
// steps:
//   filter  : fold   -- each block folds its elements sequentially into the
//                       block element (A, b, C, eta, J);
//             tree   -- work-efficient up-sweep (full element combine) and
//                       down-sweep (prefix applied to an element) over the
//                       block elements -> filtering moments entering each block;
//             final  -- each block re-runs its steps from that prefix, giving
//                       m^f_t, P^f_t and the predictive log-likelihood terms.
//   sampler : build  -- one team per t: E_t, U_t = g_t + chol(L_t) xi_t;
//             fold   -- suffix aggregate of (E, U) per block;
//             tree   -- up-sweep (E_i E_j, E_i U_j + U_i), down-sweep of the
//                       boundary states;
//             final  -- x*_t = E_t x*_{t+1} + U_t inside each block.
// Every matrix product is an f64 MFMA; Cholesky factors are FP64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "akf_team.hpp"
#include "akf_internal.h"

namespace akf {

static constexpr double LOG2PI = 1.8378770664093454835606594728112;

__device__ __forceinline__ void flag_status(int* st, int bit) { atomicOr(st, bit); }

// ---------------------------------------------------------------------------
// status word / scalar reset (graph-safe replacement for a memset)
// ---------------------------------------------------------------------------
// Also marks the root of the filter prefix tree as the identity and sets the
// state entering the sampler's last block from the right to zero (it is
// multiplied by E = 0 of the terminal step, but must be finite).
// status points at the workspace's two status words (steps alternate between
// them; the decision kernel of one step clears the next step's word), or is
// null to leave them as they are.
__global__ void k_step_init(int* status, double* root_flag, double* root_xin, int D) {
  const int tid = threadIdx.x;
  if (status && tid < 2) status[tid] = 0;
  if (tid == 0 && root_flag) *root_flag = 1.0;
  if (root_xin && tid < D) root_xin[tid] = 0.0;
}

// ---------------------------------------------------------------------------
// Emission linearisation, diagonal families (Poisson log-link, Student-t,
// stochastic volatility, Gaussian at sites).
// One thread per (t, i).  Site k observes latent site[k]; a latent observed by
// several sites sums their contributions.
//   v_i = d log h / d x_i,  Lambda_ii = d^2 log h / d x_i^2 (0 under order 1)
//   Omega_i = 1 / (2/delta - Lambda_ii),  omega_i = Omega_i (2/delta u_i + v_i - Lambda_ii x_i)
// (eq. second-order with Sigma_t = I; order 1: eq. gaussian-FK-proposal).
// ---------------------------------------------------------------------------
struct EmitOut {
  double lh, v, lam;
  double ysum;  // sum of the latent's observed y_k (order 3)
  int cnt;      // number of the latent's observed sites (order 3)
};

// One site's contribution to log h and its derivatives at x_i = xi.
__device__ __forceinline__ void emit_site(const KModel& M, double yk, double xi, EmitOut& o) {
  if (M.emit == EMIT_POISSON_LOG) {
    const double e = exp(xi);
    o.lh += yk * xi - e;
    o.v += yk - e;
    o.lam -= e;
  } else if (M.emit == EMIT_GAUSS_SITE) {
    const double s2 = M.scale * M.scale, r = yk - xi;
    o.lh += -0.5 * r * r / s2;
    o.v += r / s2;
    o.lam -= 1.0 / s2;
  } else if (M.emit == EMIT_GAUSS_QUAD) {
    const double s2 = M.scale * M.scale, dm = 1.0 + 2.0 * M.obs_beta * xi;
    const double r = yk - xi - M.obs_beta * xi * xi;
    o.lh += -0.5 * r * r / s2;
    o.v += r * dm / s2;
    o.lam += (2.0 * M.obs_beta * r - dm * dm) / s2;
  } else if (M.emit == EMIT_STOCH_VOL) {
    const double q = yk * yk * exp(-xi);  // y ~ N(0, exp(x))
    o.lh += -0.5 * xi - 0.5 * q;
    o.v += -0.5 + 0.5 * q;
    o.lam -= 0.5 * q;
  } else {
    const double a = M.nu * M.scale * M.scale;
    const double r = yk - xi, den = a + r * r;
    o.lh += -0.5 * (M.nu + 1.0) * log1p(r * r / a);
    o.v += (M.nu + 1.0) * r / den;
    o.lam += (M.nu + 1.0) * (r * r - a) / (den * den);
  }
}

// Sum over the sites observing latent i.  A site matches one lane of a wave
// (its latent), so evaluating the sites one by one would run each site's
// arithmetic with a single active lane.  Instead each pass sweeps the site
// list uniformly (scalar loads, per-lane selects) for every lane's next
// matching site, then all matched lanes load and evaluate together: one pass
// per site of the most-observed latent, plus one.
__device__ __forceinline__ EmitOut emit_diag(const KModel& M, const double* __restrict__ yt,
                                             double xi, int i) {
  EmitOut o{0.0, 0.0, 0.0, 0.0, 0};
  int start = 0;
  for (int pass = 0; pass < M.dy; ++pass) {
    int kk = -1;
    for (int k = 0; k < M.dy; ++k) {
      const int sk = M.site[k];
      kk = (kk < 0 && k >= start && sk == i) ? k : kk;
    }
    if (kk < 0) break;
    const double yk = yt[kk];
    start = kk + 1;
    if (!isnan(yk)) {  // NaN: site not observed at t
      emit_site(M, yk, xi, o);
      o.ysum += yk;
      ++o.cnt;
    }
  }
  return o;
}

// Order 3 (eq. two-lin-prop): v and Lambda become the gradient and Hessian at
// z = x of log N(y; H z + c, R), the Gaussian fitted to h around x by
// statistical linear regression with reference variable N(x, g2 I) (eq. coeffs
// with the moments of eq. general-GSLR-coeffs).  For a latent x_i observed by
// k sites with mean m(z) = z + beta z^2 and noise scale^2: each of those sites'
// rows of H is h e_i with h = 1 + 2 beta x_i, the regression mean is
// mu = x_i + beta (x_i^2 + g2), and R over those sites is scale^2 I + c 1 1'
// with c = Var m(zeta) - h^2 g2 = 2 beta^2 g2^2 (moments of a quadratic of a
// Gaussian), uncorrelated with other latents' sites.  So 1' R^{-1} =
// 1' / (scale^2 + k c), and
//   v_i = h (sum_k y_k - k mu) / (scale^2 + k c),  Lambda_ii = -h^2 k / (scale^2 + k c).
// g2 = 0 is the Taylor limit (Gauss-Newton curvature).  log h stays the true one.
__device__ __forceinline__ void slr_override(const KModel& M, double x, EmitOut& o) {
  const double be = (M.emit == EMIT_GAUSS_QUAD) ? M.obs_beta : 0.0, g2 = M.slr_var;
  const double h = 1.0 + 2.0 * be * x, mu = x + be * (x * x + g2);
  const double den = M.scale * M.scale + o.cnt * (2.0 * be * be * g2 * g2);
  o.v = h * (o.ysum - o.cnt * mu) / den;
  o.lam = -h * h * o.cnt / den;
}

// Per-(t, i) tail of the forward linearisation: draws u and writes the
// diagonal omega/Omega from v_i and Lambda_ii (0 under order 1).
__device__ __forceinline__ void lin_fwd_point(const StepArgs& A, int64_t gid, double x, double v,
                                              double lam) {
  const double u = x + sqrt(0.5 * A.delta) * A.xi_u[gid];
  A.u[gid] = u;
  const double prec = 2.0 / A.delta - lam;
  if (!(prec > 0.0) || !isfinite(v) || !isfinite(prec)) {
    flag_status(A.status, ST_FWD_NOT_PD);
    A.om[gid] = 0.0;
    A.Om[gid] = 1.0;
  } else {
    const double Om = 1.0 / prec;
    A.Om[gid] = Om;
    A.om[gid] = Om * (2.0 / A.delta * u + v - lam * x);
  }
}

// Forward linearisation at x: draws u, writes omega/Omega (diagonal), log h
// partial sums per workgroup.  blockDim.x = 256.
__device__ __forceinline__ void lin_fwd_diag_body(const KModel& M, const StepArgs& A, int item) {
  const int64_t gid = (int64_t)item * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)M.N * M.d;
  double lh = 0.0;
  if (gid < n) {
    const int t = (int)(gid / M.d), i = (int)(gid % M.d);
    const double x = A.x[gid];
    EmitOut e = emit_diag(M, A.y + (int64_t)t * M.dy, x, i);
    if (A.order == 3) slr_override(M, x, e);
    lin_fwd_point(A, gid, x, e.v, (A.order == 1) ? 0.0 : e.lam);
    lh = e.lh;
  }
  // block partial of log h(x)
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) lh += __shfl_xor(lh, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lh;
  __syncthreads();
  if (threadIdx.x == 0) A.part_lh_x[item] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_lin_fwd_diag(KModel M, StepArgs A) {
  lin_fwd_diag_body(M, A, blockIdx.x);
}

// Per-(t, i) tail of the reverse linearisation at x* with the same u: writes
// omega*/Omega* and returns the MH terms
//   [(u-x)^2 - (u-x*)^2]/delta
//   + log N(omega*_i; x_i, Omega*_i) - log N(omega_i; x*_i, Omega_i)
__device__ __forceinline__ double lin_rev_point(const StepArgs& A, int64_t gid, double xs,
                                                double v, double lam) {
  const double x = A.x[gid], u = A.u[gid];
  const double prec = 2.0 / A.delta - lam;
  double om2 = 0.0, Om2 = 1.0;
  if (!(prec > 0.0) || !isfinite(v) || !isfinite(prec)) {
    flag_status(A.status, ST_REV_NOT_PD);
  } else {
    Om2 = 1.0 / prec;
    om2 = Om2 * (2.0 / A.delta * u + v - lam * xs);
  }
  A.om2[gid] = om2;
  A.Om2[gid] = Om2;
  const double om = A.om[gid], Om = A.Om[gid];
  const double a = u - x, c = u - xs;
  const double rq = om2 - x, fq = om - xs;
  return (a * a - c * c) / A.delta +
         (-0.5 * (LOG2PI + log(Om2) + rq * rq / Om2)) - (-0.5 * (LOG2PI + log(Om) + fq * fq / Om));
}

// Reverse linearisation at x*: per-(t,i) MH terms plus log h(y|x*), reduced
// per workgroup.
__device__ __forceinline__ void lin_rev_diag_body(const KModel& M, const StepArgs& A, int item) {
  const int64_t gid = (int64_t)item * blockDim.x + threadIdx.x;
  const int64_t n = (int64_t)M.N * M.d;
  double term = 0.0, lhs = 0.0;
  if (gid < n) {
    const int t = (int)(gid / M.d), i = (int)(gid % M.d);
    const double xs = A.xs[gid];
    EmitOut e = emit_diag(M, A.y + (int64_t)t * M.dy, xs, i);
    if (A.order == 3) slr_override(M, xs, e);
    term = lin_rev_point(A, gid, xs, e.v, (A.order == 1) ? 0.0 : e.lam);
    lhs = e.lh;
  }
  __shared__ double red[8];
  for (int o = 32; o > 0; o >>= 1) {
    term += __shfl_xor(term, o);
    lhs += __shfl_xor(lhs, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = term;
    red[4 + (threadIdx.x >> 6)] = lhs;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    A.part_terms[item] = red[0] + red[1] + red[2] + red[3];
    A.part_lh_xs[item] = red[4] + red[5] + red[6] + red[7];
  }
}

__global__ void __launch_bounds__(256) k_lin_rev_diag(KModel M, StepArgs A) {
  lin_rev_diag_body(M, A, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Multivariate-t emission with precision R (Sec. "Spatio-temporal model"):
// r = y_t - x_t[site], q = r^T R r, log h = -(nu + p)/2 log(1 + q / nu) and
// v_i = (nu + p)/(nu + q) sum_{k: site[k] = i} (R r)_k.  Its Hessian couples
// every observed coordinate, so only first-order proposals (Lambda = 0) use it.
// One wave per time step, MVT_WAVES waves per workgroup sharing R, which is
// staged transposed in LDS so that lane k walks row k of R bank-conflict free.
// ---------------------------------------------------------------------------
constexpr int MVT_WAVES = kMvtWaves;

__device__ __forceinline__ void lin_mvt_body(const KModel& M, const StepArgs& A, int rev,
                                             int item) {
  constexpr int LR = 65;  // odd row stride: the transposing store is conflict-free too
  __shared__ double sRt[64 * LR];
  __shared__ double sr[MVT_WAVES * 64];
  __shared__ double sRr[MVT_WAVES * 64];
  __shared__ int ssite[64];
  __shared__ double red[2 * MVT_WAVES];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int p = M.dy, d = M.d;
  team_move<64 * MVT_WAVES, 64 * 64>(
      p * p, [&](int e) { return M.R[e]; },
      [&](int e, double v) { sRt[(e % p) * LR + e / p] = v; });
  if (tid < p) ssite[tid] = M.site[tid];
  const int t = item * MVT_WAVES + w;
  const bool active = t < M.N;
  const int64_t base = (int64_t)t * d;
  const double* xt = (rev ? A.xs : A.x) + base;
  double r = 0.0;
  if (active && lane < p) r = A.y[(int64_t)t * p + lane] - xt[M.site[lane]];
  sr[w * 64 + lane] = r;
  __syncthreads();
  double Rr = 0.0;
  if (active && lane < p) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int l = 0;
    for (; l + 4 <= p; l += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = fma(sRt[(l + u) * LR + lane], sr[w * 64 + l + u], acc[u]);
    }
    for (; l < p; ++l) acc[0] = fma(sRt[l * LR + lane], sr[w * 64 + l], acc[0]);
    Rr = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
  double q = r * Rr;
  for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o);
  sRr[w * 64 + lane] = Rr;
  __syncthreads();
  const double a = M.nu + p;
  double lh = 0.0, term = 0.0;
  if (active) {
    lh = -0.5 * a * log1p(q / M.nu);
    if (lane < d) {
      double sv = 0.0;
#pragma unroll 8
      for (int k = 0; k < p; ++k) sv += (ssite[k] == lane) ? sRr[w * 64 + k] : 0.0;
      const double v = a / (M.nu + q) * sv;
      if (rev)
        term = lin_rev_point(A, base + lane, xt[lane], v, 0.0);
      else
        lin_fwd_point(A, base + lane, xt[lane], v, 0.0);
    }
  }
  for (int o = 32; o > 0; o >>= 1) term += __shfl_xor(term, o);
  if (lane == 0) {
    red[w] = lh;
    red[MVT_WAVES + w] = term;
  }
  __syncthreads();
  if (tid == 0) {
    double sl = 0.0, st = 0.0;
    for (int k = 0; k < MVT_WAVES; ++k) {
      sl += red[k];
      st += red[MVT_WAVES + k];
    }
    if (rev) {
      A.part_lh_xs[item] = sl;
      A.part_terms[item] = st;
    } else {
      A.part_lh_x[item] = sl;
    }
  }
}

__global__ void __launch_bounds__(64 * MVT_WAVES) k_lin_mvt(KModel M, StepArgs A, int rev) {
  lin_mvt_body(M, A, rev, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Gaussian emissions y = H x + N(0, R): v = G (y - H x), Lambda = -G H with
// G = H^T R^{-1}; constant dense Omega under order 2.
// gprep (workspace, written once per step by k_gauss_prep):
//   g_G = G^T = R^{-1} H [dy, d] (row k holds column k of G),
//   g_Ht = H^T [d, dy], g_Rinv = R^{-1} [dy, dy],
//   g_Omd_inv = 2/delta I + G H [d, d] (order 2; 2/delta I under order 1),
//   g_Omd = its inverse, g_scal[0] = log det g_Omd.
// The symmetric matrices and the transposed copies let a wave read column
// i of a product as lane i of one coalesced row.
// ---------------------------------------------------------------------------
constexpr int GP_LD = 65;

// In-place Gauss-Jordan inverse of the n x n SPD matrix in sM (LDS, leading
// dimension GP_LD) into sI, which holds the identity on entry; no pivoting.
// Thread j < n owns column j of both, so an elimination step is one pass over
// rows with independent iterations.  Returns sum log(pivot) (every thread).
__device__ double gp_invert(double* sM, double* sI, double* colk, int n) {
  const int j = threadIdx.x;
  double logdet = 0.0;
  for (int k = 0; k < n; ++k) {
    if (j < n) colk[j] = sM[j * GP_LD + k];
    __syncthreads();
    const double piv = colk[k];
    logdet += log(piv);
    if (j < n) {
      const double inv = 1.0 / piv;
      const double mk = sM[k * GP_LD + j] * inv, ik = sI[k * GP_LD + j] * inv;
      for (int i = 0; i < n; ++i) {
        if (i == k) continue;
        const double f = colk[i];
        sM[i * GP_LD + j] -= f * mk;
        sI[i * GP_LD + j] -= f * ik;
      }
      sM[k * GP_LD + j] = mk;
      sI[k * GP_LD + j] = ik;
    }
    __syncthreads();
  }
  return logdet;
}

__global__ void __launch_bounds__(256) k_gauss_prep(KModel M, StepArgs A) {
  __shared__ double sM[64 * GP_LD], sI[64 * GP_LD], sH[64 * GP_LD], sG[64 * GP_LD];
  __shared__ double colk[64];
  const int tid = threadIdx.x, d = M.d, p = M.dy;
  team_move<256, 64 * 64>(
      p * d, [&](int e) { return M.H[e]; },
      [&](int e, double v) { sH[(e / d) * GP_LD + e % d] = v; });
  team_move<256, 64 * 64>(
      p * p, [&](int e) { return M.R[e]; },
      [&](int e, double v) { sM[(e / p) * GP_LD + e % p] = v; });
  for (int e = tid; e < 64 * GP_LD; e += 256) sI[e] = (e % GP_LD == e / GP_LD) ? 1.0 : 0.0;
  __syncthreads();
  gp_invert(sM, sI, colk, p);  // sI = R^{-1}
  for (int e = tid; e < p * p; e += 256) {
    const int i = e / p, j = e % p;
    A.g_Rinv[e] = 0.5 * (sI[i * GP_LD + j] + sI[j * GP_LD + i]);
  }
  // G^T = R^{-1} H and H^T
  for (int e = tid; e < p * d; e += 256) {
    const int k = e / d, i = e % d;
    double acc = 0.0;
    for (int l = 0; l < p; ++l) acc = fma(0.5 * (sI[k * GP_LD + l] + sI[l * GP_LD + k]),
                                          sH[l * GP_LD + i], acc);
    sG[k * GP_LD + i] = acc;
    A.g_G[e] = acc;
    A.g_Ht[i * p + k] = sH[k * GP_LD + i];
  }
  __syncthreads();
  // precision 2/delta I - Lambda = 2/delta I + G H; Omd = its inverse
  const double two_d = 2.0 / A.delta;
  for (int e = tid; e < 64 * GP_LD; e += 256) {
    const int i = e / GP_LD, j = e % GP_LD;
    double v = 0.0;
    if (i < d && j < d) {
      if (A.order != 1)
        for (int k = 0; k < p; ++k) v = fma(sG[k * GP_LD + i], sH[k * GP_LD + j], v);
      if (i == j) v += two_d;
      A.g_Omd_inv[i * d + j] = v;
    }
    sM[e] = v;
    sI[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const double logdet_prec = gp_invert(sM, sI, colk, d);
  for (int e = tid; e < d * d; e += 256) {
    const int i = e / d, j = e % d;
    A.g_Omd[e] = 0.5 * (sI[i * GP_LD + j] + sI[j * GP_LD + i]);
  }
  if (tid == 0) A.g_scal[0] = -logdet_prec;  // log det Omega
}

// One wave per time step (grid-stride over t, GL_WAVES waves per workgroup),
// lane i for coordinate i (or observation k).  rev = 0: forward (draw u,
// linearise at x); rev = 1: reverse (linearise at x*, same u) plus the MH
// terms.  Order 2 gives a constant dense Omega (omega = Omega (2/delta u +
// G y)); order 1 gives the diagonal Omega = delta/2 with omega = u + delta/2 v.
// log h(y_t | x) = -1/2 (y - H x)^T R^{-1} (y - H x) (constants dropped).
constexpr int GL_WAVES = 4;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// lane i: sum_j Mt[j * ld + i] v[j] for j < n (Mt row j is column j of the
// product's matrix; v in LDS, read as a broadcast), two accumulators.
__device__ __forceinline__ double gl_col_dot(const double* __restrict__ Mt, int ld, int i,
                                              const double* v, int n) {
  double a0 = 0.0, a1 = 0.0;
  int j = 0;
  for (; j + 1 < n; j += 2) {
    a0 = fma(Mt[j * ld + i], v[j], a0);
    a1 = fma(Mt[(j + 1) * ld + i], v[j + 1], a1);
  }
  if (j < n) a0 = fma(Mt[j * ld + i], v[j], a0);
  return a0 + a1;
}

__global__ void __launch_bounds__(64 * GL_WAVES) k_lin_gauss(KModel M, StepArgs A, int rev) {
  __shared__ double sv[GL_WAVES][3][64];
  __shared__ double red[GL_WAVES][2];
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int d = M.d, p = M.dy;
  const double half_d = 0.5 * A.delta, sq = sqrt(0.5 * A.delta);
  double lh_acc = 0.0, term_acc = 0.0;
  double* s0 = sv[w][0];
  double* s1 = sv[w][1];
  double* s2 = sv[w][2];
  for (int t0 = blockIdx.x * GL_WAVES; t0 < M.N; t0 += gridDim.x * GL_WAVES) {
    const int t = t0 + w;
    const bool act = t < M.N;
    const int64_t bd = (int64_t)t * d, bp = (int64_t)t * p;
    const bool li = act && l < d, lk = act && l < p;
    const double xl = li ? A.x[bd + l] : 0.0;
    const double xsl = (li && rev) ? A.xs[bd + l] : 0.0;
    double ul;
    if (!rev) {
      ul = li ? xl + sq * A.xi_u[bd + l] : 0.0;
      if (li) A.u[bd + l] = ul;
    } else {
      ul = li ? A.u[bd + l] : 0.0;
    }
    const double yk = lk ? A.y[bp + l] : 0.0;
    s0[l] = rev ? xsl : xl;  // linearisation point
    s2[l] = yk;
    __syncthreads();
    // residual r = y - H x (lane k)
    const double rk = lk ? yk - gl_col_dot(A.g_Ht, p, l, s0, d) : 0.0;
    s1[l] = rk;
    __syncthreads();
    const double Rr = lk ? gl_col_dot(A.g_Rinv, p, l, s1, p) : 0.0;
    const double lh = -0.5 * wave_sum(rk * Rr);
    double oml, Oml;
    if (A.order == 1) {
      const double v = li ? gl_col_dot(A.g_G, d, l, s1, p) : 0.0;
      Oml = half_d;
      oml = ul + half_d * v;
    } else {
      const double rhs = li ? 2.0 / A.delta * ul + gl_col_dot(A.g_G, d, l, s2, p) : 0.0;
      __syncthreads();
      s0[l] = rhs;
      __syncthreads();
      oml = li ? gl_col_dot(A.g_Omd, d, l, s0, d) : 0.0;
      Oml = li ? A.g_Omd[l * d + l] : 0.0;
    }
    double* om = rev ? A.om2 : A.om;
    double* Om = rev ? A.Om2 : A.Om;
    if (li) {
      om[bd + l] = oml;
      Om[bd + l] = Oml;
    }
    if (act) lh_acc += lh;
    if (rev) {
      // MH terms (log h difference is added from the partial sums)
      const double a = ul - xl, c = ul - xsl;
      double term = li ? (a * a - c * c) / A.delta : 0.0;
      const double omf = li ? A.om[bd + l] : 0.0;
      const double rq = li ? oml - xl : 0.0, fq = li ? omf - xsl : 0.0;
      if (A.order == 1) {
        term += li ? (-0.5 * rq * rq + 0.5 * fq * fq) / half_d : 0.0;
      } else {
        // same dense Omega both ways: log-determinants cancel
        __syncthreads();
        s0[l] = rq;
        s1[l] = fq;
        __syncthreads();
        const double sr = li ? gl_col_dot(A.g_Omd_inv, d, l, s0, d) : 0.0;
        const double sf = li ? gl_col_dot(A.g_Omd_inv, d, l, s1, d) : 0.0;
        term += -0.5 * rq * sr + 0.5 * fq * sf;
      }
      term = wave_sum(term);
      if (act) term_acc += term;
    }
    __syncthreads();
  }
  if (l == 0) {
    red[w][0] = lh_acc;
    red[w][1] = term_acc;
  }
  __syncthreads();
  if (tid == 0) {
    double lh = 0.0, term = 0.0;
    for (int i = 0; i < GL_WAVES; ++i) {
      lh += red[i][0];
      term += red[i][1];
    }
    if (rev) {
      A.part_terms[blockIdx.x] = term;
      A.part_lh_xs[blockIdx.x] = lh;
    } else {
      A.part_lh_x[blockIdx.x] = lh;
    }
  }
}

// ---------------------------------------------------------------------------
// Shared pieces of the filter kernels
// ---------------------------------------------------------------------------

// S = P + Omega_t into LDS buffer s (diagonal Omega from om_diag, or the dense
// constant Omega when dense != nullptr).  Team-wide; ends synchronised.
template <int D>
__device__ __forceinline__ void build_S(double* s, const RM<D>& P, const double* __restrict__ Om_t,
                                        const double* __restrict__ dense, int d) {
  rm_stage<D>(P, s);
  team_sync();
  const int tid = threadIdx.x;
  if (dense) {
    team_move<Cfg<D>::NT, D * D, 4>(
        d * d, [&](int e) { return dense[e]; },
        [&](int e, double v) { s[(e / d) * Cfg<D>::LD + (e % d)] += v; });
  } else if (tid < d) {
    s[tid * Cfg<D>::LD + tid] += Om_t[tid];
  }
  team_sync();
}

// Load a d x d user matrix into an LDS buffer, zero padded.
// (A rolled loop: its callers sit in per-step loops that hold most of the
// register file, where the unrolled form of lds_fill keeps its addresses live
// across the loop and spills.)
template <int D>
__device__ __forceinline__ void lds_load_mat(double* s, const double* __restrict__ g, int d) {
  for (int e = threadIdx.x; e < D * D; e += Cfg<D>::NT) {
    const int i = e / D, j = e % D;
    s[i * Cfg<D>::LD + j] = (i < d && j < d) ? g[i * d + j] : 0.0;
  }
}

// Load a padded D x D workspace matrix into an LDS buffer.
// G = 0: a rolled loop, for persistent kernels, whose outer loop would keep
// the unrolled form's addresses live (and spill).
template <int D, int G = D * D / Cfg<D>::NT>
__device__ __forceinline__ void lds_load_pad(double* s, const double* __restrict__ g) {
  if constexpr (G == 0) {
    for (int e = threadIdx.x; e < D * D; e += Cfg<D>::NT) s[(e / D) * Cfg<D>::LD + (e % D)] = g[e];
  } else {
    lds_fill<D, G>(s, [=](int i, int j) { return g[i * D + j]; });
  }
}

template <int D>
__device__ __forceinline__ void vec_load(double* s, const double* __restrict__ g, int d) {
  const int tid = threadIdx.x;
  if (tid < D) s[tid] = (tid < d && g) ? g[tid] : 0.0;
}

// Load a rows x cols user matrix (row-major) into an LDS buffer, zero padded.
template <int D>
__device__ __forceinline__ void lds_load_rect(double* s, const double* __restrict__ g, int rows,
                                              int cols) {
  for (int e = threadIdx.x; e < D * D; e += Cfg<D>::NT) {
    const int i = e / D, j = e % D;
    s[i * Cfg<D>::LD + j] = (i < rows && j < cols) ? g[i * cols + j] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Filter, phase 1: fold the elements of one block.
// State (A, b, C, eta, J) represents p(x_t | omega_{s:t}, x_{s-1}) =
// N(A x_{s-1} + b, C) and p(omega_{s:t} | x_{s-1}) ~ exp(-x'Jx/2 + eta'x).
// Appending step t (predict through the dynamics, condition on omega_t):
//   Pp = F C F' + Q, T = F A, mu = F b + bias,  S = Pp + Omega_t (inverted in
//   registers by Gauss-Jordan), w = omega_t - mu
//   C <- Pp - Pp S^{-1} Pp,  A <- T - Pp S^{-1} T,  J <- J + T' S^{-1} T,
//   b <- mu + Pp S^{-1} w,   eta <- eta + T' S^{-1} w
// which is the element combine of App. A with the raw element of step t
// written in terms of F, Q and Omega_t.  The block containing t = 0 starts
// from the prior (A = 0 throughout).  Output element layout: ElemLayout.
// GH (general observation y_t = H x_t + N(0, R), D <= 32): S = H Pp H' + R,
// Pp S^{-1} Pp -> (H Pp)' S^{-1} (H Pp), T' S^{-1} T -> (H T)' S^{-1} (H T),
// w = y_t - H mu.
// ---------------------------------------------------------------------------
// FIRST: the block contains t = 0 (its element has A = 0 and J = 0).  The
// two cases are compiled separately so that A and T hold no registers across
// the inverse.
template <int D, int OBS, bool FIRST, int U = 4>
__device__ __forceinline__ void filter_fold_impl(const KModel& M, const FilterArgs& P, int item) {
  using C = Cfg<D>;
  constexpr bool GH = (OBS == OBS_GH);
  static_assert(!GH || D <= 32, "general observation matrices need D <= 32");
  extern __shared__ double lds[];
  double* sF = lds;
  double* B1 = sF + C::MAT;
  double* B2 = B1 + C::MAT;
  double* B3 = B2 + C::MAT;
  double* sH = B3 + C::MAT;                // GH only
  double* vb = sH + (GH ? C::MAT : 0);     // b
  double* veta = vb + D;                   // eta
  double* vmu = veta + D;                  // mu
  double* vw = vmu + D;                    // omega - mu  (GH: y - H mu)
  double* vs = vw + D;                     // S^{-1} w
  double* vom = vs + D;                    // diagonal Omega_t
  double* red = vom + D;
  const int blk = item, tid = threadIdx.x, d = M.d;
  const int s0 = blk * P.B, s1 = min(M.N, s0 + P.B);
  constexpr bool first = FIRST;
  // lc: log of the normaliser, the sum over the block's steps of the
  // x_prev-independent part of log N(omega_t; T x_prev + mu, S),
  // -(dobs log 2 pi + log det S + w' S^{-1} w) / 2; log det S and this thread's
  // share of w' S^{-1} w are accumulated, the team sum is taken once at the end
  double ld_sum = 0.0, q_part = 0.0;
  const int dobs = GH ? P.dyo : d;
  if (!P.Ft) lds_load_mat<D>(sF, M.F, d);
  if (GH) lds_load_rect<D>(sH, P.Ho, P.dyo, d);
  if (tid < D) {
    vb[tid] = 0.0;
    veta[tid] = 0.0;
  }
  RM<D> A, Cc, J, T, R1, R2;
  rm_eye<D>(A, d);
  rm_zero<D>(Cc);
  rm_zero<D>(J);
  team_sync();
  bool ok = true;
  for (int t = s0; t < s1; ++t) {
    RM<D> Pp;
    if (t == 0) {
      rm_load<D>(Pp, M.P0, d, d);
      if (tid < D) vmu[tid] = (tid < d) ? M.m0[tid] : 0.0;
    } else {
      const double* bt = M.b;
      if (P.Ft) {  // per-step dynamics: F_t replaces F in LDS
        team_sync();
        lds_load_mat<D>(sF, P.Ft + (int64_t)t * d * d, d);
        bt = P.bt + (int64_t)t * d;
      }
      rm_load<D>(Pp, M.Q, d, d);  // issued early: its latency overlaps F C
      rm_stage<D>(Cc, B1);
      // below D = 64 F C and T = F A are formed together; at D = 64 the
      // register file cannot hold both through the next product
      constexpr bool PAIR = (D < 64);
      if (first || !PAIR) {
        team_sync();
        gemm<D, false, false, false, U>(R1, sF, B1);  // F C
      } else {
        rm_stage<D>(A, B3);
        team_sync();
        gemm2<D, false, false, U>(R1, T, sF, B1, B3);  // F C and T = F A
      }
      team_sync();
      rm_stage<D>(R1, B1);
      team_sync();
      gemm<D, false, true, true, U>(Pp, B1, sF);  // Q + (F C) F'
      matvec<D, false>(vmu, sF, vb);
      if (tid < d && bt) vmu[tid] += bt[tid];
      if (!first && !PAIR) {
        rm_stage<D>(A, B1);
        team_sync();
        gemm<D, false, false, false, U>(T, sF, B1);  // T = F A
      }
      team_sync();
    }
    if constexpr (OBS == OBS_DIAG) {
      // diagonal Omega_t: with S = Pp + Omega, I - Pp S^{-1} = Omega S^{-1}, so
      // C = Omega S^{-1} Pp, A = Omega S^{-1} T, b = omega - Omega S^{-1} w.
      const double* Om = P.Om + (int64_t)t * d;
      R2 = Pp;
      AKF_RM_FOR(D, q, r, i, j) if (i == j && i < d) R2.t[q][r] += Om[i];
      if (tid < D) {
        vom[tid] = (tid < d) ? Om[tid] : 0.0;
        vw[tid] = (tid < d) ? P.om[(int64_t)t * d + tid] - vmu[tid] : 0.0;
      }
      // Pp and T go to LDS before the inverse, so they hold no registers
      // across it (B1 = Pp, B3 = T, B2 = the inverse's scratch, then S^{-1})
      rm_stage<D>(Pp, B1);
      if (!first) rm_stage<D>(T, B3);
      double logdet;
      ok = spd_inv<D>(R2, d, B2, &logdet) && ok;  // R2 = S^{-1}
      rm_stage<D>(R2, B2);
      team_sync();
      // S^{-1} Pp and S^{-1} T formed together (not in the batched D = 64
      // fold, U = 4, whose register allocation spills more with the pair)
      constexpr bool PAIR2 = !(D == 64 && U < 8);
      if (first || !PAIR2)
        gemm<D, false, false, false, U>(Cc, B2, B1);  // S^{-1} Pp
      else
        gemm2<D, false, false, U>(Cc, R1, B2, B1, B3);  // S^{-1} Pp, S^{-1} T
      AKF_RM_FOR(D, q, r, i, j) Cc.t[q][r] *= vom[i];
      matvec<D, false>(vs, B2, vw);  // S^{-1} w (ends synchronised: B1 is free)
      ld_sum += logdet;
      if (tid < D) q_part += vw[tid] * vs[tid];
      if (!first) {
        if (!PAIR2) gemm<D, false, false, false, U>(R1, B2, B3);  // S^{-1} T
        rm_stage<D>(R1, B1);
        team_sync();
        // fully unrolled where the register budget still allows it
        gemm<D, true, false, true, (OBS == OBS_DIAG && D == 64) ? D / 4 : U>(J, B3, B1);  // J += T' S^{-1} T
        AKF_RM_FOR(D, q, r, i, j) A.t[q][r] = vom[i] * R1.t[q][r];
        matvec<D, true>(veta, B3, vs, veta);  // eta += T' S^{-1} w
      }
      if (tid < D) vb[tid] = (tid < d) ? P.om[(int64_t)t * d + tid] - vom[tid] * vs[tid] : 0.0;
      rm_symmetrise<D>(Cc, B2);
      continue;
    }
    // B1 <- Mo (Pp, or H Pp); R2 <- S; vw <- innovation
    rm_stage<D>(Pp, B1);
    if constexpr (GH) {
      team_sync();
      gemm<D, false, false, false, U>(R1, sH, B1);  // H Pp
      team_sync();
      rm_stage<D>(R1, B1);
      team_sync();
      gemm<D, false, true, false, U>(R2, B1, sH);  // H Pp H'
      rm_add_load<D>(R2, P.Ro, P.dyo, P.dyo);
      matvec<D, false>(vw, sH, vmu);
      team_sync();
      if (tid < D) vw[tid] = (tid < P.dyo) ? P.yo[(int64_t)t * P.dyo + tid] - vw[tid] : 0.0;
    } else {
      R2 = Pp;
      if (P.Omd) {
        rm_add_load<D>(R2, P.Omd, d, d);
      } else {
        const double* Om = P.Om + (int64_t)t * d;
        AKF_RM_FOR(D, q, r, i, j) if (i == j && i < d) R2.t[q][r] += Om[i];
      }
      if (tid < D) vw[tid] = (tid < d) ? P.om[(int64_t)t * d + tid] - vmu[tid] : 0.0;
    }
    double logdet;
    ok = spd_inv<D>(R2, dobs, B2, &logdet) && ok;  // R2 = S^{-1}
    rm_stage<D>(R2, B3);
    team_sync();
    gemm<D, false, false, false, U>(R1, B3, B1);  // S^{-1} Mo
    matvec<D, false>(vs, B3, vw);              // S^{-1} w
    ld_sum += logdet;
    if (tid < D) q_part += vw[tid] * vs[tid];
    team_sync();
    rm_stage<D>(R1, B2);
    team_sync();
    gemm<D, true, false, false, U>(Cc, B1, B2);  // Mo' S^{-1} Mo
    rm_rsub<D>(Cc, Pp);  // C = Pp - Mo' S^{-1} Mo
    matvec<D, true>(vb, B1, vs, vmu);  // b = mu + Mo' S^{-1} w
    if (!first) {
      team_sync();
      rm_stage<D>(T, B2);  // B2 <- Mt (T, or H T)
      if constexpr (GH) {
        team_sync();
        gemm<D, false, false, false, U>(R1, sH, B2);  // H T
        team_sync();
        rm_stage<D>(R1, B2);
      }
      team_sync();
      gemm<D, false, false, false, U>(R1, B3, B2);  // S^{-1} Mt
      team_sync();
      rm_stage<D>(R1, B3);
      team_sync();
      gemm<D, true, false, true, U>(J, B2, B3);   // J += Mt' S^{-1} Mt
      gemm<D, true, false, false, U>(A, B1, B3);  // Mo' S^{-1} Mt
      rm_rsub<D>(A, T);  // A = T - Mo' S^{-1} Mt
      matvec<D, true>(veta, B2, vs, veta);  // eta += Mt' S^{-1} w
    } else if (first) {
      rm_zero<D>(A);
    }
    rm_symmetrise<D>(Cc, B2);
  }
  if (!ok && tid == 0) flag_status(P.status, P.fail_bit);
  if (first) {
    rm_zero<D>(A);
    rm_zero<D>(J);
  }
  rm_symmetrise<D>(J, B1);
  double* out = P.elem + (int64_t)blk * ElemLayout<D>::SIZE;
  rm_store<D>(A, out + ElemLayout<D>::A, D, D);
  rm_store<D>(Cc, out + ElemLayout<D>::C, D, D);
  rm_store<D>(J, out + ElemLayout<D>::J, D, D);
  if (tid < D) {
    out[ElemLayout<D>::b + tid] = vb[tid];
    out[ElemLayout<D>::eta + tid] = veta[tid];
  }
  const double q = team_sum<D>(q_part, red);
  if (tid == 0) out[ElemLayout<D>::lc] = -0.5 * ((s1 - s0) * dobs * LOG2PI + ld_sum + q);
}

template <int D, int OBS, int U = 4>
__device__ __forceinline__ void filter_fold_body(const KModel& M, const FilterArgs& P, int item) {
  if (item == 0)
    filter_fold_impl<D, OBS, true, U>(M, P, item);
  else
    filter_fold_impl<D, OBS, false, U>(M, P, item);
}

template <int D, int OBS>
__global__ void __launch_bounds__(Cfg<D>::NT) k_filter_fold(KModel M, FilterArgs P) {
  // k-steps per unrolled GEMM iteration: the most that fits the register budget
  // without spills (the D = 64 diagonal fold holds 512 registers per lane)
  constexpr int U = (D < 64) ? D / 4 : (OBS == OBS_DIAG ? 8 : 4);
  if (gate_shut(M.gate)) return;
  filter_fold_body<D, OBS, U>(M, P, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Filter, phase 2 up-sweep: node k of a level = left (earlier) (x) right.
// With C_i = L L' (register Cholesky), W = I + L' J_j L (SPD, eigenvalues
// >= 1, inverted by Gauss-Jordan) and M = L W^{-1} L' = (I + C_i J_j)^{-1} C_i:
//   A   = A_j (A_i - M J_j A_i)
//   b   = A_j (b_i + M c) + b_j,             c = eta_j - J_j b_i
//   C   = A_j M A_j' + C_j
//   eta = A_i' (c - J_j M c) + eta_i
//   J   = A_i' J_j A_i - (J_j A_i)' M (J_j A_i) + J_i = Z' J_j A_i + J_i,
//         Z = A_i - M J_j A_i
//   lc  = lc_i + lc_j - log det W / 2 + b_i' (eta_j + c) / 2 + c' M c / 2
// (the filtering-element combine of App. A, "Prefix-sums and the parallel
// Kalman filter"; lc is the constant of the Gaussian integral over the shared
// state, with log det W = log det (I + C_i J_j)).
// ---------------------------------------------------------------------------
// SIDE 0 writes the whole element.  A node of a level that fits on the chip
// twice is combined by two workgroups, each forming M (the factorisations and
// their products) and then one side of the outputs: SIDE 1 the J side (J,
// eta, A: four products after M), SIDE 2 the C side (C, b and lc: two), so a
// level waits for the prefix and four products instead of eight.
template <int D, int U = 4, int G = D * D / Cfg<D>::NT, int SIDE = 0>
__device__ __forceinline__ void filter_combine(const KModel& M, const double* __restrict__ ei,
                                               const double* __restrict__ ej,
                                               double* __restrict__ out, int* status,
                                               int fail_bit) {
  using C = Cfg<D>;
  using EL = ElemLayout<D>;
  extern __shared__ double lds[];
  double* S0 = lds;
  double* S1 = S0 + C::MAT;
  double* S2 = S1 + C::MAT;
  double* S3 = S2 + C::MAT;
  double* vbi = S3 + C::MAT;
  double* vc = vbi + D;
  double* vw = vc + D;
  double* vk = vw + D;
  double* red = vk + D;
  const int tid = threadIdx.x, d = M.d;
  bool ok = true;
  double ld;
  RM<D> R1, R2, R3;
  rm_load<D>(R1, ei + EL::C, D, d);
  lds_load_pad<D, G>(S1, ej + EL::J);
  if (tid < D) vbi[tid] = ei[EL::b + tid];
  // the operands needed later are fetched now, so their HBM latency overlaps
  // the factorisations (no global stores precede the barriers until then)
  RM<D> Ai, Ji, Aj, Cj;
  rm_load<D>(Ai, ei + EL::A, D, D);
  rm_load<D>(Ji, ei + EL::J, D, D);
  rm_load<D>(Aj, ej + EL::A, D, D);
  rm_load<D>(Cj, ej + EL::C, D, D);
  ok = chol_reg<D>(R1, d, S3, &ld) && ok;  // R1 = L
  rm_stage<D>(R1, S0);                        // S0 = L
  team_sync();
  gemm<D, false, false, false, U>(R2, S1, S0);  // J_j L
  rm_stage<D>(R2, S2);
  team_sync();
  gemm<D, true, false, false, U>(R2, S0, S2);  // L' J_j L
  AKF_RM_FOR(D, q, r, i, j) if (i == j && i < d) R2.t[q][r] += 1.0;
  ok = spd_inv<D>(R2, d, S3, &ld) && ok;  // W^{-1}
  const double ldW = ld;
  rm_stage<D>(R2, S2);
  team_sync();
  gemm<D, false, false, false, U>(R3, S0, S2);  // L W^{-1}
  rm_stage<D>(R3, S3);
  team_sync();
  gemm<D, false, true, false, U>(R2, S3, S0);  // M = L W^{-1} L'
  matvec<D, false>(vc, S1, vbi);            // J_j b_i
  team_sync();
  rm_stage<D>(R2, S2);  // S2 = M
  if (tid < D) vc[tid] = ej[EL::eta + tid] - vc[tid];
  team_sync();
  matvec<D, false>(vw, S2, vc);     // w = M c
  const double lc = ei[EL::lc] + ej[EL::lc] - 0.5 * ldW +
                    0.5 * team_sum<D>(tid < D ? vbi[tid] * (ej[EL::eta + tid] + vc[tid]) +
                                                    vc[tid] * vw[tid]
                                              : 0.0,
                                      red);
  if constexpr (SIDE != 2) {
    rm_stage<D>(Ai, S0);  // S0 = A_i
    team_sync();
    matvec<D, false>(vk, S1, vw);              // J_j w
    gemm<D, false, false, false, U>(R1, S1, S0);  // P = J_j A_i
    rm_stage<D>(R1, S3);                       // S3 = P
    team_sync();
    if (tid < D) vk[tid] = vc[tid] - vk[tid];  // c - J_j M c
    gemm<D, false, false, false, U>(R2, S2, S3);  // M P
    R3 = Ai;
    rm_axpy<D>(R3, -1.0, R2);  // Z1 = A_i - M P
    team_sync();
    matvec<D, true>(out + EL::eta, S0, vk, ei + EL::eta);  // eta = A_i' (c - J_j M c) + eta_i
    rm_stage<D>(R3, S1);  // S1 = Z1
    team_sync();
    gemm<D, true, false, false, U>(R1, S1, S3);  // J = Z1' P + J_i = A_i'P - P'MP + J_i
    rm_axpy<D>(R1, 1.0, Ji);
    rm_symmetrise<D>(R1, S3);  // ends synchronised
    rm_store<D>(R1, out + EL::J, D, D);
  }
  rm_stage<D>(Aj, S0);  // S0 = A_j
  if (tid < D) vw[tid] += vbi[tid];
  team_sync();
  // both sides: A_j Z1 and A_j M formed together (not in the batched D = 64
  // up-sweep, U = 4, whose register allocation spills more with the pair)
  constexpr bool PAIR = (SIDE == 0) && !(D == 64 && U < 8);
  if constexpr (PAIR) {
    gemm2<D, false, false, U>(R3, R2, S0, S1, S2);  // A = A_j Z1, A_j M
    rm_store<D>(R3, out + EL::A, D, D);
  } else if constexpr (SIDE != 2) {
    gemm<D, false, false, false, U>(R3, S0, S1);  // A = A_j Z1
    rm_store<D>(R3, out + EL::A, D, D);
  }
  if constexpr (SIDE != 1) {
    if constexpr (!PAIR) gemm<D, false, false, false, U>(R2, S0, S2);  // A_j M
    matvec<D, false>(vc, S0, vw);              // A_j (b_i + M c)
    rm_stage<D>(R2, S3);
    team_sync();
    gemm<D, false, true, false, U>(R3, S3, S0);  // A_j M A_j'
    rm_axpy<D>(R3, 1.0, Cj);
    if (tid < D) out[EL::b + tid] = vc[tid] + ej[EL::b + tid];
    if (tid == 0) out[EL::lc] = lc;
    rm_symmetrise<D>(R3, S1);
    rm_store<D>(R3, out + EL::C, D, D);
  }
  if (!ok && tid == 0) flag_status(status, fail_bit);
}

template <int D, int U = 4, int G = D * D / Cfg<D>::NT>
__device__ __forceinline__ void filter_up_body(const KModel& M, const TreeArgs& T, int item) {
  using EL = ElemLayout<D>;
  const int k = item, tid = threadIdx.x;
  const double* ei = T.src + (int64_t)(2 * k) * EL::SIZE;
  double* out = T.dst + (int64_t)k * EL::SIZE;
  if (2 * k + 1 >= T.n_src) {
    if constexpr (G > 0) {
      team_copy<Cfg<D>::NT>(out, ei, EL::SIZE);
    } else {
      for (int e = tid; e < EL::SIZE; e += Cfg<D>::NT) out[e] = ei[e];
    }
    return;
  }
  filter_combine<D, U, G>(M, ei, ei + EL::SIZE, out, T.status, T.fail_bit);
}

// One node per two workgroups (see filter_combine's SIDE); a left child
// without a partner is copied by the first of them.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_filter_up_split(KModel M, TreeArgs T) {
  if (gate_shut(M.gate)) return;
  using EL = ElemLayout<D>;
  const int k = blockIdx.x >> 1, side = blockIdx.x & 1;
  const double* ei = T.src + (int64_t)(2 * k) * EL::SIZE;
  double* out = T.dst + (int64_t)k * EL::SIZE;
  if (2 * k + 1 >= T.n_src) {
    if (side == 0) team_copy<Cfg<D>::NT>(out, ei, EL::SIZE);
    return;
  }
  if (side == 0)
    filter_combine<D, D / 4, D * D / Cfg<D>::NT, 1>(M, ei, ei + EL::SIZE, out, T.status,
                                                      T.fail_bit);
  else
    filter_combine<D, D / 4, D * D / Cfg<D>::NT, 2>(M, ei, ei + EL::SIZE, out, T.status,
                                                      T.fail_bit);
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_filter_up(KModel M, TreeArgs T) {
  filter_up_body<D, D / 4>(M, T, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Filter, phase 2 down-sweep: the prefix entering node k of a level is known
// (pre_src, as a filtering moment pair (m, P), or the identity for the left
// spine).  Its children: left gets the same prefix, right gets
// prefix (x) element(left child) (moment_combine).  With the identity prefix
// the result is the left child's (b, C) (its A = 0).
// ---------------------------------------------------------------------------
// Moment pair (m, P) (x) element el -> (m', P'), written to mout / Pout:
// with P = L L', W = I + L' J L and M = L W^{-1} L' = (P^{-1} + J)^{-1},
//   m' = A (m + M (eta - J m)) + b,   P' = A M A' + C,
// and, when lcout is given, the normaliser as in filter_combine with b_i = m.
template <int D, int U = 4>
__device__ __forceinline__ void moment_combine(const KModel& M, const double* Pin,
                                               const double* min_, const double* el,
                                               double* Pout, double* mout, int* status,
                                               int fail_bit, const double* lcin = nullptr,
                                               double* lcout = nullptr) {
  using C = Cfg<D>;
  using EL = ElemLayout<D>;
  extern __shared__ double lds[];
  double* S0 = lds;
  double* S1 = S0 + C::MAT;
  double* S2 = S1 + C::MAT;
  double* S3 = S2 + C::MAT;
  double* vm = S3 + C::MAT;
  double* vc = vm + D;
  double* vz = vc + D;
  double* vw = vz + D;
  double* red = vw + D;
  const int tid = threadIdx.x, d = M.d;
  bool ok = true;
  double ld;
  RM<D> R1, R2, Ae, Ce;
  rm_load<D>(R1, Pin, D, d);
  lds_load_pad<D>(S1, el + EL::J);
  if (tid < D) vm[tid] = min_[tid];
  rm_load<D>(Ae, el + EL::A, D, D);  // needed after the factorisations
  rm_load<D>(Ce, el + EL::C, D, D);
  ok = chol_reg<D>(R1, d, S3, &ld) && ok;  // R1 = L
  rm_stage<D>(R1, S0);
  team_sync();
  gemm<D, false, false, false, U>(R2, S1, S0);  // J L
  rm_stage<D>(R2, S2);
  team_sync();
  gemm<D, true, false, false, U>(R2, S0, S2);  // L' J L
  AKF_RM_FOR(D, q, r, i, j) if (i == j && i < d) R2.t[q][r] += 1.0;
  ok = spd_inv<D>(R2, d, S3, &ld) && ok;  // W^{-1}
  const double ldW = ld;
  rm_stage<D>(R2, S2);
  team_sync();
  gemm<D, false, false, false, U>(R1, S0, S2);  // L W^{-1}
  rm_stage<D>(R1, S3);
  team_sync();
  gemm<D, false, true, false, U>(R2, S3, S0);  // M
  matvec<D, false>(vc, S1, vm);             // J m
  team_sync();
  rm_stage<D>(R2, S2);  // S2 = M
  if (tid < D) vc[tid] = el[EL::eta + tid] - vc[tid];
  rm_stage<D>(Ae, S3);  // S3 = A
  team_sync();
  matvec<D, false>(vw, S2, vc);              // M (eta - J m)
  if (lcout) {
    const double q = team_sum<D>(
        tid < D ? vm[tid] * (el[EL::eta + tid] + vc[tid]) + vc[tid] * vw[tid] : 0.0, red);
    if (tid == 0) *lcout = *lcin + el[EL::lc] - 0.5 * ldW + 0.5 * q;
  }
  gemm<D, false, false, false, U>(R1, S3, S2);  // A M
  rm_stage<D>(R1, S0);
  team_sync();
  if (tid < D) vw[tid] += vm[tid];
  gemm<D, false, true, false, U>(R2, S0, S3);  // A M A'
  rm_axpy<D>(R2, 1.0, Ce);
  team_sync();
  matvec<D, false>(vz, S3, vw);
  if (tid < D) mout[tid] = vz[tid] + el[EL::b + tid];
  rm_symmetrise<D>(R2, S1);
  rm_store<D>(R2, Pout, D, D);
  if (!ok && tid == 0) flag_status(status, fail_bit);
}


template <int D, int U = 4>
__device__ __forceinline__ void filter_down_body(const KModel& M, const TreeArgs& T, int item) {
  using C = Cfg<D>;
  using EL = ElemLayout<D>;
  using PL = PrefLayout<D>;
  const int k = item, tid = threadIdx.x;
  const double* pin = T.pre_src + (int64_t)k * PL::SIZE;
  const bool ident = pin[PL::flag] != 0.0;
  // left child: same prefix
  double* pl = T.pre_dst + (int64_t)(2 * k) * PL::SIZE;
  team_copy<C::NT>(pl, pin, PL::SIZE);
  if (2 * k + 1 >= T.n_dst) return;
  double* pr = T.pre_dst + (int64_t)(2 * k + 1) * PL::SIZE;
  const double* el = T.src + (int64_t)(2 * k) * EL::SIZE;  // left child's element
  if (ident) {
    team_copy<C::NT>(pr + PL::P, el + EL::C, D * D);
    if (tid < D) pr[PL::m + tid] = el[EL::b + tid];
    if (tid == 0) pr[PL::flag] = 0.0;
    return;
  }
  moment_combine<D, U>(M, pin + PL::P, pin + PL::m, el, pr + PL::P, pr + PL::m, T.status,
                    T.fail_bit);
  if (tid == 0) pr[PL::flag] = 0.0;
}

// Hillis-Steele scan level: element k >= s becomes src[k - s] (x) src[k].  When
// k < 2s the left operand covers block 0, so it is a filtering moment pair
// (A = 0, J = 0): the combine reduces to the moment update and the result is
// again a moment pair.
template <int D, int U = 4>
__device__ __forceinline__ void filter_hs_body(const KModel& M, const HsArgs& H, int k) {
  using EL = ElemLayout<D>;
  const int tid = threadIdx.x;
  const double* ej = H.src + (int64_t)k * EL::SIZE;
  double* out = H.dst + (int64_t)k * EL::SIZE;
  if (k < H.s) {
    team_copy<Cfg<D>::NT>(out, ej, EL::SIZE);
    return;
  }
  const double* ei = H.src + (int64_t)(k - H.s) * EL::SIZE;
  if (k < 2 * H.s) {
    moment_combine<D, U>(M, ei + EL::C, ei + EL::b, ej, out + EL::C, out + EL::b, H.status,
                      H.fail_bit, ei + EL::lc, out + EL::lc);
    for (int e = tid; e < D * D; e += Cfg<D>::NT) {
      out[EL::A + e] = 0.0;
      out[EL::J + e] = 0.0;
    }
    if (tid < D) out[EL::eta + tid] = 0.0;
  } else {
    filter_combine<D, U>(M, ei, ej, out, H.status, H.fail_bit);
  }
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_filter_hs(KModel M, HsArgs H) {
  if (gate_shut(M.gate)) return;
  filter_hs_body<D, D / 4>(M, H, blockIdx.x);
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_filter_down(KModel M, TreeArgs T) {
  filter_down_body<D, D / 4>(M, T, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Filter, phase 3: each block re-runs its steps from the prefix entering it
// (sequential Kalman filter, App. A "Kalman filter"), with the predictive-
// form likelihood term ell_t = log N(omega_t; m^p_t, P^p_t + Omega_t).
// Writes m^f_t, P^f_t (when requested) and ell_t.
// ---------------------------------------------------------------------------
template <int D, int OBS, int U = 4>
__device__ __forceinline__ void filter_final_body(const KModel& M, const FilterArgs& P, int item) {
  using C = Cfg<D>;
  using PL = PrefLayout<D>;
  constexpr bool GH = (OBS == OBS_GH);
  static_assert(!GH || D <= 32, "general observation matrices need D <= 32");
  extern __shared__ double lds[];
  double* sF = lds;
  double* B1 = sF + C::MAT;
  double* B2 = B1 + C::MAT;
  double* B3 = B2 + C::MAT;
  double* sH = B3 + C::MAT;  // GH only
  double* vm = sH + (GH ? C::MAT : 0);
  double* vmp = vm + D;
  double* vw = vmp + D;
  double* vs = vw + D;
  double* vom = vs + D;  // diagonal Omega_t
  double* red = vom + D;
  const int blk = item, tid = threadIdx.x, d = M.d;
  const int s0 = blk * P.B, s1 = min(M.N, s0 + P.B);
  if (!P.Ft) lds_load_mat<D>(sF, M.F, d);
  if (GH) lds_load_rect<D>(sH, P.Ho, P.dyo, d);
  const int dobs = GH ? P.dyo : d;
  RM<D> Pm, Pp, T, R2;
  if (s0 > 0) {
    if (P.pre_elem) {
      const double* pin = P.pre_elem + (int64_t)(blk - 1) * ElemLayout<D>::SIZE;
      rm_load<D>(Pm, pin + ElemLayout<D>::C, D, D);
      if (tid < D) vm[tid] = pin[ElemLayout<D>::b + tid];
    } else {
      const double* pin = P.pre + (int64_t)blk * PL::SIZE;
      rm_load<D>(Pm, pin + PL::P, D, D);
      if (tid < D) vm[tid] = pin[PL::m + tid];
    }
  }
  team_sync();
  bool ok = true;
  for (int t = s0; t < s1; ++t) {
    if (t == 0) {
      rm_load<D>(Pp, M.P0, d, d);
      if (tid < D) vmp[tid] = (tid < d) ? M.m0[tid] : 0.0;
    } else {
      const double* bt = M.b;
      if (P.Ft) {  // per-step dynamics: F_t replaces F in LDS
        team_sync();
        lds_load_mat<D>(sF, P.Ft + (int64_t)t * d * d, d);
        bt = P.bt + (int64_t)t * d;
      }
      rm_load<D>(Pp, M.Q, d, d);  // issued early: its latency overlaps F P
      rm_stage<D>(Pm, B1);
      team_sync();
      gemm<D, false, false, false, U>(T, sF, B1);
      team_sync();
      rm_stage<D>(T, B1);
      team_sync();
      gemm<D, false, true, true, U>(Pp, B1, sF);  // Q + (F P) F'
      matvec<D, false>(vmp, sF, vm);
      team_sync();
      if (tid < d && bt) vmp[tid] += bt[tid];
      team_sync();
    }
    if constexpr (OBS == OBS_DIAG) {
      // diagonal Omega_t: P^f = Omega S^{-1} Pp, m^f = omega - Omega S^{-1} w
      const double* Om = P.Om + (int64_t)t * d;
      R2 = Pp;
      AKF_RM_FOR(D, q, r, i, j) if (i == j && i < d) R2.t[q][r] += Om[i];
      if (tid < D) {
        vom[tid] = (tid < d) ? Om[tid] : 0.0;
        vw[tid] = (tid < d) ? P.om[(int64_t)t * d + tid] - vmp[tid] : 0.0;
      }
      double logdet;
      ok = spd_inv<D>(R2, d, B2, &logdet) && ok;
      if (P.Sinv) {
        rm_store_t<D>(R2, P.Sinv + (int64_t)t * D * D, D);
        if (tid == 0) P.ldS[t] = logdet;
      }
      rm_stage<D>(R2, B3);
      rm_stage<D>(Pp, B1);
      team_sync();
      gemm<D, false, false, false, U>(Pm, B3, B1);  // S^{-1} Pp
      matvec<D, false>(vs, B3, vw);
      AKF_RM_FOR(D, q, r, i, j) Pm.t[q][r] *= vom[i];
      const double rr = team_sum<D>(tid < D ? vw[tid] * vs[tid] : 0.0, red);
      if (tid < D) vm[tid] = (tid < d) ? P.om[(int64_t)t * d + tid] - vom[tid] * vs[tid] : 0.0;
      if (tid == 0) P.ell[t] = -0.5 * (d * LOG2PI + logdet + rr);
      rm_symmetrise<D>(Pm, B2);
      if (P.mf) {
        if (tid < d) P.mf[(int64_t)t * P.ldm + tid] = vm[tid];
        rm_store<D>(Pm, P.Pf + (int64_t)t * P.ldm * P.ldm, P.ldm, d);
      }
      continue;
    }
    rm_stage<D>(Pp, B1);
    if constexpr (GH) {
      team_sync();
      gemm<D, false, false, false, U>(T, sH, B1);  // H Pp
      team_sync();
      rm_stage<D>(T, B1);
      team_sync();
      gemm<D, false, true, false, U>(R2, B1, sH);
      rm_add_load<D>(R2, P.Ro, P.dyo, P.dyo);
      matvec<D, false>(vw, sH, vmp);
      team_sync();
      if (tid < D) vw[tid] = (tid < P.dyo) ? P.yo[(int64_t)t * P.dyo + tid] - vw[tid] : 0.0;
    } else {
      R2 = Pp;
      if (P.Omd) {
        rm_add_load<D>(R2, P.Omd, d, d);
      } else {
        const double* Om = P.Om + (int64_t)t * d;
        AKF_RM_FOR(D, q, r, i, j) if (i == j && i < d) R2.t[q][r] += Om[i];
      }
      if (tid < D) vw[tid] = (tid < d) ? P.om[(int64_t)t * d + tid] - vmp[tid] : 0.0;
    }
    double logdet;
    ok = spd_inv<D>(R2, dobs, B2, &logdet) && ok;
    rm_stage<D>(R2, B3);
    team_sync();
    gemm<D, false, false, false, U>(T, B3, B1);  // S^{-1} Mo
    matvec<D, false>(vs, B3, vw);
    team_sync();
    rm_stage<D>(T, B2);
    const double rr = team_sum<D>(tid < D ? vw[tid] * vs[tid] : 0.0, red);
    gemm<D, true, false, false, U>(Pm, B1, B2);  // Mo' S^{-1} Mo
    rm_rsub<D>(Pm, Pp);  // P^f = Pp - Mo' S^{-1} Mo
    matvec<D, true>(vm, B1, vs, vmp);  // m^f = m^p + Mo' S^{-1} w
    if (tid == 0) P.ell[t] = -0.5 * (dobs * LOG2PI + logdet + rr);
    rm_symmetrise<D>(Pm, B2);
    if (P.mf) {
      if (tid < d) P.mf[(int64_t)t * P.ldm + tid] = vm[tid];
      rm_store<D>(Pm, P.Pf + (int64_t)t * P.ldm * P.ldm, P.ldm, d);
    }
  }
  if (!ok && tid == 0) flag_status(P.status, P.fail_bit);
}

template <int D, int OBS>
__global__ void __launch_bounds__(Cfg<D>::NT) k_filter_final(KModel M, FilterArgs P) {
  if (gate_shut(M.gate)) return;
  filter_final_body<D, OBS, D / 4>(M, P, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Sampler, element build (eq. backward, Alg. "Parallel RTS sampler"), one team
// per t:  G = F P^f,  P^p = G F' + Q (inverted by Gauss-Jordan),
//   E_t = G' (P^p)^{-1} = P^f F' (P^p)^{-1},   L_t = P^f - E_t G,
//   g_t = m^f - E_t (F m^f + bias),            U_t = g_t + chol(L_t) xi_t.
// Terminal step: E = 0, U = m^f + chol(P^f) xi.
// ---------------------------------------------------------------------------
template <int D, int U = 4>
__device__ __forceinline__ void samp_build_body(const KModel& M, const SampArgs& S, int item) {
  // two LDS matrices (X, Y), so that two teams share a CU: both buffers serve
  // the inverse as scratch, and G = F P^f is formed again after it
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* X = lds;
  double* Y = X + C::MAT;
  double* vm = Y + C::MAT;
  double* vmp = vm + D;
  double* vg = vmp + D;
  double* vxi = vg + D;
  const int t = item, tid = threadIdx.x, d = M.d;
  RM<D> Pf, R1, R2;
  rm_load<D>(Pf, S.Pf + (int64_t)t * S.ldm * S.ldm, S.ldm, d);
  if (tid < D) {
    vm[tid] = (tid < d) ? S.mf[(int64_t)t * S.ldm + tid] : 0.0;
    vxi[tid] = (tid < d) ? S.xi_x[(int64_t)t * d + tid] : 0.0;
  }
  bool ok = true;
  double ld;
  if (t == M.N - 1) {
    ok = chol_reg<D>(Pf, d, X, &ld);
    if (S.Lc) rm_store_t<D>(Pf, S.Lc + (int64_t)t * D * D, D);
    rm_stage<D>(Pf, Y);
    team_sync();
    if (tid < D) {
      double s = vm[tid];
      for (int j = 0; j <= tid; ++j) s = fma(Y[tid * C::LD + j], vxi[j], s);
      S.U[(int64_t)t * D + tid] = s;
    }
    RM<D> Z;
    rm_zero<D>(Z);
    rm_store<D>(Z, S.E + (int64_t)t * D * D, D, D);
    if (S.Et) rm_store<D>(Z, S.Et + (int64_t)t * D * D, D, D);
  } else {
    rm_load<D>(R2, M.Q, d, d);  // issued early: its latency overlaps G = F P^f
    // the transition into step t + 1
    lds_load_mat<D>(X, S.Ft ? S.Ft + (int64_t)(t + 1) * d * d : M.F, d);  // X = F
    const double* bt = S.Ft ? S.bt + (int64_t)(t + 1) * d : M.b;
    rm_stage<D>(Pf, Y);
    team_sync();
    // at D = 64 the first two products fully unrolled: the register budget
    // allows it here (and the allocator then spills less than with U)
    gemm<D, false, false, false, (D == 64 ? D / 4 : U)>(R1, X, Y);  // G = F P^f
    team_sync();
    rm_stage<D>(R1, Y);  // Y = G
    team_sync();
    gemm<D, false, true, true, (D == 64 ? D / 4 : U)>(R2, Y, X);  // Q + G F'
    matvec<D, false>(vmp, X, vm);
    if (tid < d && bt) vmp[tid] += bt[tid];
    {
      const RM<D> Pp = R2;
      ok = spd_inv<D>(R2, d, X, &ld) && ok;  // (P^p)^{-1}
      inv_refine<D>(R2, Pp, d, X, Y);        // P^p inherits the conditioning of Q
    }
    // G again (cheaper than holding it in registers through the inverse)
    lds_load_mat<D>(X, S.Ft ? S.Ft + (int64_t)(t + 1) * d * d : M.F, d);  // X = F
    rm_stage<D>(Pf, Y);
    team_sync();
    gemm<D, false, false, false, U>(R1, X, Y);  // G = F P^f
    team_sync();
    rm_stage<D>(R2, X);  // X = (P^p)^{-1}
    rm_stage<D>(R1, Y);  // Y = G
    team_sync();
    gemm<D, true, false, false, U>(R1, Y, X);  // E = G' (P^p)^{-1}
    rm_store<D>(R1, S.E + (int64_t)t * D * D, D, D);
    if (S.Et) rm_store_t<D>(R1, S.Et + (int64_t)t * D * D, D);
    team_sync();
    rm_stage<D>(R1, X);  // X = E
    team_sync();
    gemm<D, false, false, false, U>(R2, X, Y);  // E G
    rm_rsub<D>(R2, Pf);                      // L_t = P^f - E G
    matvec<D, false>(vg, X, vmp);
    if (tid < D) vg[tid] = vm[tid] - vg[tid];  // g = m^f - E m^p
    rm_symmetrise<D>(R2, Y);
    ok = chol_reg<D>(R2, d, X, &ld) && ok;
    if (S.Lc) rm_store_t<D>(R2, S.Lc + (int64_t)t * D * D, D);
    rm_stage<D>(R2, Y);
    team_sync();
    if (tid < D) {
      double s = vg[tid];
      for (int j = 0; j <= tid; ++j) s = fma(Y[tid * C::LD + j], vxi[j], s);
      S.U[(int64_t)t * D + tid] = s;
    }
  }
  if (!ok && tid == 0) flag_status(S.status, ST_FWD_NOT_PD);
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT, 2) k_samp_build(KModel M, SampArgs S) {
  if (gate_shut(M.gate)) return;
  samp_build_body<D, (D == 64 ? 8 : D / 4)>(M, S, blockIdx.x);  // no more spills than U = 4
}

// Sampler, block fold: suffix aggregate (E~, U~) of a block, folding from its
// last step backwards: (E~, U~) <- (E_t E~, E_t U~ + U_t).
template <int D, int U = 4>
__device__ __forceinline__ void samp_fold_body(const KModel& M, const SampArgs& S, int item) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* vu = B2 + C::MAT;
  double* vn = vu + D;
  const int blk = item, tid = threadIdx.x;
  const int s0 = blk * S.B, s1 = min(M.N, s0 + S.B);
  RM<D> Et;
  rm_load<D>(Et, S.E + (int64_t)(s1 - 1) * D * D, D, D);
  if (tid < D) vu[tid] = S.U[(int64_t)(s1 - 1) * D + tid];
  // E of the next step is fetched into registers while this step's products
  // run, so the loop does not wait on HBM (each thread holds PER entries)
  constexpr int PER = D * D / C::NT;
  double pre[PER];
  auto fetch = [&](int t) {
#pragma unroll
    for (int m = 0; m < PER; ++m) pre[m] = S.E[(int64_t)t * D * D + tid + m * C::NT];
  };
  if (s1 - 2 >= s0) fetch(s1 - 2);
  for (int t = s1 - 2; t >= s0; --t) {
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = tid + m * C::NT;
      B1[(e / D) * C::LD + e % D] = pre[m];
    }
    rm_stage<D>(Et, B2);
    team_sync();
    if (t - 1 >= s0) fetch(t - 1);
    gemm<D, false, false, false, U>(Et, B1, B2);
    matvec<D, false>(vn, B1, vu);
    team_sync();
    if (tid < D) vu[tid] = vn[tid] + S.U[(int64_t)t * D + tid];
    team_sync();
  }
  double* out = S.agg + (int64_t)blk * SampLayout<D>::SIZE;
  rm_store<D>(Et, out + SampLayout<D>::E, D, D);
  if (tid < D) out[SampLayout<D>::U + tid] = vu[tid];
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_samp_fold(KModel M, SampArgs S) {
  if (gate_shut(M.gate)) return;
  samp_fold_body<D, D / 4>(M, S, blockIdx.x);
}

// Sampler tree up-sweep: node k = left (earlier) o right = (E_l E_r, E_l U_r + U_l).
template <int D>
__device__ __forceinline__ void samp_up_body(const KModel& M, const TreeArgs& T, int item) {
  using C = Cfg<D>;
  using SL = SampLayout<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* vu = B2 + C::MAT;
  double* vn = vu + D;
  const int k = item, tid = threadIdx.x;
  const double* el = T.src + (int64_t)(2 * k) * SL::SIZE;
  double* out = T.dst + (int64_t)k * SL::SIZE;
  if (2 * k + 1 >= T.n_src) {
    team_copy<C::NT>(out, el, SL::SIZE);
    return;
  }
  const double* er = el + SL::SIZE;
  lds_load_pad<D>(B1, el + SL::E);
  lds_load_pad<D>(B2, er + SL::E);
  if (tid < D) vu[tid] = er[SL::U + tid];
  team_sync();
  RM<D> R;
  gemm<D, false, false, false, D / 4>(R, B1, B2);
  matvec<D, false>(vn, B1, vu);
  rm_store<D>(R, out + SL::E, D, D);
  team_sync();
  if (tid < D) out[SL::U + tid] = vn[tid] + el[SL::U + tid];
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_samp_up(KModel M, TreeArgs T) {
  if (gate_shut(M.gate)) return;
  samp_up_body<D>(M, T, blockIdx.x);
}

// Sampler tree down-sweep: xin[node] is x* at the step just after the node's
// range.  Right child inherits it; left child gets E_r xin + U_r.
template <int D>
__device__ __forceinline__ void samp_down_body(const KModel& M, const TreeArgs& T, int item) {
  using SL = SampLayout<D>;
  const int k = item, tid = threadIdx.x;
  const double* xin = T.pre_src + (int64_t)k * D;
  double* xl = T.pre_dst + (int64_t)(2 * k) * D;
  const bool has_right = (2 * k + 1 < T.n_dst);
  if (!has_right) {
    if (tid < D) xl[tid] = xin[tid];
    return;
  }
  double* xr = T.pre_dst + (int64_t)(2 * k + 1) * D;
  const double* er = T.src + (int64_t)(2 * k + 1) * SL::SIZE;
  if (tid < D) {
    double s = er[SL::U + tid];
    for (int j = 0; j < D; ++j) s = fma(er[SL::E + tid * D + j], xin[j], s);
    xr[tid] = xin[tid];
    xl[tid] = s;
  }
}

template <int D>
__global__ void __launch_bounds__(64) k_samp_down(KModel M, TreeArgs T) {
  if (gate_shut(M.gate)) return;
  samp_down_body<D>(M, T, blockIdx.x);
}

// Sampler, block final: x*_t = E_t x*_{t+1} + U_t inside each block.
template <int D>
__device__ __forceinline__ void samp_final_body(const KModel& M, const SampArgs& S, int item) {
  __shared__ double vx[64];
  __shared__ double vn[64];
  const int blk = item, tid = threadIdx.x, d = M.d;
  const int s0 = blk * S.B, s1 = min(M.N, s0 + S.B);
  if (tid < D) vx[tid] = S.xin[(int64_t)blk * D + tid];
  __syncthreads();
  for (int t = s1 - 1; t >= s0; --t) {
    const double* Et = S.E + (int64_t)t * D * D;
    if (tid < D) {
      double s = S.U[(int64_t)t * D + tid];
      for (int j = 0; j < D; ++j) s = fma(Et[tid * D + j], vx[j], s);
      vn[tid] = s;
    }
    __syncthreads();
    if (tid < D) vx[tid] = vn[tid];
    if (tid < d) S.xs[(int64_t)t * d + tid] = vn[tid];
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(64) k_samp_final(KModel M, SampArgs S) {
  if (gate_shut(M.gate)) return;
  samp_final_body<D>(M, S, blockIdx.x);
}

// ---------------------------------------------------------------------------
// MH decision: log r = terms + [log h(x*) - log h(x)] + log Z(x) - log Z(x*);
// accept iff log U < log r and no status bit is set.  One team of 256.
// ---------------------------------------------------------------------------
__device__ double block_sum(const double* a, int n, double* red) {
  // four independent accumulators keep four loads in flight per thread
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  const int stride = blockDim.x;
  int i = threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
#pragma unroll
    for (int q = 0; q < 4; ++q) s4[q] += a[i + q * stride];
  }
  for (; i < n; i += stride) s4[0] += a[i];
  double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double tot = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) tot += red[i];
  __syncthreads();
  return tot;
}

__device__ __forceinline__ void mh_finalize_body(const KModel& M, const StepArgs& A,
                                                 const FinalArgs& F) {
  __shared__ double red[4];
  const int n_ell = F.n_ell > 0 ? F.n_ell : M.N;
  const double lzf = block_sum(A.ell, n_ell, red);
  const double lzr = F.lz_rev ? *F.lz_rev : block_sum(A.ell2, n_ell, red);
  const double terms = block_sum(A.part_terms, F.n_part_rev, red);
  const double lhx = block_sum(A.part_lh_x, F.n_part_fwd, red);
  const double lhs = block_sum(A.part_lh_xs, F.n_part_rev, red);
  const double dyn = F.part_dyn ? block_sum(F.part_dyn, F.n_part_dyn, red) : 0.0;
  if (threadIdx.x == 0) {
    int st = *A.status;
    // a failed forward proposal makes x* (and everything computed from it)
    // meaningless: report only the forward failure
    if (st & ST_FWD_NOT_PD) st = ST_FWD_NOT_PD;
    double lr = terms + (lhs - lhx) + (lzf - lzr) + dyn;
    if (st == 0 && !isfinite(lr)) st |= ST_NONFINITE;
    if (st != 0) lr = -INFINITY;
    const int acc = (st == 0) && (log(F.unif[0]) < lr);
    *A.accept_flag = acc;
    *A.status = st;
    if (F.log_ratio) *F.log_ratio = lr;
    if (F.accepted) *F.accepted = acc;
    if (F.logZ_fwd) *F.logZ_fwd = lzf;
    if (F.logZ_rev) *F.logZ_rev = lzr;
    if (F.status_out) *F.status_out = st;
  }
}

__global__ void __launch_bounds__(256) k_mh_finalize(KModel M, StepArgs A, FinalArgs F) {
  mh_finalize_body(M, A, F);
}

// One chain: the decision fused with the select.  Every workgroup forms the
// same sums in the same order, hence the same decision; workgroup 0 writes the
// outputs and clears the next step's status word; each workgroup writes its
// slice of x_out = accept ? x* : x.
__global__ void __launch_bounds__(256) k_mh_decide(KModel M, StepArgs A, FinalArgs F,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ x_out, int64_t n,
                                                   int64_t per_block) {
  __shared__ double red[4];
  __shared__ int sacc;
  const int n_ell = F.n_ell > 0 ? F.n_ell : M.N;
  const double lzf = block_sum(A.ell, n_ell, red);
  const double lzr = F.lz_rev ? *F.lz_rev : block_sum(A.ell2, n_ell, red);
  const double terms = block_sum(A.part_terms, F.n_part_rev, red);
  const double lhx = block_sum(A.part_lh_x, F.n_part_fwd, red);
  const double lhs = block_sum(A.part_lh_xs, F.n_part_rev, red);
  const double dyn = F.part_dyn ? block_sum(F.part_dyn, F.n_part_dyn, red) : 0.0;
  if (threadIdx.x == 0) {
    int st = *A.status;
    if (st & ST_FWD_NOT_PD) st = ST_FWD_NOT_PD;
    double lr = terms + (lhs - lhx) + (lzf - lzr) + dyn;
    if (st == 0 && !isfinite(lr)) st |= ST_NONFINITE;
    if (st != 0) lr = -INFINITY;
    const int acc = (st == 0) && (log(F.unif[0]) < lr);
    sacc = acc;
    if (blockIdx.x == 0) {
      *A.accept_flag = acc;  // for callers that read the decision back
      if (F.log_ratio) *F.log_ratio = lr;
      if (F.accepted) *F.accepted = acc;
      if (F.logZ_fwd) *F.logZ_fwd = lzf;
      if (F.logZ_rev) *F.logZ_rev = lzr;
      if (F.status_out) *F.status_out = st;
      if (F.status_next) *F.status_next = 0;
    }
  }
  __syncthreads();
  const bool acc = sacc != 0;
  const int64_t i0 = (int64_t)blockIdx.x * per_block;
  const int64_t i1 = i0 + per_block < n ? i0 + per_block : n;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) x_out[i] = acc ? A.xs[i] : x[i];
}

__device__ __forceinline__ void mh_select_body(int64_t n, const double* __restrict__ x,
                                               const double* __restrict__ xs,
                                               double* __restrict__ x_out,
                                               const int* __restrict__ accept_flag, int item) {
  const int64_t i = (int64_t)item * blockDim.x + threadIdx.x;
  if (i < n) x_out[i] = (*accept_flag) ? xs[i] : x[i];
}

__global__ void __launch_bounds__(256) k_mh_select(int64_t n, const double* __restrict__ x,
                                                   const double* __restrict__ xs,
                                                   double* __restrict__ x_out,
                                                   const int* __restrict__ accept_flag) {
  mh_select_body(n, x, xs, x_out, accept_flag, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Host-side launch helpers (templated on D), used by akf_capi.cpp
// ---------------------------------------------------------------------------
template <int D>
size_t lds_bytes_filter(bool gh = false) {
  return (size_t)((gh ? 5 : 4) * Cfg<D>::MAT + 12 * D + 16) * sizeof(double);
}
// the sampler element build: two matrices and four vectors (two teams per CU)
template <int D>
size_t lds_bytes_samp_build() {
  return (size_t)(2 * Cfg<D>::MAT + 4 * D) * sizeof(double);
}
template <int D>
size_t lds_bytes_samp2() {
  return (size_t)(2 * Cfg<D>::MAT + 2 * D) * sizeof(double);
}

template <int D, int OBS>
hipError_t launch_filter(const KModel& M, FilterArgs P, TreeArgs* lv_up, TreeArgs* lv_down,
                         int n_levels, hipStream_t st) {
  const size_t lds = lds_bytes_filter<D>(OBS == OBS_GH);
  const int nb = (M.N + P.B - 1) / P.B;
  timing_mark(FAM_FILTER_FOLD, 1, st);
  hipLaunchKernelGGL((k_filter_fold<D, OBS>), dim3(nb), dim3(Cfg<D>::NT), lds, st, M, P);
  timing_mark(FAM_FILTER_FOLD, 0, st);
  for (int l = 0; l < n_levels; ++l) {
    timing_mark(FAM_FILTER_UP, 1, st);
    hipLaunchKernelGGL(k_filter_up<D>, dim3(lv_up[l].n_dst), dim3(Cfg<D>::NT), lds, st, M,
                       lv_up[l]);
    timing_mark(FAM_FILTER_UP, 0, st);
  }
  for (int l = n_levels - 1; l >= 0; --l) {
    timing_mark(FAM_FILTER_DOWN, 1, st);
    hipLaunchKernelGGL(k_filter_down<D>, dim3(lv_down[l].n_src), dim3(Cfg<D>::NT), lds, st, M,
                       lv_down[l]);
    timing_mark(FAM_FILTER_DOWN, 0, st);
  }
  timing_mark(FAM_FILTER_FINAL, 1, st);
  hipLaunchKernelGGL((k_filter_final<D, OBS>), dim3(nb), dim3(Cfg<D>::NT), lds, st, M, P);
  timing_mark(FAM_FILTER_FINAL, 0, st);
  return hipGetLastError();
}

template <int D, int OBS>
hipError_t launch_filter_scan(const KModel& M, FilterArgs P, const HsArgs* lv, int n_levels,
                              hipStream_t st) {
  const size_t lds = lds_bytes_filter<D>(OBS == OBS_GH);
  const int nb = (M.N + P.B - 1) / P.B;
  timing_mark(FAM_FILTER_FOLD, 1, st);
  hipLaunchKernelGGL((k_filter_fold<D, OBS>), dim3(nb), dim3(Cfg<D>::NT), lds, st, M, P);
  timing_mark(FAM_FILTER_FOLD, 0, st);
  for (int l = 0; l < n_levels; ++l) {
    timing_mark(FAM_FILTER_UP, 1, st);
    hipLaunchKernelGGL(k_filter_hs<D>, dim3(nb), dim3(Cfg<D>::NT), lds, st, M, lv[l]);
    timing_mark(FAM_FILTER_UP, 0, st);
  }
  timing_mark(FAM_FILTER_FINAL, 1, st);
  hipLaunchKernelGGL((k_filter_final<D, OBS>), dim3(nb), dim3(Cfg<D>::NT), lds, st, M, P);
  timing_mark(FAM_FILTER_FINAL, 0, st);
  return hipGetLastError();
}

// log Z only: fold, then the up-sweep reduction of the block elements; the
// root's normaliser is log p(omega_{0:N-1}).
// compute units of the current device (queried once per process)
static int compute_units() {
  static const int n = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    return v;
  }();
  return n;
}

template <int D, int OBS>
hipError_t launch_filter_logz(const KModel& M, FilterArgs P, const TreeArgs* up, int n_levels,
                              hipStream_t st) {
  const size_t lds = lds_bytes_filter<D>(OBS == OBS_GH);
  const int nb = (M.N + P.B - 1) / P.B;
  timing_mark(FAM_FILTER_FOLD, 1, st);
  hipLaunchKernelGGL((k_filter_fold<D, OBS>), dim3(nb), dim3(Cfg<D>::NT), lds, st, M, P);
  timing_mark(FAM_FILTER_FOLD, 0, st);
  // a level whose nodes fit on the chip twice runs each node on two workgroups
  const int n_cu = compute_units();
  for (int l = 0; l < n_levels; ++l) {
    timing_mark(FAM_FILTER_UP, 1, st);
    if (2 * up[l].n_dst <= n_cu)
      hipLaunchKernelGGL(k_filter_up_split<D>, dim3(2 * up[l].n_dst), dim3(Cfg<D>::NT), lds, st,
                         M, up[l]);
    else
      hipLaunchKernelGGL(k_filter_up<D>, dim3(up[l].n_dst), dim3(Cfg<D>::NT), lds, st, M,
                         up[l]);
    timing_mark(FAM_FILTER_UP, 0, st);
  }
  return hipGetLastError();
}

template <int D>
hipError_t launch_samp_scan(const KModel& M, SampArgs S, TreeArgs* lv_up, TreeArgs* lv_down,
                            int n_levels, hipStream_t st) {
  const int nb = (M.N + S.B - 1) / S.B;
  timing_mark(FAM_SAMP_FOLD, 1, st);
  hipLaunchKernelGGL(k_samp_fold<D>, dim3(nb), dim3(Cfg<D>::NT), lds_bytes_samp2<D>(), st, M, S);
  timing_mark(FAM_SAMP_FOLD, 0, st);
  for (int l = 0; l < n_levels; ++l) {
    timing_mark(FAM_SAMP_UP, 1, st);
    hipLaunchKernelGGL(k_samp_up<D>, dim3(lv_up[l].n_dst), dim3(Cfg<D>::NT), lds_bytes_samp2<D>(),
                       st, M, lv_up[l]);
    timing_mark(FAM_SAMP_UP, 0, st);
  }
  for (int l = n_levels - 1; l >= 0; --l) {
    timing_mark(FAM_SAMP_DOWN, 1, st);
    hipLaunchKernelGGL(k_samp_down<D>, dim3(lv_down[l].n_src), dim3(64), 0, st, M, lv_down[l]);
    timing_mark(FAM_SAMP_DOWN, 0, st);
  }
  timing_mark(FAM_SAMP_FINAL, 1, st);
  hipLaunchKernelGGL(k_samp_final<D>, dim3(nb), dim3(64), 0, st, M, S);
  timing_mark(FAM_SAMP_FINAL, 0, st);
  return hipGetLastError();
}

template <int D>
hipError_t launch_sampler(const KModel& M, SampArgs S, TreeArgs* lv_up, TreeArgs* lv_down,
                          int n_levels, hipStream_t st) {
  timing_mark(FAM_SAMP_BUILD, 1, st);
  hipLaunchKernelGGL(k_samp_build<D>, dim3(M.N), dim3(Cfg<D>::NT), lds_bytes_samp_build<D>(), st,
                     M, S);
  timing_mark(FAM_SAMP_BUILD, 0, st);
  return launch_samp_scan<D>(M, S, lv_up, lv_down, n_levels, st);
}

hipError_t launch_samp_scan_any(int D, const KModel& M, SampArgs S, TreeArgs* up, TreeArgs* down,
                                int nl, hipStream_t st) {
  switch (D) {
    case 16: return launch_samp_scan<16>(M, S, up, down, nl, st);
    case 32: return launch_samp_scan<32>(M, S, up, down, nl, st);
    case 64: return launch_samp_scan<64>(M, S, up, down, nl, st);
  }
  return hipErrorInvalidValue;
}

__global__ void k_zero(double* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

hipError_t launch_zero(double* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

template <int D>
hipError_t set_lds_limits() {
  hipError_t e;
  const int lf = (int)lds_bytes_filter<D>();
  const void* fns[] = {(const void*)k_filter_fold<D, OBS_DIAG>,
                       (const void*)k_filter_fold<D, OBS_DENSE>,
                       (const void*)k_filter_final<D, OBS_DIAG>,
                       (const void*)k_filter_final<D, OBS_DENSE>,
                       (const void*)k_filter_hs<D>};
  for (const void* f : fns)
    if ((e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lf)) != hipSuccess)
      return e;
  if ((e = hipFuncSetAttribute((const void*)k_filter_up<D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lf)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_filter_up_split<D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lf)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_filter_down<D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lf)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_samp_build<D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lf)) != hipSuccess)
    return e;
  return hipSuccess;
}

hipError_t launch_filter_scan_any(int D, const KModel& M, FilterArgs P, const HsArgs* lv,
                                  int nl, hipStream_t st) {
  if (P.Ho) {
    switch (D) {
      case 16: return launch_filter_scan<16, OBS_GH>(M, P, lv, nl, st);
      case 32: return launch_filter_scan<32, OBS_GH>(M, P, lv, nl, st);
    }
    return hipErrorInvalidValue;
  }
  if (P.Omd) {
    switch (D) {
      case 16: return launch_filter_scan<16, OBS_DENSE>(M, P, lv, nl, st);
      case 32: return launch_filter_scan<32, OBS_DENSE>(M, P, lv, nl, st);
      case 64: return launch_filter_scan<64, OBS_DENSE>(M, P, lv, nl, st);
    }
    return hipErrorInvalidValue;
  }
  switch (D) {
    case 16: return launch_filter_scan<16, OBS_DIAG>(M, P, lv, nl, st);
    case 32: return launch_filter_scan<32, OBS_DIAG>(M, P, lv, nl, st);
    case 64: return launch_filter_scan<64, OBS_DIAG>(M, P, lv, nl, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_filter_any(int D, const KModel& M, FilterArgs P, TreeArgs* up, TreeArgs* down,
                             int nl, hipStream_t st) {
  if (P.Ho) {
    switch (D) {
      case 16: return launch_filter<16, OBS_GH>(M, P, up, down, nl, st);
      case 32: return launch_filter<32, OBS_GH>(M, P, up, down, nl, st);
    }
    return hipErrorInvalidValue;
  }
  if (P.Omd) {
    switch (D) {
      case 16: return launch_filter<16, OBS_DENSE>(M, P, up, down, nl, st);
      case 32: return launch_filter<32, OBS_DENSE>(M, P, up, down, nl, st);
      case 64: return launch_filter<64, OBS_DENSE>(M, P, up, down, nl, st);
    }
    return hipErrorInvalidValue;
  }
  switch (D) {
    case 16: return launch_filter<16, OBS_DIAG>(M, P, up, down, nl, st);
    case 32: return launch_filter<32, OBS_DIAG>(M, P, up, down, nl, st);
    case 64: return launch_filter<64, OBS_DIAG>(M, P, up, down, nl, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_filter_logz_any(int D, const KModel& M, FilterArgs P, TreeArgs* up, int nl,
                                  hipStream_t st) {
  if (P.Ho) {
    switch (D) {
      case 16: return launch_filter_logz<16, OBS_GH>(M, P, up, nl, st);
      case 32: return launch_filter_logz<32, OBS_GH>(M, P, up, nl, st);
    }
    return hipErrorInvalidValue;
  }
  if (P.Omd) {
    switch (D) {
      case 16: return launch_filter_logz<16, OBS_DENSE>(M, P, up, nl, st);
      case 32: return launch_filter_logz<32, OBS_DENSE>(M, P, up, nl, st);
      case 64: return launch_filter_logz<64, OBS_DENSE>(M, P, up, nl, st);
    }
    return hipErrorInvalidValue;
  }
  switch (D) {
    case 16: return launch_filter_logz<16, OBS_DIAG>(M, P, up, nl, st);
    case 32: return launch_filter_logz<32, OBS_DIAG>(M, P, up, nl, st);
    case 64: return launch_filter_logz<64, OBS_DIAG>(M, P, up, nl, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sampler_any(int D, const KModel& M, SampArgs S, TreeArgs* up, TreeArgs* down,
                              int nl, hipStream_t st) {
  switch (D) {
    case 16: return launch_sampler<16>(M, S, up, down, nl, st);
    case 32: return launch_sampler<32>(M, S, up, down, nl, st);
    case 64: return launch_sampler<64>(M, S, up, down, nl, st);
  }
  return hipErrorInvalidValue;
}

hipError_t set_lds_limits_all() {
  hipError_t e;
  if ((e = set_lds_limits<16>()) != hipSuccess) return e;
  if ((e = set_lds_limits<32>()) != hipSuccess) return e;
  return set_lds_limits<64>();
}

hipError_t launch_lin(const KModel& M, StepArgs A, int rev, int* n_part, hipStream_t st) {
  timing_mark(FAM_LIN, 1, st);
  if (M.emit == EMIT_GAUSSIAN) {
    const int nblk = (M.N + kGaussStepsPerBlock - 1) / kGaussStepsPerBlock;
    *n_part = nblk;
    if (!rev) hipLaunchKernelGGL(k_gauss_prep, dim3(1), dim3(256), 0, st, M, A);
    hipLaunchKernelGGL(k_lin_gauss, dim3(nblk), dim3(64 * GL_WAVES), 0, st, M, A, rev);
  } else if (M.emit == EMIT_MVT) {
    const int nblk = (M.N + MVT_WAVES - 1) / MVT_WAVES;
    *n_part = nblk;
    hipLaunchKernelGGL(k_lin_mvt, dim3(nblk), dim3(64 * MVT_WAVES), 0, st, M, A, rev);
  } else {
    const int64_t n = (int64_t)M.N * M.d;
    const int nblk = (int)((n + 255) / 256);
    *n_part = nblk;
    if (!rev)
      hipLaunchKernelGGL(k_lin_fwd_diag, dim3(nblk), dim3(256), 0, st, M, A);
    else
      hipLaunchKernelGGL(k_lin_rev_diag, dim3(nblk), dim3(256), 0, st, M, A);
  }
  timing_mark(FAM_LIN, 0, st);
  return hipGetLastError();
}

// The branch of the next step of a run that reuses a rejected proposal's
// matrices: 0 = a fresh forward pass (after an acceptance or a failure),
// 1 = reuse whose trees are still to be formed (after a fresh pass), 2 = reuse
// with the trees formed.
__global__ void k_reuse_gate(const int* accept, const int* status, int* gate) {
  if (threadIdx.x == 0) {
    const int g = *gate;
    *gate = (*accept != 0 || *status != 0) ? 0 : (g == 0 ? 1 : 2);
  }
}

hipError_t launch_reuse_gate(const int* accept, const int* status, int* gate, hipStream_t st) {
  hipLaunchKernelGGL(k_reuse_gate, dim3(1), dim3(64), 0, st, accept, status, gate);
  return hipGetLastError();
}

hipError_t launch_step_init(int* status, double* root_flag, double* root_xin, int D,
                            hipStream_t st) {
  timing_mark(FAM_MH, 1, st);
  hipLaunchKernelGGL(k_step_init, dim3(1), dim3(64), 0, st, status, root_flag, root_xin, D);
  timing_mark(FAM_MH, 0, st);
  return hipGetLastError();
}

hipError_t launch_finalize(const KModel& M, StepArgs A, FinalArgs F, const double* x,
                           double* x_out, hipStream_t st) {
  const int64_t n = (int64_t)M.N * M.d;
  const int64_t per_block = 2048;
  const unsigned grid = (unsigned)((n + per_block - 1) / per_block);
  timing_mark(FAM_MH, 1, st);
  hipLaunchKernelGGL(k_mh_decide, dim3(grid), dim3(256), 0, st, M, A, F, x, x_out, n, per_block);
  timing_mark(FAM_MH, 0, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched chains.  Each persistent kernel walks a table of (chain, item) pairs
// (grid-stride); every pair runs the same body as the single-chain kernel with
// that chain's descriptor.  Per-step inputs (normals, uniform) and outputs are
// offset by the device step counter, so one captured step is replayed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ StepArgs step_args(const ChainDev& c, int step) {
  StepArgs A = c.A;
  A.xi_u = c.xi_base + (int64_t)step * c.xi_stride;
  return A;
}

__global__ void __launch_bounds__(64) kb_init(BatchLaunch L, int D) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const ChainDev& c = L.cd[L.items[w].c];
    if (threadIdx.x == 0) {
      *c.A.status = 0;
      *c.root_flag = 1.0;
    }
    if ((int)threadIdx.x < D) c.root_xin[threadIdx.x] = 0.0;
  }
}

__global__ void __launch_bounds__(256) kb_lin(BatchLaunch L, int rev, const int* step) {
  const int s = *step;
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    const StepArgs A = step_args(c, s);
    if (rev)
      lin_rev_diag_body(c.M, A, I.i);
    else
      lin_fwd_diag_body(c.M, A, I.i);
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT, D == 16 ? 3 : 1) kb_fold(BatchLaunch L, int rev) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    filter_fold_body<D, OBS_DIAG, (D < 64 ? D / 4 : 4)>(c.M, rev ? c.Fr : c.Ff, I.i);
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT, D == 16 ? 3 : D == 32 ? 2 : 1) kb_final(BatchLaunch L, int rev) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    filter_final_body<D, OBS_DIAG, D / 4>(c.M, rev ? c.Fr : c.Ff, I.i);
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) kb_up(BatchLaunch L, int level, int rev) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    TreeArgs T = c.fup[level - 1];
    T.fail_bit = rev ? ST_REV_NOT_PD : ST_FWD_NOT_PD;
    filter_up_body<D, (D < 64 ? D / 4 : 4), 0>(c.M, T, I.i);
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT, D == 16 ? 3 : 1) kb_down(BatchLaunch L, int level, int rev) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    TreeArgs T = c.fdown[level - 1];
    T.fail_bit = rev ? ST_REV_NOT_PD : ST_FWD_NOT_PD;
    filter_down_body<D, (D < 64 ? D / 4 : 4)>(c.M, T, I.i);
    __syncthreads();
  }
}

// two teams per SIMD where the persistent loop's registers still fit (D <= 32)
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT, D == 64 ? 1 : D == 16 ? 3 : 2) kb_sbuild(BatchLaunch L,
                                                                     const int* step) {
  const int s = *step;
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    SampArgs S = c.S;
    S.xi_x = c.xi_base + (int64_t)s * c.xi_stride + (int64_t)c.M.N * c.M.d;
    samp_build_body<D>(c.M, S, I.i);  // two teams per SIMD: the register budget keeps U = 4
    __syncthreads();
  }
}

// the same with one team per SIMD and the whole register file: no spills and
// fully unrolled products, half the teams (the autotuner times both layouts)
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT, 1) kb_sbuild1(BatchLaunch L, const int* step) {
  const int s = *step;
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    SampArgs S = c.S;
    S.xi_x = c.xi_base + (int64_t)s * c.xi_stride + (int64_t)c.M.N * c.M.d;
    samp_build_body<D, D / 4>(c.M, S, I.i);
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) kb_sfold(BatchLaunch L) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    samp_fold_body<D, D / 4>(c.M, c.S, I.i);
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) kb_sup(BatchLaunch L, int level) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    samp_up_body<D>(c.M, c.sup[level - 1], I.i);
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(64) kb_sdown(BatchLaunch L, int level) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    samp_down_body<D>(c.M, c.sdown[level - 1], I.i);
    __syncthreads();
  }
}

template <int D>
__global__ void __launch_bounds__(64) kb_sfinal(BatchLaunch L) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    samp_final_body<D>(c.M, c.S, I.i);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) kb_finalize(BatchLaunch L, const int* step) {
  const int s = *step;
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const ChainDev& c = L.cd[L.items[w].c];
    FinalArgs F = c.Fin;
    F.unif = c.unif_base + s;
    F.log_ratio = c.lr_base ? c.lr_base + s : nullptr;
    F.accepted = c.acc_base ? c.acc_base + s : nullptr;
    F.logZ_fwd = c.lzf_base ? c.lzf_base + s : nullptr;
    F.logZ_rev = c.lzr_base ? c.lzr_base + s : nullptr;
    F.status_out = c.st_base ? c.st_base + s : nullptr;
    mh_finalize_body(c.M, c.A, F);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) kb_select(BatchLaunch L) {
  for (int w = blockIdx.x; w < L.n_items; w += gridDim.x) {
    const Item I = L.items[w];
    const ChainDev& c = L.cd[I.c];
    mh_select_body((int64_t)c.M.N * c.M.d, c.x, c.A.xs, c.x, c.A.accept_flag, I.i);
  }
}

__global__ void k_step_advance(int* step, int reset) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step = reset ? 0 : *step + 1;
}

hipError_t launch_step_advance(int* step, int reset, hipStream_t st) {
  hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, st, step, reset);
  return hipGetLastError();
}

template <int D>
size_t batch_lds_bytes_t(int phase) {
  if (phase == BP_FOLD || phase == BP_UP || phase == BP_DOWN || phase == BP_FINAL)
    return lds_bytes_filter<D>();
  if (phase == BP_SBUILD || phase == BP_SBUILD1) return lds_bytes_samp_build<D>();
  if (phase == BP_SFOLD || phase == BP_SUP) return lds_bytes_samp2<D>();
  return 0;
}

size_t batch_lds_bytes(int D, int phase) {
  switch (D) {
    case 16: return batch_lds_bytes_t<16>(phase);
    case 32: return batch_lds_bytes_t<32>(phase);
    case 64: return batch_lds_bytes_t<64>(phase);
  }
  return 0;
}

// Workgroups of `kernel` that the chip holds at once: its occupancy per CU
// (registers and LDS) times the CU count.  A persistent phase launches no more
// than that, so every workgroup starts at once and none waits for a slot.
template <typename K>
int resident_grid(K kernel, int threads, size_t lds) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * std::max(1, compute_units());
}

// The cap of each team phase, queried once per kernel (batch_caps() queries
// them all when a plan is made, outside any graph capture).
template <int D>
int batch_cap(int phase) {
  constexpr int NT = Cfg<D>::NT;
  switch (phase) {
    case BP_FOLD: { static const int c = resident_grid(kb_fold<D>, NT, batch_lds_bytes(D, phase)); return c; }
    case BP_UP: { static const int c = resident_grid(kb_up<D>, NT, batch_lds_bytes(D, phase)); return c; }
    case BP_DOWN: { static const int c = resident_grid(kb_down<D>, NT, batch_lds_bytes(D, phase)); return c; }
    case BP_FINAL: { static const int c = resident_grid(kb_final<D>, NT, batch_lds_bytes(D, phase)); return c; }
    case BP_SBUILD: { static const int c = resident_grid(kb_sbuild<D>, NT, batch_lds_bytes(D, phase)); return c; }
    case BP_SBUILD1: {
      static const int c = D == 64 ? batch_cap<D>(BP_SBUILD)
                                   : resident_grid(kb_sbuild1<D>, NT, batch_lds_bytes(D, phase));
      return c;
    }
    case BP_SFOLD: { static const int c = resident_grid(kb_sfold<D>, NT, batch_lds_bytes(D, phase)); return c; }
    case BP_SUP: { static const int c = resident_grid(kb_sup<D>, NT, batch_lds_bytes(D, phase)); return c; }
    case BP_SDOWN: { static const int c = resident_grid(kb_sdown<D>, 64, 0); return c; }
    case BP_SFINAL: { static const int c = resident_grid(kb_sfinal<D>, 64, 0); return c; }
  }
  return 0;  // the other phases keep the plan's grid
}

void batch_caps(int D) {
  for (int ph = 0; ph <= BP_SBUILD1; ++ph) {
    switch (D) {
      case 16: batch_cap<16>(ph); break;
      case 32: batch_cap<32>(ph); break;
      case 64: batch_cap<64>(ph); break;
    }
  }
}

template <int D>
hipError_t launch_batch_phase_t(int phase, BatchLaunch L, int level, int rev, const int* step,
                                hipStream_t st) {
  if (L.n_items <= 0) return hipSuccess;
  if (phase >= BP_FOLD_LANE)
    return launch_lane_phase(phase, L, rev, step, st);
  const int cap = batch_cap<D>(phase);
  if (cap > 0) L.grid = std::min(L.n_items, cap);
  const dim3 g(L.grid), bt(Cfg<D>::NT), b64(64), b256(256);
  const size_t lds = batch_lds_bytes(D, phase);
  switch (phase) {
    case BP_INIT: hipLaunchKernelGGL(kb_init, g, b64, 0, st, L, D); break;
    case BP_LIN_FWD: hipLaunchKernelGGL(kb_lin, g, b256, 0, st, L, 0, step); break;
    case BP_LIN_REV: hipLaunchKernelGGL(kb_lin, g, b256, 0, st, L, 1, step); break;
    case BP_FOLD: hipLaunchKernelGGL(kb_fold<D>, g, bt, lds, st, L, rev); break;
    case BP_UP: hipLaunchKernelGGL(kb_up<D>, g, bt, lds, st, L, level, rev); break;
    case BP_DOWN: hipLaunchKernelGGL(kb_down<D>, g, bt, lds, st, L, level, rev); break;
    case BP_FINAL: hipLaunchKernelGGL(kb_final<D>, g, bt, lds, st, L, rev); break;
    case BP_SBUILD: hipLaunchKernelGGL(kb_sbuild<D>, g, bt, lds, st, L, step); break;
    case BP_SBUILD1:
      if constexpr (D == 64)
        hipLaunchKernelGGL(kb_sbuild<D>, g, bt, lds, st, L, step);  // one team per CU either way
      else
        hipLaunchKernelGGL(kb_sbuild1<D>, g, bt, lds, st, L, step);
      break;
    case BP_SFOLD: hipLaunchKernelGGL(kb_sfold<D>, g, bt, lds, st, L); break;
    case BP_SUP: hipLaunchKernelGGL(kb_sup<D>, g, bt, lds, st, L, level); break;
    case BP_SDOWN: hipLaunchKernelGGL(kb_sdown<D>, g, b64, 0, st, L, level); break;
    case BP_SFINAL: hipLaunchKernelGGL(kb_sfinal<D>, g, b64, 0, st, L); break;
    case BP_FINALIZE: hipLaunchKernelGGL(kb_finalize, g, b256, 0, st, L, step); break;
    case BP_SELECT: hipLaunchKernelGGL(kb_select, g, b256, 0, st, L); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_phase(int D, int phase, BatchLaunch L, int level, int rev,
                              const int* step, hipStream_t st) {
  switch (D) {
    case 16: return launch_batch_phase_t<16>(phase, L, level, rev, step, st);
    case 32: return launch_batch_phase_t<32>(phase, L, level, rev, step, st);
    case 64: return launch_batch_phase_t<64>(phase, L, level, rev, step, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace akf
