// akf_lane.hip -- batched chains with a state of at most four coordinates:
// one lane per item (a block of the filter fold, the re-scan, the sampler's
// block fold and final pass; a time step of the sampler element build), its
// matrices 4 x 4 in registers.
//
// Such chains belong to the 16-wide class (their element, moment and sampler
// arrays are padded to 16, and every other phase runs on 16-wide teams), but a
// 16 x 16 team spends a whole wave on a 4 x 4 problem.  Here a wave carries 64
// items at once with scalar FP64 arithmetic: the same recursions as the team
// bodies (filter fold and re-scan: App. A, "Prefix-sums and the parallel
// Kalman filter", with a diagonal Omega_t; sampler element: eq. backward, Alg.
// "Parallel RTS sampler"), and the same padded outputs (zeros beyond d; the
// element and E_t arrays keep the zero padding the batch plan gives them).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "akf_internal.h"

namespace akf {

namespace {

constexpr int K = kLaneMaxD;  // largest state dimension a lane handles
constexpr int DP = 16;  // padding of the arrays of the class these chains run in
constexpr double kLog2Pi = 1.8378770664093454835606594728112;

struct M4 {
  double a[K][K];
};

__device__ __forceinline__ void flag(int* st, int bit) { atomicOr(st, bit); }

__device__ __forceinline__ void m_zero(M4& m) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) m.a[i][j] = 0.0;
}

// entries i, j < d of a row-major matrix with leading dimension ld; zero beyond
__device__ __forceinline__ void m_load(M4& m, const double* __restrict__ g, int ld, int d) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) m.a[i][j] = (i < d && j < d) ? g[i * ld + j] : 0.0;
}

// entry (i, j) of the 4 x 4 corner, zero outside it (i, j compile-time after unrolling)
__device__ __forceinline__ double m_at(const M4& m, int i, int j) {
  return (i < K && j < K) ? m.a[i < K ? i : 0][j < K ? j : 0] : 0.0;
}

// the whole DP x DP block (row-major, ld DP), zero beyond the 4 x 4 corner;
// T: stored transposed
template <bool T = false>
__device__ __forceinline__ void m_store_pad(const M4& m, double* __restrict__ g) {
#pragma unroll
  for (int i = 0; i < DP; ++i)
#pragma unroll
    for (int j = 0; j < DP; ++j) g[i * DP + j] = T ? m_at(m, j, i) : m_at(m, i, j);
}

// the 4 x 4 corner of a DP x DP block (row-major, ld DP): the batch plan zeroes
// its workspace when it is made, and nothing but these kernels writes the
// arrays they fill, so the padding is already zero
__device__ __forceinline__ void m_store_corner(const M4& m, double* __restrict__ g) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) g[i * DP + j] = m.a[i][j];
}

// a K-vector written as DP entries, zero beyond d
__device__ __forceinline__ void v_store_pad(const double* v, int d, double* __restrict__ g) {
#pragma unroll
  for (int i = 0; i < DP; ++i) g[i] = (i < K && i < d) ? v[i < K ? i : 0] : 0.0;
}

// c = a b, c = a b', c = a' b
__device__ __forceinline__ void m_mul(M4& c, const M4& a, const M4& b) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) s = fma(a.a[i][k], b.a[k][j], s);
      c.a[i][j] = s;
    }
}
__device__ __forceinline__ void m_mul_nt(M4& c, const M4& a, const M4& b) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) s = fma(a.a[i][k], b.a[j][k], s);
      c.a[i][j] = s;
    }
}
__device__ __forceinline__ void m_mul_tn(M4& c, const M4& a, const M4& b) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) s = fma(a.a[k][i], b.a[k][j], s);
      c.a[i][j] = s;
    }
}

// y = a x, y = a' x
__device__ __forceinline__ void m_vec(double* y, const M4& a, const double* x) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) s = fma(a.a[i][k], x[k], s);
    y[i] = s;
  }
}
__device__ __forceinline__ void m_vec_t(double* y, const M4& a, const double* x) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) s = fma(a.a[k][i], x[k], s);
    y[i] = s;
  }
}

__device__ __forceinline__ void m_sym(M4& m) {
#pragma unroll
  for (int i = 0; i < K; ++i)
#pragma unroll
    for (int j = 0; j < i; ++j) {
      const double v = 0.5 * (m.a[i][j] + m.a[j][i]);
      m.a[i][j] = v;
      m.a[j][i] = v;
    }
}

// Lower Cholesky factor of the leading d x d block of an SPD matrix (zero
// elsewhere); false when a pivot is not positive.  *logdet = log det.
__device__ __forceinline__ bool m_chol(M4& l, const M4& s, int d, double* logdet) {
  bool ok = true;
  double ld = 0.0;
  m_zero(l);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < d) {
      double p = s.a[j][j];
#pragma unroll
      for (int k = 0; k < j; ++k) p = fma(-l.a[j][k], l.a[j][k], p);
      if (!(p > 0.0)) {
        ok = false;
        p = 1.0;
      }
      const double r = sqrt(p), ri = 1.0 / r;
      ld += log(p);
      l.a[j][j] = r;
#pragma unroll
      for (int i = j + 1; i < K; ++i) {
        if (i < d) {
          double v = s.a[i][j];
#pragma unroll
          for (int k = 0; k < j; ++k) v = fma(-l.a[i][k], l.a[j][k], v);
          l.a[i][j] = v * ri;
        }
      }
    }
  }
  *logdet = ld;
  return ok;
}

// Inverse of the leading d x d block of an SPD matrix through its Cholesky
// factor, S^{-1} = L^{-T} L^{-1} (zero beyond d).
__device__ __forceinline__ bool m_spd_inv(M4& x, const M4& s, int d, double* logdet) {
  M4 l, li;
  const bool ok = m_chol(l, s, d, logdet);
  m_zero(li);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < d) {
      li.a[j][j] = 1.0 / l.a[j][j];
#pragma unroll
      for (int i = j + 1; i < K; ++i) {
        if (i < d) {
          double v = 0.0;
#pragma unroll
          for (int k = j; k < i; ++k) v = fma(-l.a[i][k], li.a[k][j], v);
          li.a[i][j] = v / l.a[i][i];
        }
      }
    }
  }
  m_mul_tn(x, li, li);
  return ok;
}

// ---------------------------------------------------------------------------
// Filter fold of block `blk` (diagonal Omega_t): the recursion of the team
// fold, appending step t to the block element (A, b, C, eta, J):
//   Pp = F C F' + Q, T = F A, mu = F b + bias, S = Pp + Omega_t, w = omega_t - mu,
//   C <- Omega S^{-1} Pp, A <- Omega S^{-1} T, b <- omega - Omega S^{-1} w,
//   J <- J + T' S^{-1} T, eta <- eta + T' S^{-1} w,
// lc accumulating -(d log 2 pi + log det S + w' S^{-1} w) / 2 per step.
// ---------------------------------------------------------------------------
__device__ void lane_fold(const KModel& M, const FilterArgs& P, int blk) {
  using EL = ElemLayout<DP>;
  const int d = M.d;
  const int s0 = blk * P.B, s1 = min(M.N, s0 + P.B);
  const bool first = (blk == 0);
  M4 F, Q, A, C, J;
  m_load(F, M.F, d, d);
  m_load(Q, M.Q, d, d);
  double bias[K], b[K], eta[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    bias[i] = (i < d && M.b) ? M.b[i] : 0.0;
    b[i] = 0.0;
    eta[i] = 0.0;
  }
  m_zero(A);
#pragma unroll
  for (int i = 0; i < K; ++i)
    if (i < d) A.a[i][i] = 1.0;
  m_zero(C);
  m_zero(J);
  double ld_sum = 0.0, q = 0.0;
  bool ok = true;
  for (int t = s0; t < s1; ++t) {
    M4 Pp, T;
    double mu[K];
    if (t == 0) {
      m_load(Pp, M.P0, d, d);
#pragma unroll
      for (int i = 0; i < K; ++i) mu[i] = (i < d) ? M.m0[i] : 0.0;
    } else {
      M4 FC;
      m_mul(FC, F, C);
      m_mul_nt(Pp, FC, F);
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) Pp.a[i][j] += Q.a[i][j];
      m_vec(mu, F, b);
#pragma unroll
      for (int i = 0; i < K; ++i) mu[i] += bias[i];
      if (!first) m_mul(T, F, A);
    }
    const double* Om = P.Om + (int64_t)t * d;
    const double* om = P.om + (int64_t)t * d;
    double vom[K], w[K], vs[K];
    M4 S = Pp;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      vom[i] = (i < d) ? Om[i] : 0.0;
      w[i] = (i < d) ? om[i] - mu[i] : 0.0;
      S.a[i][i] += vom[i];
    }
    M4 Si, X;
    double logdet;
    ok = m_spd_inv(Si, S, d, &logdet) && ok;
    m_mul(X, Si, Pp);
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) C.a[i][j] = vom[i] * X.a[i][j];
    m_vec(vs, Si, w);
    ld_sum += logdet;
#pragma unroll
    for (int i = 0; i < K; ++i) q = fma(w[i], vs[i], q);
    if (!first) {
      M4 R1, TR;
      m_mul(R1, Si, T);
      m_mul_tn(TR, T, R1);
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) {
          J.a[i][j] += TR.a[i][j];
          A.a[i][j] = vom[i] * R1.a[i][j];
        }
      double tv[K];
      m_vec_t(tv, T, vs);
#pragma unroll
      for (int i = 0; i < K; ++i) eta[i] += tv[i];
    }
#pragma unroll
    for (int i = 0; i < K; ++i) b[i] = (i < d) ? om[i] - vom[i] * vs[i] : 0.0;
    m_sym(C);
  }
  if (!ok) flag(P.status, P.fail_bit);
  if (first) {
    m_zero(A);
    m_zero(J);
  }
  m_sym(J);
  double* out = P.elem + (int64_t)blk * EL::SIZE;
  m_store_corner(A, out + EL::A);
  m_store_corner(C, out + EL::C);
  m_store_corner(J, out + EL::J);
  v_store_pad(b, d, out + EL::b);
  v_store_pad(eta, d, out + EL::eta);
  out[EL::lc] = -0.5 * ((s1 - s0) * d * kLog2Pi + ld_sum + q);
}

// ---------------------------------------------------------------------------
// Re-scan of block `blk`: a sequential Kalman filter from the filtering
// moments entering the block, writing m^f_t, P^f_t and the predictive terms
// ell_t = -(d log 2 pi + log det S_t + w' S_t^{-1} w) / 2.
// ---------------------------------------------------------------------------
__device__ void lane_final(const KModel& M, const FilterArgs& P, int blk) {
  const int d = M.d;
  const int s0 = blk * P.B, s1 = min(M.N, s0 + P.B);
  M4 F, Q, Pm;
  m_load(F, M.F, d, d);
  m_load(Q, M.Q, d, d);
  double bias[K], m[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    bias[i] = (i < d && M.b) ? M.b[i] : 0.0;
    m[i] = 0.0;
  }
  m_zero(Pm);
  if (s0 > 0) {
    const double* pin;
    int op, om_;
    if (P.pre_elem) {
      pin = P.pre_elem + (int64_t)(blk - 1) * ElemLayout<DP>::SIZE;
      op = ElemLayout<DP>::C;
      om_ = ElemLayout<DP>::b;
    } else {
      pin = P.pre + (int64_t)blk * PrefLayout<DP>::SIZE;
      op = PrefLayout<DP>::P;
      om_ = PrefLayout<DP>::m;
    }
    m_load(Pm, pin + op, DP, d);
#pragma unroll
    for (int i = 0; i < K; ++i) m[i] = (i < d) ? pin[om_ + i] : 0.0;
  }
  bool ok = true;
  for (int t = s0; t < s1; ++t) {
    M4 Pp;
    double mp[K];
    if (t == 0) {
      m_load(Pp, M.P0, d, d);
#pragma unroll
      for (int i = 0; i < K; ++i) mp[i] = (i < d) ? M.m0[i] : 0.0;
    } else {
      M4 FP;
      m_mul(FP, F, Pm);
      m_mul_nt(Pp, FP, F);
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) Pp.a[i][j] += Q.a[i][j];
      m_vec(mp, F, m);
#pragma unroll
      for (int i = 0; i < K; ++i) mp[i] += bias[i];
    }
    const double* Om = P.Om + (int64_t)t * d;
    const double* om = P.om + (int64_t)t * d;
    double vom[K], w[K], vs[K];
    M4 S = Pp;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      vom[i] = (i < d) ? Om[i] : 0.0;
      w[i] = (i < d) ? om[i] - mp[i] : 0.0;
      S.a[i][i] += vom[i];
    }
    M4 Si, X;
    double logdet;
    ok = m_spd_inv(Si, S, d, &logdet) && ok;
    if (P.Sinv) {
      m_store_pad<true>(Si, P.Sinv + (int64_t)t * DP * DP);
      P.ldS[t] = logdet;
    }
    m_mul(X, Si, Pp);
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) Pm.a[i][j] = vom[i] * X.a[i][j];
    m_vec(vs, Si, w);
    double rr = 0.0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      rr = fma(w[i], vs[i], rr);
      m[i] = (i < d) ? om[i] - vom[i] * vs[i] : 0.0;
    }
    P.ell[t] = -0.5 * (d * kLog2Pi + logdet + rr);
    m_sym(Pm);
    if (P.mf) {
#pragma unroll
      for (int i = 0; i < K; ++i)
        if (i < d) P.mf[(int64_t)t * P.ldm + i] = m[i];
      double* pf = P.Pf + (int64_t)t * P.ldm * P.ldm;
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j)
          if (i < d && j < d) pf[i * P.ldm + j] = Pm.a[i][j];
    }
  }
  if (!ok) flag(P.status, P.fail_bit);
}

// ---------------------------------------------------------------------------
// Sampler element of step t: G = F P^f, P^p = G F' + Q (inverted through its
// Cholesky factor, then one Newton-Schulz step X <- X + X (I - P^p X), as the
// team build refines it), E_t = G' (P^p)^{-1}, L_t = P^f - E_t G,
// g_t = m^f - E_t (F m^f + bias), U_t = g_t + chol(L_t) xi_t; at the last
// step E = 0 and U = m^f + chol(P^f) xi.
// ---------------------------------------------------------------------------
__device__ void lane_sbuild(const KModel& M, const SampArgs& S, int t) {
  const int d = M.d;
  M4 Pf, L;
  m_load(Pf, S.Pf + (int64_t)t * S.ldm * S.ldm, S.ldm, d);
  double m[K], xi[K], g[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    m[i] = (i < d) ? S.mf[(int64_t)t * S.ldm + i] : 0.0;
    xi[i] = (i < d) ? S.xi_x[(int64_t)t * d + i] : 0.0;
  }
  bool ok = true;
  double ld;
  M4 E;
  m_zero(E);
  if (t == M.N - 1) {
    ok = m_chol(L, Pf, d, &ld);
#pragma unroll
    for (int i = 0; i < K; ++i) g[i] = m[i];
  } else {
    const double* Fp = S.Ft ? S.Ft + (int64_t)(t + 1) * d * d : M.F;
    const double* bp = S.Ft ? S.bt + (int64_t)(t + 1) * d : M.b;
    M4 F, G, Pp, Pi;
    m_load(F, Fp, d, d);
    m_load(Pp, M.Q, d, d);
    m_mul(G, F, Pf);
    {
      M4 GF;
      m_mul_nt(GF, G, F);
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) Pp.a[i][j] += GF.a[i][j];
    }
    double mp[K];
    m_vec(mp, F, m);
#pragma unroll
    for (int i = 0; i < K; ++i) mp[i] += (i < d && bp) ? bp[i] : 0.0;
    ok = m_spd_inv(Pi, Pp, d, &ld) && ok;
    {  // X + X (I - P^p X)
      M4 R, Z;
      m_mul(R, Pp, Pi);
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) R.a[i][j] = ((i == j && i < d) ? 1.0 : 0.0) - R.a[i][j];
      m_mul(Z, Pi, R);
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) Pi.a[i][j] += Z.a[i][j];
    }
    m_mul_tn(E, G, Pi);
    M4 EG;
    m_mul(EG, E, G);
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int j = 0; j < K; ++j) EG.a[i][j] = Pf.a[i][j] - EG.a[i][j];
    double em[K];
    m_vec(em, E, mp);
#pragma unroll
    for (int i = 0; i < K; ++i) g[i] = m[i] - em[i];
    m_sym(EG);
    ok = m_chol(L, EG, d, &ld) && ok;
  }
  m_store_corner(E, S.E + (int64_t)t * DP * DP);
  if (S.Et) m_store_pad<true>(E, S.Et + (int64_t)t * DP * DP);
  if (S.Lc) m_store_pad<true>(L, S.Lc + (int64_t)t * DP * DP);
  double u[K];
  m_vec(u, L, xi);
#pragma unroll
  for (int i = 0; i < K; ++i) u[i] += g[i];
  v_store_pad(u, d, S.U + (int64_t)t * DP);
  if (!ok) flag(S.status, ST_FWD_NOT_PD);
}

// ---------------------------------------------------------------------------
// Sampler, block fold: the suffix aggregate of block `blk`, folding from its
// last step backwards, (E~, U~) <- (E_t E~, E_t U~ + U_t).
// ---------------------------------------------------------------------------
__device__ void lane_sfold(const KModel& M, const SampArgs& S, int blk) {
  const int d = M.d;
  const int s0 = blk * S.B, s1 = min(M.N, s0 + S.B);
  M4 Ea;
  double ua[K];
  m_load(Ea, S.E + (int64_t)(s1 - 1) * DP * DP, DP, d);
#pragma unroll
  for (int i = 0; i < K; ++i) ua[i] = (i < d) ? S.U[(int64_t)(s1 - 1) * DP + i] : 0.0;
  for (int t = s1 - 2; t >= s0; --t) {
    M4 Et, P;
    m_load(Et, S.E + (int64_t)t * DP * DP, DP, d);
    m_mul(P, Et, Ea);
    Ea = P;
    double nu[K];
    m_vec(nu, Et, ua);
#pragma unroll
    for (int i = 0; i < K; ++i) ua[i] = nu[i] + ((i < d) ? S.U[(int64_t)t * DP + i] : 0.0);
  }
  double* out = S.agg + (int64_t)blk * SampLayout<DP>::SIZE;
  m_store_corner(Ea, out + SampLayout<DP>::E);
  v_store_pad(ua, d, out + SampLayout<DP>::U);
}

// Sampler, block final pass: x*_t = E_t x*_{t+1} + U_t from the state entering
// the block on the right.
__device__ void lane_sfinal(const KModel& M, const SampArgs& S, int blk) {
  const int d = M.d;
  const int s0 = blk * S.B, s1 = min(M.N, s0 + S.B);
  double x[K];
#pragma unroll
  for (int i = 0; i < K; ++i) x[i] = (i < d) ? S.xin[(int64_t)blk * DP + i] : 0.0;
  for (int t = s1 - 1; t >= s0; --t) {
    M4 Et;
    m_load(Et, S.E + (int64_t)t * DP * DP, DP, d);
    double nx[K];
    m_vec(nx, Et, x);
#pragma unroll
    for (int i = 0; i < K; ++i) {
      x[i] = nx[i] + ((i < d) ? S.U[(int64_t)t * DP + i] : 0.0);
      if (i < d) S.xs[(int64_t)t * d + i] = x[i];
    }
  }
}

// one lane per item; PH: 0 fold, 1 re-scan, 2 sampler element build,
// 3 sampler block fold, 4 sampler block final pass
template <int PH>
__global__ void __launch_bounds__(64) kl_phase(BatchLaunch L, int rev, const int* step) {
  const int w = blockIdx.x * 64 + threadIdx.x;
  if (w >= L.n_items) return;
  const Item I = L.items[w];
  const ChainDev& c = L.cd[I.c];
  if constexpr (PH == 0) {
    lane_fold(c.M, rev ? c.Fr : c.Ff, I.i);
  } else if constexpr (PH == 1) {
    lane_final(c.M, rev ? c.Fr : c.Ff, I.i);
  } else if constexpr (PH == 2) {
    SampArgs S = c.S;
    S.xi_x = c.xi_base + (int64_t)(*step) * c.xi_stride + (int64_t)c.M.N * c.M.d;
    lane_sbuild(c.M, S, I.i);
  } else if constexpr (PH == 3) {
    lane_sfold(c.M, c.S, I.i);
  } else {
    lane_sfinal(c.M, c.S, I.i);
  }
}

}  // namespace

hipError_t launch_lane_phase(int phase, BatchLaunch L, int rev, const int* step,
                             hipStream_t st) {
  if (L.n_items <= 0) return hipSuccess;
  const dim3 g((unsigned)((L.n_items + 63) / 64)), b(64);
  switch (phase) {
    case BP_FOLD_LANE: hipLaunchKernelGGL(kl_phase<0>, g, b, 0, st, L, rev, step); break;
    case BP_FINAL_LANE: hipLaunchKernelGGL(kl_phase<1>, g, b, 0, st, L, rev, step); break;
    case BP_SBUILD_LANE: hipLaunchKernelGGL(kl_phase<2>, g, b, 0, st, L, rev, step); break;
    case BP_SFOLD_LANE: hipLaunchKernelGGL(kl_phase<3>, g, b, 0, st, L, rev, step); break;
    case BP_SFINAL_LANE: hipLaunchKernelGGL(kl_phase<4>, g, b, 0, st, L, rev, step); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace akf
