// akf_team.hpp -- device-side dense FP64 linear algebra for one workgroup
// ("team") working on D x D matrices, D in {16, 32, 64}, on gfx950.
//
// Layout conventions
//  * A team is 1 wavefront (D <= 32) or 4 wavefronts (D = 64).  Each wave owns
//    a QD x QD quadrant (QD = min(D, 32)) made of 16 x 16 tiles.
//  * Register matrices (RM) hold the quadrant in the accumulator layout of
//    v_mfma_f64_16x16x4f64: in tile q, lane l, register r holds element
//    (row0 + 4*r + l/16, col0 + l%16) (measured on gfx950).  Every RM in a team uses the same
//    ownership map, so element-wise arithmetic needs no data movement.
//  * LDS matrices are row-major with leading dimension LD = D + 1 doubles (the
//    odd stride spreads column accesses over the banks).
//  * Runtime size d <= D: padded rows/columns are zero in every matrix
//    (factors and inverses included).
//
// GEMMs run on the f64 matrix cores.  Inverses of SPD matrices (block
// Gauss-Jordan) and Cholesky factors (blocked, right-looking) are computed in
// registers: each 16 x 16 pivot tile is swept inside one wave (lane
// broadcasts, no LDS), the pivot block row or column is staged through a
// double-buffered LDS panel (one barrier per panel), and every other product
// is an MFMA chain.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace akf {

typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int D_>
struct Cfg {
  static constexpr int D = D_;
  static constexpr int QD = D < 32 ? D : 32;
  static constexpr int NW = (D / QD) * (D / QD);
  static constexpr int NT = 64 * NW;
  static constexpr int TS = QD / 16;
  static constexpr int TPW = TS * TS;
  static constexpr int NB = D / 16;
  static constexpr int LD = D + 1;
  static constexpr int MAT = D * LD;
};

__device__ __forceinline__ double lane_bcast(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, src);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Orders this wave's LDS accesses (LDS operations of one wave complete in
// issue order; this keeps the compiler from moving them across the point).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Team barrier that orders LDS only: threads of a team exchange data through
// LDS, never through global memory within one launch, so the barrier waits
// for the team's LDS operations but not for its outstanding global loads and
// stores (a per-step store of a result need not finish before the next step).
__device__ __forceinline__ void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int D>
struct RM {
  dbl4 t[Cfg<D>::TPW];
};

template <int D>
__device__ __forceinline__ int rm_row(int q, int r) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r0 = (D == 64) ? 32 * (w >> 1) : 0;
  return r0 + 16 * (q / Cfg<D>::TS) + 4 * r + (l >> 4);
}

template <int D>
__device__ __forceinline__ int rm_col(int q) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int c0 = (D == 64) ? 32 * (w & 1) : 0;
  return c0 + 16 * (q % Cfg<D>::TS) + (l & 15);
}

#define AKF_RM_FOR(D, q, r, i, j)                                   \
  _Pragma("unroll") for (int q = 0; q < Cfg<D>::TPW; ++q)           \
    _Pragma("unroll") for (int r = 0; r < 4; ++r)                   \
      if (const int i = rm_row<D>(q, r), j = rm_col<D>(q); true)

template <int D>
__device__ __forceinline__ void rm_zero(RM<D>& a) {
#pragma unroll
  for (int q = 0; q < Cfg<D>::TPW; ++q) a.t[q] = dbl4{0.0, 0.0, 0.0, 0.0};
}

// identity on the leading d x d block
template <int D>
__device__ __forceinline__ void rm_eye(RM<D>& a, int d) {
  AKF_RM_FOR(D, q, r, i, j) a.t[q][r] = (i == j && i < d) ? 1.0 : 0.0;
}

// a = G[i*ld + j] on the leading d x d block, zero elsewhere (global memory)
template <int D>
__device__ __forceinline__ void rm_load(RM<D>& a, const double* __restrict__ g, int ld, int d) {
  AKF_RM_FOR(D, q, r, i, j) a.t[q][r] = (i < d && j < d) ? g[(size_t)i * ld + j] : 0.0;
}

template <int D>
__device__ __forceinline__ void rm_add_load(RM<D>& a, const double* __restrict__ g, int ld, int d) {
  AKF_RM_FOR(D, q, r, i, j) if (i < d && j < d) a.t[q][r] += g[(size_t)i * ld + j];
}

template <int D>
__device__ __forceinline__ void rm_store(const RM<D>& a, double* __restrict__ g, int ld, int d) {
  AKF_RM_FOR(D, q, r, i, j) if (i < d && j < d) g[(size_t)i * ld + j] = a.t[q][r];
}

// transposed store of the whole D x D tile: G[j*ld + i] = a_ij
template <int D>
__device__ __forceinline__ void rm_store_t(const RM<D>& a, double* __restrict__ g, int ld) {
  AKF_RM_FOR(D, q, r, i, j) g[(size_t)j * ld + i] = a.t[q][r];
}

template <int D>
__device__ __forceinline__ void rm_stage(const RM<D>& a, double* s) {
  AKF_RM_FOR(D, q, r, i, j) s[i * Cfg<D>::LD + j] = a.t[q][r];
}

template <int D>
__device__ __forceinline__ void rm_stage_t(const RM<D>& a, double* s) {
  AKF_RM_FOR(D, q, r, i, j) s[j * Cfg<D>::LD + i] = a.t[q][r];
}

template <int D>
__device__ __forceinline__ void rm_unstage(RM<D>& a, const double* s) {
  AKF_RM_FOR(D, q, r, i, j) a.t[q][r] = s[i * Cfg<D>::LD + j];
}

// store(e, load(e)) for every e < n (n <= CAP) by a team of NT threads, each
// lane issuing G loads before their stores (all of them by default).  A
// lane-strided loop (e = tid; e < n; e += NT) has no trip count the compiler
// can see, stays rolled and waits out one memory latency per iteration (16
// round trips for a 64 x 64 matrix over 256 lanes, about 20k cycles).  Code
// that holds most of the register file passes a small G: each group of G
// loads costs one round trip and 2 G registers.
template <int NT, int CAP, int G = (CAP + NT - 1) / NT, typename L, typename S>
__device__ __forceinline__ void team_move(int n, L load, S store) {
  constexpr int PER = (CAP + NT - 1) / NT;
  const int tid = threadIdx.x;
#pragma unroll
  for (int k0 = 0; k0 < PER; k0 += G) {
    double v[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int e = tid + (k0 + k) * NT;
      v[k] = (k0 + k < PER && e < n) ? load(e) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int e = tid + (k0 + k) * NT;
      if (k0 + k < PER && e < n) store(e, v[k]);
    }
  }
}

// LDS matrix s (leading dimension LD) from element (i, j) = at(i, j) of the
// D x D block, read from global memory by the whole team, G loads per lane
// in flight (see team_move).
template <int D, int G = D * D / Cfg<D>::NT, typename F>
__device__ __forceinline__ void lds_fill(double* s, F at) {
  using C = Cfg<D>;
  team_move<C::NT, D * D, G>(
      D * D, [&](int e) { return at(e / D, e % D); },
      [&](int e, double v) { s[(e / D) * C::LD + (e % D)] = v; });
}

// dst[e] = src[e] for e < n by NT threads, eight loads per lane in flight
// before their stores (same reason as lds_fill).
template <int NT>
__device__ __forceinline__ void team_copy(double* __restrict__ dst,
                                          const double* __restrict__ src, int n) {
  const int tid = threadIdx.x;
  for (int base = 0; base < n; base += 8 * NT) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = base + k * NT + tid;
      v[k] = e < n ? src[e] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = base + k * NT + tid;
      if (e < n) dst[e] = v[k];
    }
  }
}

// y += alpha * x
template <int D>
__device__ __forceinline__ void rm_axpy(RM<D>& y, double alpha, const RM<D>& x) {
#pragma unroll
  for (int q = 0; q < Cfg<D>::TPW; ++q) y.t[q] += alpha * x.t[q];
}

// y = x - y
template <int D>
__device__ __forceinline__ void rm_rsub(RM<D>& y, const RM<D>& x) {
#pragma unroll
  for (int q = 0; q < Cfg<D>::TPW; ++q) y.t[q] = x.t[q] - y.t[q];
}

// 0.5 (a + a^T) through an LDS scratch matrix (team-wide; starts and ends
// with a barrier, so s may still be in use by a preceding product)
template <int D>
__device__ __forceinline__ void rm_symmetrise(RM<D>& a, double* s) {
  team_sync();
  rm_stage_t<D>(a, s);
  team_sync();
  AKF_RM_FOR(D, q, r, i, j) a.t[q][r] = 0.5 * (a.t[q][r] + s[i * Cfg<D>::LD + j]);
  team_sync();
}

// c = op(A) op(B) (+ c when ACC), A and B D x D in LDS.  U k-steps per
// unrolled iteration: the full D / 4 lets every operand load issue ahead of
// the products that need it (one team at D = 64: 4.4k cycles, against 6.5k
// with U = 4), at the price of registers, so kernels near the register limit
// keep U = 4.
template <int D, bool TA, bool TB, bool ACC, int U = 4>
__device__ __forceinline__ void gemm(RM<D>& c, const double* sA, const double* sB) {
  using C = Cfg<D>;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r0 = (D == 64) ? 32 * (w >> 1) : 0, c0 = (D == 64) ? 32 * (w & 1) : 0;
  const int li = l & 15, lk = l >> 4;
  if (!ACC) rm_zero<D>(c);
#pragma unroll U
  for (int kb = 0; kb < D / 4; ++kb) {
    const int k = 4 * kb + lk;
    double a[C::TS], b[C::TS];
#pragma unroll
    for (int ti = 0; ti < C::TS; ++ti) {
      const int i = r0 + 16 * ti + li;
      a[ti] = TA ? sA[k * C::LD + i] : sA[i * C::LD + k];
    }
#pragma unroll
    for (int tj = 0; tj < C::TS; ++tj) {
      const int j = c0 + 16 * tj + li;
      b[tj] = TB ? sB[j * C::LD + k] : sB[k * C::LD + j];
    }
#pragma unroll
    for (int ti = 0; ti < C::TS; ++ti)
#pragma unroll
      for (int tj = 0; tj < C::TS; ++tj)
        c.t[ti * C::TS + tj] =
            __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], c.t[ti * C::TS + tj], 0, 0, 0);
  }
}

// c1 = op(A) B1, c2 = op(A) B2 (+ c when ACC): two products that share their
// left operand, interleaved so that each k-step loads A's fragments once and
// issues twice as many independent MFMA chains behind its loads.
template <int D, bool TA, bool ACC, int U = 4>
__device__ __forceinline__ void gemm2(RM<D>& c1, RM<D>& c2, const double* sA, const double* sB1,
                                      const double* sB2) {
  using C = Cfg<D>;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r0 = (D == 64) ? 32 * (w >> 1) : 0, c0 = (D == 64) ? 32 * (w & 1) : 0;
  const int li = l & 15, lk = l >> 4;
  if (!ACC) {
    rm_zero<D>(c1);
    rm_zero<D>(c2);
  }
#pragma unroll U
  for (int kb = 0; kb < D / 4; ++kb) {
    const int k = 4 * kb + lk;
    double a[C::TS], b1[C::TS], b2[C::TS];
#pragma unroll
    for (int ti = 0; ti < C::TS; ++ti) {
      const int i = r0 + 16 * ti + li;
      a[ti] = TA ? sA[k * C::LD + i] : sA[i * C::LD + k];
    }
#pragma unroll
    for (int tj = 0; tj < C::TS; ++tj) {
      const int j = c0 + 16 * tj + li;
      b1[tj] = sB1[k * C::LD + j];
      b2[tj] = sB2[k * C::LD + j];
    }
#pragma unroll
    for (int ti = 0; ti < C::TS; ++ti)
#pragma unroll
      for (int tj = 0; tj < C::TS; ++tj) {
        c1.t[ti * C::TS + tj] =
            __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b1[tj], c1.t[ti * C::TS + tj], 0, 0, 0);
        c2.t[ti * C::TS + tj] =
            __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b2[tj], c2.t[ti * C::TS + tj], 0, 0, 0);
      }
  }
}

// element (ti, tj, r) of a register matrix with a runtime tile index ti or tj
// (TS <= 2).  Both candidates are read as values before the select: a select
// between two element lvalues would index the register array at run time and
// push it to scratch memory.
template <int D>
__device__ __forceinline__ double rm_pick_row(const RM<D>& A, int ti, int tj, int r) {
  if constexpr (Cfg<D>::TS == 1) {
    return A.t[0][r];
  } else {
    const double a = static_cast<double>(A.t[tj][r]);
    const double b = static_cast<double>(A.t[Cfg<D>::TS + tj][r]);
    return ti ? b : a;
  }
}
template <int D>
__device__ __forceinline__ double rm_pick_col(const RM<D>& A, int ti, int tj, int r) {
  if constexpr (Cfg<D>::TS == 1) {
    return A.t[0][r];
  } else {
    const double a = static_cast<double>(A.t[ti * Cfg<D>::TS][r]);
    const double b = static_cast<double>(A.t[ti * Cfg<D>::TS + 1][r]);
    return tj ? b : a;
  }
}

// 16 x 16 x 16 tile product on one wave: c + A B with the operands given as
// per-k-step fragments: a[s] = A[l%16][4s + l/16], b[s] = B[4s + l/16][l%16].
// In the accumulator layout, register s of a tile M is M[4s + l/16][l%16], so
// the registers of M are its own B fragments and the A fragments of M'.
__device__ __forceinline__ dbl4 mfma16(const double a[4], const double b[4], dbl4 c) {
#pragma unroll
  for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[s], c, 0, 0, 0);
  return c;
}
__device__ __forceinline__ void tile_regs(const dbl4& t, double x[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) x[s] = t[s];
}

// log-determinant accumulator: mantissa product and binary exponent sum
struct LogDet {
  double m = 1.0;
  int e = 0;
  __device__ __forceinline__ void mul(double x) {
    int ex;
    m = frexp(m * x, &ex);
    e += ex;
  }
  __device__ __forceinline__ double value() const { return log(m) + e * 0.69314718055994530942; }
};

// f(integral_constant<int, K>) for K = B .. E-1 (compile-time loop)
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Broadcast of lane K of every row of 16 lanes to the whole row (64-bit DPP
// row_newbcast).
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xF, 0xF, true);
}

// v from lane src of the wave (ds_bpermute; no LDS memory involved)
__device__ __forceinline__ double lane_fetch(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// 1/q for q > 0: hardware reciprocal estimate refined by two Newton-Raphson
// steps r <- r + r (1 - q r) (each step squares the relative error).
__device__ __forceinline__ double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// 1/sqrt(q) for q > 0: hardware estimate refined by two Newton-Raphson steps
// r <- r (3 - q r^2) / 2.
__device__ __forceinline__ double rsqrt_nr(double q) {
  double r = __builtin_amdgcn_rsq(q);
  const double h = 0.5 * q;
  r = r * fma(-h * r, r, 1.5);
  r = r * fma(-h * r, r, 1.5);
  return r;
}

// One wave inverts a symmetric positive definite 16 x 16 tile held in the
// accumulator layout (p[r] = P[4r + l/16][l%16]) by 16 steps of the symmetric
// sweep operator: with c = column k of the current matrix and pivot q = c_k,
//   a_ij <- a_ij - c_i c_j / q (i, j != k),  a_ik = a_ki <- c_i / q,  a_kk <- -1/q,
// which leaves -P^{-1}.  The matrix stays symmetric, so column k is also row k.
// Column k reaches the lanes of each row of 16 by a DPP row broadcast of lane
// k (c_i for the lane's rows i = 4r + l/16), row k by a lane permute (c_j for
// the lane's column j = l%16), the pivot by a lane read.  Every element update
// is one FMA, a' = f_i r_j + m a, with f_i = -c_i/q (f_k = 1/q), r_j = c_j
// (r_k = -1) and m = 0 on row and column k, 1 elsewhere.  The pivots are those
// of the LDL' factorisation; with CHOL the lower Cholesky factor is captured
// on the way (L_ik = c_i / sqrt(q), i >= k).  Indices >= nv are padding: they
// get a unit diagonal.  A non-positive pivot clears ok (the results are then
// unspecified).
template <bool CHOL, bool PART = false>
__device__ __forceinline__ void tile_sweep16(double p[4], int nv, double Lk[4], LogDet& ld,
                                             bool& ok) {
  const int l = threadIdx.x & 63, lg = l >> 4, lc = l & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (4 * r + lg >= nv && 4 * r + lg == lc) p[r] = 1.0;
    if constexpr (CHOL) Lk[r] = 0.0;
  }
  double prod = 1.0;
  auto step = [&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int rk = k >> 2;
    double ci[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ci[r] = row_bcast<k>(p[r]);
    const double q = lane_bcast(p[rk], 16 * (k & 3) + k);
    const double cj = lane_fetch(p[rk], 16 * (k & 3) + lc);
    ok = ok && (q > 0.0);
    const double iq = recip(q);
    prod *= q;
    if constexpr ((k & 3) == 3) {
      ld.mul(prod);
      prod = 1.0;
    }
    const bool jk = (lc == k), ik = (lg == (k & 3));
    const double rj = jk ? -1.0 : cj;
    const double mc = jk ? 0.0 : 1.0;         // rows other than k
    const double mk = (jk || ik) ? 0.0 : 1.0;  // register rk (holds row k when ik)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double fi = -ci[r] * iq;
      if (r == rk) fi = ik ? iq : fi;
      p[r] = fma(fi, rj, p[r] * (r == rk ? mk : mc));
    }
    if constexpr (CHOL) {
      const double isq = rsqrt_nr(q);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double lv;
        if (r > rk) lv = ci[r] * isq;
        else if (r < rk) lv = 0.0;
        else lv = (lg > (k & 3)) ? ci[r] * isq : (ik ? q * isq : 0.0);
        Lk[r] = jk ? lv : Lk[r];
      }
    }
  };
  if (!PART || nv >= 16) {
    static_for<0, 16>(step);
  } else {
    // PART, a tile with padding (a team wider than d): the steps of padded
    // pivots change no valid entry (their column is zero there), so they are
    // skipped and the padded part is set to what they would have left (unit
    // diagonal).  Only the 16-wide teams take this path: in wider teams the
    // second code path costs registers that the big kernels do not have.
    auto some = [&](auto kc) {
      if (decltype(kc)::value < nv) step(kc);
    };
    static_for<0, 16>(some);
    ld.mul(prod);  // pivots of an unfinished group of four
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * r + lg;
      if (i >= nv || lc >= nv) {
        p[r] = (i == lc) ? -1.0 : 0.0;  // negated below
        if constexpr (CHOL) Lk[r] = (i == lc) ? 1.0 : 0.0;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) p[r] = -p[r];
}

// G = L^{-T} for a 16 x 16 tile from its Cholesky factor (Lk, acc layout) and
// the inverse of the tile (ainv, symmetric): G0 = A^{-1} L, then one Newton
// step G = G0 + G0 (I - L' G0), with L^{-1} ~ L' A^{-1} as G0' in the
// correction.  Forming L^{-T} through A^{-1} alone loses accuracy with the
// conditioning of the tile; the Newton step restores it.
__device__ __forceinline__ void chol_tile_rinv(const double ainv[4], const double Lk[4],
                                               double G[4]) {
  const int l = threadIdx.x & 63, lg = l >> 4, lc = l & 15;
  const dbl4 z = {0.0, 0.0, 0.0, 0.0};
  double H[4], R[4];
  tile_regs(mfma16(ainv, Lk, z), G);  // A^{-1} L  (acc of L^{-T})
  tile_regs(mfma16(Lk, ainv, z), H);  // L' A^{-1} (acc of L^{-1})
  const dbl4 T = mfma16(Lk, G, z);    // L' G ~ I
#pragma unroll
  for (int r = 0; r < 4; ++r) R[r] = ((4 * r + lg == lc) ? 1.0 : 0.0) - T[r];
  dbl4 g = {G[0], G[1], G[2], G[3]};
  tile_regs(mfma16(H, R, g), G);  // G + G (I - L' G)
}

// One Newton-Schulz step X <- X + X (I - A X) on an approximate inverse X of
// the register matrix A (both zero outside the leading d x d block): squares
// the residual, so an inverse accurate to r relative becomes accurate to
// ~cond(A) r^2 plus rounding.  s1, s2: free LDS matrices.  Team-wide; ends
// synchronised.
template <int D>
__device__ void inv_refine(RM<D>& X, const RM<D>& A, int d, double* s1, double* s2) {
  team_sync();
  rm_stage<D>(X, s1);
  rm_stage<D>(A, s2);
  team_sync();
  RM<D> T;
  gemm<D, false, false, false>(T, s2, s1);  // A X
  AKF_RM_FOR(D, q, r, i, j) T.t[q][r] = ((i == j && i < d) ? 1.0 : 0.0) - T.t[q][r];
  team_sync();
  rm_stage<D>(T, s2);
  team_sync();
  gemm<D, false, false, true>(X, s1, s2);  // X + X (I - A X)
  team_sync();
}

// LDS scratch (doubles) needed by spd_inv and chol_reg: the staged block row
// or column, double-buffered across waves (none at D = 16: one tile).
template <int D>
constexpr int inv_scratch() {
  using C = Cfg<D>;
  constexpr int nbuf = C::NW > 1 ? 2 : 1;
  constexpr int rows = nbuf * 16 * (D + 1), cols = nbuf * D * 17;
  return D == 16 ? 0 : (rows > cols ? rows : cols);
}

// In-place inverse of a symmetric positive definite matrix held in registers
// (zero outside the leading d x d block) by block Gauss-Jordan elimination
// with 16 x 16 pivot blocks P = A_KK:
//   A_KK <- P^{-1},  A_KJ <- P^{-1} A_KJ,  A_IK <- -A_IK P^{-1},
//   A_IJ <- A_IJ - A_IK P^{-1} A_KJ.
// The pivot block is inverted by every wave (tile_sweep16); the block row K
// is staged through LDS and every other product is a 16 x 16 x 16 MFMA chain.
// The elimination keeps A_IK = s_I A_KI' (s_I = -1 for processed blocks I < K,
// +1 otherwise), so A_IK P^{-1} = s_I (P^{-1} A_KI)' needs only block row K.
// Returns false on a non-positive pivot (the result is then unspecified);
// *logdet = log det A from the pivots.  scr: inv_scratch<D>() doubles of LDS,
// free at entry; the call begins and ends with a team barrier.
template <int D>
__device__ bool spd_inv(RM<D>& A, int d, double* scr, double* logdet) {
  using C = Cfg<D>;
  static_assert(inv_scratch<D>() <= C::MAT, "scratch must fit one LDS matrix");
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lg = l >> 4, lc = l & 15;
  bool ok = true;
  LogDet ld;
  team_sync();
  if constexpr (D == 16) {
    double p[4], dummy[4];
    tile_regs(A.t[0], p);
    tile_sweep16<false, D == 16>(p, d, dummy, ld, ok);
#pragma unroll
    for (int r = 0; r < 4; ++r) A.t[0][r] = p[r];
  } else {
    constexpr int nbuf = C::NW > 1 ? 2 : 1, LDR = D + 1;
    const int R0 = (D == 64) ? 2 * (w >> 1) : 0, C0 = (D == 64) ? 2 * (w & 1) : 0;
    const int nb = (d + 15) / 16;
    for (int kb = 0; kb < nb; ++kb) {
      double* BR = scr + (kb % nbuf) * 16 * LDR;
      const int ti_k = kb - R0;
      if (ti_k >= 0 && ti_k < C::TS) {
#pragma unroll
        for (int tj = 0; tj < C::TS; ++tj)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            BR[(4 * r + lg) * LDR + 16 * (C0 + tj) + lc] = rm_pick_row<D>(A, ti_k, tj, r);
      }
      team_sync();
      auto brow = [&](int T, double x[4]) {  // B fragments of A_KT
#pragma unroll
        for (int s = 0; s < 4; ++s) x[s] = BR[(4 * s + lg) * LDR + 16 * T + lc];
      };
      double pv[4], dummy[4];
      brow(kb, pv);
      tile_sweep16<false, D == 16>(pv, d - 16 * kb, dummy, ld, ok);  // pv = P^{-1}
      const dbl4 z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ti = 0; ti < C::TS; ++ti) {
        const int TI = R0 + ti;
        const double sI = (TI < kb) ? -1.0 : 1.0;
        double bi[4], xa[4];
        brow(TI, bi);
        if (TI != kb) {
          const dbl4 xr = mfma16(pv, bi, z);  // P^{-1} A_KI
#pragma unroll
          for (int s = 0; s < 4; ++s) xa[s] = -sI * xr[s];
        }
#pragma unroll
        for (int tj = 0; tj < C::TS; ++tj) {
          const int TJ = C0 + tj, q = ti * C::TS + tj;
          if (TI == kb && TJ == kb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) A.t[q][r] = pv[r];
          } else if (TI == kb) {
            double bj[4];
            brow(TJ, bj);
            A.t[q] = mfma16(pv, bj, z);  // P^{-1} A_KJ
          } else if (TJ == kb) {
            const dbl4 y = mfma16(bi, pv, z);  // A_KI' P^{-1}
            A.t[q] = -sI * y;
          } else {
            double bj[4];
            brow(TJ, bj);
            A.t[q] = mfma16(xa, bj, A.t[q]);  // A_IJ - s_I (P^{-1} A_KI)' A_KJ
          }
        }
      }
    }
  }
  AKF_RM_FOR(D, q, r, i, j) if (i >= d || j >= d) A.t[q][r] = 0.0;
  team_sync();
  *logdet = ld.value();
  return ok;
}

// Lower Cholesky factor (positive diagonal) of a symmetric positive definite
// matrix held in registers (zero outside the leading d x d block), in place,
// blocked right-looking with 16-column panels: the diagonal block is factored
// by every wave (tile_sweep16, which also yields A_KK^{-1}); the panel is
// L_IK = A_IK L_KK^{-T} (chol_tile_rinv); the trailing lower blocks get
// A_IJ -= L_IK L_JK'.  The block column K is staged through LDS; products are
// 16 x 16 x 16 MFMA chains.  The strict upper triangle is zeroed.  Returns
// false on a non-positive pivot; *logdet = log det A.  Same scr contract as
// spd_inv.
template <int D>
__device__ bool chol_reg(RM<D>& A, int d, double* scr, double* logdet) {
  using C = Cfg<D>;
  static_assert(inv_scratch<D>() <= C::MAT, "scratch must fit one LDS matrix");
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lg = l >> 4, lc = l & 15;
  bool ok = true;
  LogDet ld;
  team_sync();
  if constexpr (D == 16) {
    double p[4], Lk[4];
    tile_regs(A.t[0], p);
    tile_sweep16<true, D == 16>(p, d, Lk, ld, ok);
#pragma unroll
    for (int r = 0; r < 4; ++r) A.t[0][r] = Lk[r];
  } else {
    constexpr int nbuf = C::NW > 1 ? 2 : 1, LDC = 17;
    const int R0 = (D == 64) ? 2 * (w >> 1) : 0, C0 = (D == 64) ? 2 * (w & 1) : 0;
    const int nb = (d + 15) / 16;
    for (int kb = 0; kb < nb; ++kb) {
      double* BC = scr + (kb % nbuf) * D * LDC;
      const int tj_k = kb - C0;
      if (tj_k >= 0 && tj_k < C::TS) {
#pragma unroll
        for (int ti = 0; ti < C::TS; ++ti)
          if (R0 + ti >= kb) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              BC[(16 * (R0 + ti) + 4 * r + lg) * LDC + lc] = rm_pick_col<D>(A, ti, tj_k, r);
          }
      }
      team_sync();
      auto bcolt = [&](int T, double x[4]) {  // A fragments of A_TK (= B fragments of A_TK')
#pragma unroll
        for (int s = 0; s < 4; ++s) x[s] = BC[(16 * T + lc) * LDC + 4 * s + lg];
      };
      double pv[4], Lk[4], G[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) pv[r] = BC[(16 * kb + 4 * r + lg) * LDC + lc];
      tile_sweep16<true, D == 16>(pv, d - 16 * kb, Lk, ld, ok);  // pv = A_KK^{-1}, Lk = L_KK
      const dbl4 z = {0.0, 0.0, 0.0, 0.0};
      chol_tile_rinv(pv, Lk, G);  // G = L_KK^{-T}
      double LTr[C::TS][4], LTc[C::TS][4];  // (L_TK)' for the wave's row / column tiles
#pragma unroll
      for (int t = 0; t < C::TS; ++t) {
        if (R0 + t > kb) {
          double a[4];
          bcolt(R0 + t, a);
          tile_regs(mfma16(G, a, z), LTr[t]);
#pragma unroll
          for (int s = 0; s < 4; ++s) LTr[t][s] = -LTr[t][s];
        }
        if (C0 + t > kb) {
          double a[4];
          bcolt(C0 + t, a);
          tile_regs(mfma16(G, a, z), LTc[t]);
        }
      }
#pragma unroll
      for (int ti = 0; ti < C::TS; ++ti) {
        const int TI = R0 + ti;
#pragma unroll
        for (int tj = 0; tj < C::TS; ++tj) {
          const int TJ = C0 + tj, q = ti * C::TS + tj;
          if (TI == kb && TJ == kb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) A.t[q][r] = Lk[r];
          } else if (TJ == kb && TI > kb) {
            double a[4];
            bcolt(TI, a);
            A.t[q] = mfma16(a, G, z);  // L_IK = A_IK G
          } else if (TI > kb && TJ > kb && TI >= TJ) {
            A.t[q] = mfma16(LTr[ti], LTc[tj], A.t[q]);  // A_IJ - L_IK L_JK'
          }
        }
      }
    }
  }
  AKF_RM_FOR(D, q, r, i, j) if (j > i || i >= d) A.t[q][r] = 0.0;
  team_sync();
  *logdet = ld.value();
  return ok;
}

// y[i] = add[i] + sum_j op(A)[i][j] x[j] for i < D (LDS matrix; add may be
// null, may alias y, and may live in global memory; x must not alias y).
// Every wave takes D / NW rows and splits each row over 64 / (D / NW) lanes,
// reduced by lane shuffles, so the dependent chain is 16 (D >= 32) or 4 FMAs
// long.  Team-wide; ends with a barrier, after which y is visible to all.
template <int D, bool TA>
__device__ __forceinline__ void matvec(double* y, const double* sA, const double* x,
                                       const double* add = nullptr) {
  using C = Cfg<D>;
  constexpr int R = D / C::NW;  // rows per wave
  constexpr int P = 64 / R;     // lanes per row
  constexpr int JL = D / P;     // columns per lane
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int i = w * R + (l % R), j0 = (l / R) * JL;
  double s = 0.0;
#pragma unroll
  for (int jj = 0; jj < JL; ++jj) {
    const int j = j0 + jj;
    s = fma(TA ? sA[j * C::LD + i] : sA[i * C::LD + j], x[j], s);
  }
#pragma unroll
  for (int m = R; m < 64; m <<= 1) s += __shfl_xor(s, m);
  if (l < R) y[i] = (add ? add[i] : 0.0) + s;
  team_sync();
}

// team-wide sum of one double per thread (result returned to every thread)
template <int D>
__device__ __forceinline__ double team_sum(double v, double* sRed) {
  using C = Cfg<D>;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) sRed[tid >> 6] = v;
  team_sync();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < C::NW; ++i) s += sRed[i];
  team_sync();
  return s;
}

}  // namespace akf
