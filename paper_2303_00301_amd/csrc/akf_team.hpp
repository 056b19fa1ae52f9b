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
// GEMMs run on the f64 matrix cores.  Inverses of SPD matrices (Gauss-Jordan)
// and Cholesky factors are computed in registers, one pivot per sweep, with
// the pivot row/column broadcast through a small double-buffered LDS vector
// (one barrier per sweep).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

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

__device__ __forceinline__ void team_sync() { __syncthreads(); }

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

// c = op(A) op(B) (+ c when ACC), A and B D x D in LDS.
template <int D, bool TA, bool TB, bool ACC>
__device__ __forceinline__ void gemm(RM<D>& c, const double* sA, const double* sB) {
  using C = Cfg<D>;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int r0 = (D == 64) ? 32 * (w >> 1) : 0, c0 = (D == 64) ? 32 * (w & 1) : 0;
  const int li = l & 15, lk = l >> 4;
  if (!ACC) rm_zero<D>(c);
#pragma unroll 4
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

// Pivot sweeps on a register matrix.  Sweeps run in groups of 16 (the pivot
// index k = 16 kb + kk with kk unrolled), so the register that holds row k or
// column k of a lane's tiles is known at compile time up to the tile index:
//   row k    -> tile row kb - r0/16, register kk/4, lanes with l/16 == kk%4;
//   column k -> tile column kb - c0/16, lanes with l%16 == kk.
template <int D>
struct Sweep {
  using C = Cfg<D>;
  int r0, c0, lg, lc;
  __device__ __forceinline__ Sweep() {
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    r0 = (D == 64) ? 32 * (w >> 1) : 0;
    c0 = (D == 64) ? 32 * (w & 1) : 0;
    lg = l >> 4;
    lc = l & 15;
  }
  __device__ __forceinline__ int row(int ti, int r) const { return r0 + 16 * ti + 4 * r + lg; }
  __device__ __forceinline__ int col(int tj) const { return c0 + 16 * tj + lc; }
};

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

// In-place inverse of a symmetric positive definite matrix held in registers
// (zero outside the leading d x d block) by d Gauss-Jordan sweeps:
//   p = A_kk;  A_kk <- 1/p;  A_kj <- A_kj/p;  A_ik <- -A_ik/p;
//   A_ij <- A_ij - A_ik A_kj / p            (i, j != k)
// The pivots p are those of the LDL' factorisation, so the matrix is PD iff
// all are > 0 and log det = sum log p.  Pivot row/column are broadcast through
// sbuf (4*D doubles of LDS, double-buffered: one barrier per sweep).  Returns
// false on a non-positive pivot (the result is then unspecified).  On entry no
// thread of the team may still be reading sbuf (a barrier separates any
// earlier use); the leading barrier also publishes earlier LDS writes.
template <int D>
__device__ bool spd_inv(RM<D>& A, int d, double* sbuf, double* logdet) {
  using C = Cfg<D>;
  const Sweep<D> o;
  bool ok = true;
  double ld = 0.0;
  for (int kb = 0; 16 * kb < d; ++kb) {
    const int ti_k = kb - o.r0 / 16, tj_k = kb - o.c0 / 16;
    const bool in_r = ti_k >= 0 && ti_k < C::TS, in_c = tj_k >= 0 && tj_k < C::TS;
    double prod = 1.0;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * kb + kk;
      if (k >= d) continue;  // uniform; keeps the trip count constant for unrolling
      double* sr = sbuf + (kk & 1) * D;
      double* sc = sbuf + 2 * D + (kk & 1) * D;
      const bool row_owner = in_r && o.lg == (kk & 3);
      const bool col_owner = in_c && o.lc == kk;
      if (row_owner) {
#pragma unroll
        for (int tj = 0; tj < C::TS; ++tj) sr[o.col(tj)] = rm_pick_row<D>(A, ti_k, tj, kk >> 2);
      }
      if (col_owner) {
#pragma unroll
        for (int ti = 0; ti < C::TS; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) sc[o.row(ti, r)] = rm_pick_col<D>(A, ti, tj_k, r);
      }
      team_sync();
      const double p = sr[k];
      ok = ok && (p > 0.0);
      const double ip = (p > 0.0) ? 1.0 / p : 0.0;
      prod *= (p > 0.0) ? p : 1.0;
      double rk[C::TS];
#pragma unroll
      for (int tj = 0; tj < C::TS; ++tj) rk[tj] = sr[o.col(tj)];
#pragma unroll
      for (int ti = 0; ti < C::TS; ++ti) {
        const bool rowk = row_owner && ti == ti_k;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double f = -sc[o.row(ti, r)] * ip;
#pragma unroll
          for (int tj = 0; tj < C::TS; ++tj) {
            const bool colk = col_owner && tj == tj_k;
            double v = A.t[ti * C::TS + tj][r];
            v = colk ? f : fma(f, rk[tj], v);
            if (r == (kk >> 2)) v = rowk ? (colk ? ip : rk[tj] * ip) : v;
            A.t[ti * C::TS + tj][r] = v;
          }
        }
      }
    }
    ld += log(prod);
  }
  *logdet = ld;
  return ok;
}

// Lower Cholesky factor (positive diagonal) of a symmetric positive definite
// matrix held in registers (zero outside the leading d x d block), in place,
// right-looking: column k is scaled by 1/sqrt(A_kk) and broadcast through
// sbuf (2*D doubles, double-buffered), then the trailing lower triangle is
// updated.  The strict upper triangle is zeroed.  Returns false on a
// non-positive pivot; *logdet gets log det of the matrix.  Same sbuf entry
// condition as spd_inv.
template <int D>
__device__ bool chol_reg(RM<D>& A, int d, double* sbuf, double* logdet) {
  using C = Cfg<D>;
  const Sweep<D> o;
  bool ok = true;
  double ld = 0.0;
  for (int kb = 0; 16 * kb < d; ++kb) {
    const int tj_k = kb - o.c0 / 16;
    const bool in_c = tj_k >= 0 && tj_k < C::TS;
    double prod = 1.0;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int k = 16 * kb + kk;
      if (k >= d) continue;  // uniform; keeps the trip count constant for unrolling
      double* sc = sbuf + (kk & 1) * D;
      const bool col_owner = in_c && o.lc == kk;
      if (col_owner) {
#pragma unroll
        for (int ti = 0; ti < C::TS; ++ti)
#pragma unroll
          for (int r = 0; r < 4; ++r) sc[o.row(ti, r)] = rm_pick_col<D>(A, ti, tj_k, r);
      }
      team_sync();
      const double p = sc[k];
      ok = ok && (p > 0.0);
      const double pp = (p > 0.0) ? p : 1.0;
      const double sq = sqrt(pp), is = 1.0 / sq;
      prod *= pp;
      double ljk[C::TS];
#pragma unroll
      for (int tj = 0; tj < C::TS; ++tj) {
        const int j = o.col(tj);
        const double scj = sc[j];  // loaded unconditionally: no branch per element
        ljk[tj] = (j > k && j < d) ? scj * is : 0.0;
      }
#pragma unroll
      for (int ti = 0; ti < C::TS; ++ti)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = o.row(ti, r);
          const double sci = sc[i];
          const double lik = (i > k && i < d) ? sci * is : 0.0;
#pragma unroll
          for (int tj = 0; tj < C::TS; ++tj) {
            const int j = o.col(tj);
            const bool colk = col_owner && tj == tj_k;
            const double v = A.t[ti * C::TS + tj][r];
            A.t[ti * C::TS + tj][r] =
                colk ? ((i == k) ? sq : lik) : ((j > k && i >= j) ? fma(-lik, ljk[tj], v) : v);
          }
        }
    }
    ld += log(prod);
  }
  AKF_RM_FOR(D, q, r, i, j) if (j > i) A.t[q][r] = 0.0;
  *logdet = ld;  // log det A = sum_k log p_k (p_k = L_kk^2)
  return ok;
}

// y[i] = sum_j op(A)[i][j] x[j] for i < D (LDS matrix, LDS vectors). Caller syncs.
template <int D, bool TA>
__device__ __forceinline__ void matvec(double* y, const double* sA, const double* x) {
  using C = Cfg<D>;
  const int tid = threadIdx.x;
  if (tid < D) {
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < D; ++j) s = fma(TA ? sA[j * C::LD + tid] : sA[tid * C::LD + j], x[j], s);
    y[tid] = s;
  }
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
