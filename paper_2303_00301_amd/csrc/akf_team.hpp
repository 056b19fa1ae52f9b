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
//  * Runtime size d <= D: padded rows/columns are zero in every matrix, except
//    that a matrix about to be Cholesky-factored gets ones on its padded
//    diagonal, so every factor and inverse is block-diagonal [L 0; 0 I].
//
// GEMMs run on the f64 matrix cores; the Cholesky factorisation and the
// triangular inverse are blocked by 16: each 16 x 16 diagonal block is
// factored by one wave in registers (row per lane, cross-lane reads), and the
// panel solve and trailing update are MFMA products.
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

// One 16 x 16 tile product on one wave: acc (+)= op(A_blk) op(B_blk), where the
// blocks start at the given LDS addresses (leading dimension LD).  Returns the
// accumulator tile in the MFMA layout (lane l, reg r -> (4*r + l/16, l%16)).
template <int D, bool TA, bool TB>
__device__ __forceinline__ dbl4 tile_mma(dbl4 acc, const double* sA, const double* sB) {
  using C = Cfg<D>;
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const int k = 4 * kb + lk;
    const double a = TA ? sA[k * C::LD + li] : sA[li * C::LD + k];
    const double b = TB ? sB[li * C::LD + k] : sB[k * C::LD + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

template <int D>
__device__ __forceinline__ void tile_store(const dbl4& t, double* s) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < 4; ++r) s[(4 * r + (l >> 4)) * Cfg<D>::LD + (l & 15)] = t[r];
}

template <int D>
__device__ __forceinline__ dbl4 tile_load(const double* s) {
  const int l = threadIdx.x & 63;
  dbl4 t;
#pragma unroll
  for (int r = 0; r < 4; ++r) t[r] = s[(4 * r + (l >> 4)) * Cfg<D>::LD + (l & 15)];
  return t;
}

// Wave-local factorisation of the 16 x 16 diagonal block at sS + off: lower
// Cholesky factor written back in place (upper part zeroed) and, when sG is
// its inverse written to sG + off.  Lane r (< 16) holds row r.
// Adds log det of the block to *logdet; clears *ok on a non-positive pivot.
template <int D>
__device__ __forceinline__ void diag16_chol_inv(double* sS, double* sG, int off, bool& ok,
                                                double& logdet) {
  using C = Cfg<D>;
  const int l = threadIdx.x & 63, r = l & 15;
  double a[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) a[j] = sS[off + r * C::LD + j];
  double ld = 0.0;
  bool good = true;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const double piv = lane_bcast(a[k], k);
    good = good && (piv > 0.0);
    const double p = piv > 0.0 ? piv : 1.0;
    const double s = sqrt(p), inv = 1.0 / s;
    ld += log(p);
    a[k] = (r == k) ? s : (r > k ? a[k] * inv : 0.0);
#pragma unroll
    for (int j = k + 1; j < 16; ++j) a[j] = fma(-a[k], lane_bcast(a[k], j), a[j]);
  }
#pragma unroll
  for (int j = 0; j < 16; ++j)
    if (j > r) a[j] = 0.0;
  {
    // column r of L^{-1} by forward substitution, L_ik read from lane i
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      double s = (i == r) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < i; ++k) s = fma(-lane_bcast(a[k], i), x[k], s);
      x[i] = s / lane_bcast(a[i], i);
    }
    if (l < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) sG[off + i * C::LD + r] = x[i];
    }
  }
  if (l < 16) {
#pragma unroll
    for (int j = 0; j < 16; ++j) sS[off + r * C::LD + j] = a[j];
  }
  ok = ok && good;
  logdet += ld;
}

// Team-wide blocked Cholesky of the symmetric matrix in sS (lower triangle
// used; indices >= d replaced by the identity).  On return sS holds L (lower,
// upper zeroed).  sG is a D x D LDS buffer: with FULL it receives L^{-1}
// (lower, upper zeroed); otherwise only its diagonal 16 x 16 blocks hold the
// inverses of L's diagonal blocks.  Returns false if a pivot was not strictly
// positive; *logdet_out gets log det of the leading d x d block.  sScal is a
// 2-double LDS scratch.  Ends synchronised.
template <int D, bool FULL>
__device__ bool chol_inv(double* sS, double* sG, int d, double* logdet_out, double* sScal) {
  using C = Cfg<D>;
  const int tid = threadIdx.x, w = tid >> 6;
  // pad to the identity beyond d; zero the upper triangle
  for (int e = tid; e < D * D; e += C::NT) {
    const int i = e / D, j = e % D;
    if (i >= d || j >= d) sS[i * C::LD + j] = (i == j) ? 1.0 : 0.0;
    else if (j > i) sS[i * C::LD + j] = 0.0;
  }
  if (FULL)
    for (int e = tid; e < D * D; e += C::NT) sG[(e / D) * C::LD + (e % D)] = 0.0;
  team_sync();
  bool ok = true;
  double ld = 0.0;
#pragma unroll
  for (int K = 0; K < C::NB; ++K) {
    const int offKK = (16 * K) * C::LD + 16 * K;
    if (w == 0) diag16_chol_inv<D>(sS, sG, offKK, ok, ld);
    team_sync();
    if (K + 1 < C::NB) {
      // panel: L_IK = S_IK L_KK^{-T}, with L_KK^{-1} in the diagonal block of sG
      const int npanel = C::NB - 1 - K;
      for (int p = w; p < npanel; p += C::NW) {
        const int I = K + 1 + p;
        const int offIK = (16 * I) * C::LD + 16 * K;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = tile_mma<D, false, true>(acc, sS + offIK, sG + offKK);
        wave_lds_fence();
        tile_store<D>(acc, sS + offIK);
      }
      team_sync();
      // trailing update: S_IJ -= L_IK L_JK^T for K < J <= I
      const int m = C::NB - 1 - K;
      const int ntr = m * (m + 1) / 2;
      for (int p = w; p < ntr; p += C::NW) {
        int I = 0, J = 0, c = 0;
        for (int ii = 0; ii < m; ++ii)
          for (int jj = 0; jj <= ii; ++jj) {
            if (c == p) { I = K + 1 + ii; J = K + 1 + jj; }
            ++c;
          }
        const int offIJ = (16 * I) * C::LD + 16 * J;
        dbl4 acc = tile_load<D>(sS + offIJ);
        dbl4 prod = {0.0, 0.0, 0.0, 0.0};
        prod = tile_mma<D, false, true>(prod, sS + (16 * I) * C::LD + 16 * K,
                                        sS + (16 * J) * C::LD + 16 * K);
        acc -= prod;
        if (I == J) {
          // keep the diagonal tile's upper part zero (only lower is read)
          const int l = tid & 63;
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if ((l & 15) > 4 * r + (l >> 4)) acc[r] = 0.0;
        }
        wave_lds_fence();
        tile_store<D>(acc, sS + offIJ);
      }
      team_sync();
    }
  }
  if (FULL && C::NB > 1) {
    // off-diagonal blocks of L^{-1}: G_IJ = -G_II sum_{K=J}^{I-1} L_IK G_KJ, by distance
    for (int dist = 1; dist < C::NB; ++dist) {
      const int npair = C::NB - dist;
      for (int p = w; p < npair; p += C::NW) {
        const int I = dist + p, J = p;
        dbl4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int K = J; K < I; ++K)
          acc = tile_mma<D, false, false>(acc, sS + (16 * I) * C::LD + 16 * K,
                                          sG + (16 * K) * C::LD + 16 * J);
        // stage into the (unused) upper block (J, I) of sG, then multiply by -G_II
        double* scr = sG + (16 * J) * C::LD + 16 * I;
        tile_store<D>(acc, scr);
        wave_lds_fence();
        dbl4 res = {0.0, 0.0, 0.0, 0.0};
        res = tile_mma<D, false, false>(res, sG + (16 * I) * C::LD + 16 * I, scr);
        res = -res;
        wave_lds_fence();
        tile_store<D>(res, sG + (16 * I) * C::LD + 16 * J);
      }
      team_sync();
    }
    // clear the upper scratch blocks
    for (int e = tid; e < D * D; e += C::NT) {
      const int i = e / D, j = e % D;
      if (j / 16 > i / 16) sG[i * C::LD + j] = 0.0;
    }
    team_sync();
  }
  // combine per-wave results (only wave 0 factored diagonal blocks)
  if (tid == 0) {
    sScal[0] = ld;
    sScal[1] = ok ? 1.0 : 0.0;
  }
  team_sync();
  if (logdet_out) *logdet_out = sScal[0];
  const bool res = sScal[1] != 0.0;
  team_sync();
  return res;
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
