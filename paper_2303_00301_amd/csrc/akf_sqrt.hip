// akf_sqrt.hip -- square-root form of the parallel Kalman filter and of the
// pathwise RTS sampler for the auxiliary model's diagonal pseudo-observations
// omega_t = x_t + N(0, Omega_t): the form the paper points to for FP32
// robustness (Sec. "Multivariate stochastic volatility model").
//
// Covariances travel as lower-triangular factors.  A filtering element is
// (A, b, U, eta, Z) with C = U U^T and J = Z Z^T, plus its log normaliser, and
// every covariance update is a triangularisation tria(M) -- the lower L with
// L L^T = M M^T -- computed by Householder reflections applied from the right:
//   step element / fold step : tria([[Omega^1/2, U_p], [0, U_p]]) = [[P11, 0], [P21, P22]]
//                              with U_p = tria([F U, L_Q]) (the prediction),
//                              P11 P11^T = S, P21 = P_p P11^{-T}, P22 P22^T = the
//                              updated covariance;
//   combine                  : tria([[U_i^T Z_j, I], [Z_j, 0]]) = [[X11, 0], [X21, X22]],
//                              G = U_i X11^{-T}, M = I - G X21^T = (I + C_i J_j)^{-1},
//                              A = A_j M A_i, U = tria([A_j G, U_j]),
//                              Z = tria([A_i^T X22, Z_i]);
//   sampling element         : tria([[L_Q, F U^f_t], [0, U^f_t]]) gives
//                              E_t = P21 P11^{-1} and chol(L_t) = P22.
// The blocked layout is the dense path's: per-block fold, Hillis-Steele levels
// over the block elements, per-block re-scan (a square-root Kalman filter from
// the prefix), then the sampler's element build, per-block suffix fold, a scan
// of the block aggregates and the per-block path.
//
// T (float or double) is the storage and arithmetic type of every matrix and
// vector; the triangularisations accumulate in double (the factorisations), as
// do the log-likelihood terms.  Teams are 256 threads with every operand in
// LDS; products are plain FMA loops (d <= 32 here: at these sizes the
// factorisations, not the products, set the time).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "../../include/akf.h"
#include "akf_internal.h"
#include "akf_layout.h"

namespace akf {
namespace sq {

constexpr int NT = 256;
constexpr double LOG2PI = 1.8378770664093454835606594728112;

template <int D>
struct Dm {
  static constexpr int LM = D + 1;          // LDS row stride of a D x D matrix
  static constexpr int MAT = D * LM;        // entries of one LDS matrix
  static constexpr int LW = 2 * D + 1;      // row stride of the triangularisation area
  static constexpr int WSZ = 2 * D * LW;    // 2D rows (doubles)
  static constexpr int DV = 8;              // double scratch
};

// Element in the workspace: A, U, Z (D x D dense, zero padded), b, eta.
template <int D>
struct El {
  static constexpr int A = 0, U = D * D, Z = 2 * D * D, b = 3 * D * D, eta = 3 * D * D + D;
  static constexpr int SIZE = 3 * D * D + 2 * D;
};

template <class T>
struct SqArgs {
  int N, d, B, nb;
  const double *m0, *F, *b, *om, *Om, *xi;  // boundary arrays, leading dimension d
  const double *Q, *P0;
  T *Fs, *LQ, *L0;                          // [D*D] each
  T *el_in, *el_out;                        // [nb * El::SIZE]
  double *lc_in, *lc_out;                   // [nb]
  int hs;                                   // Hillis-Steele distance
  T *mfT, *UfT;                             // [N*D], [N*D*D] filter outputs for the sampler
  T *E, *Ut;                                // [N*D*D], [N*D]
  T *agg, *xin;                             // [nb*(D*D+D)], [nb*D]
  double *mf, *Uf, *ell, *xs;               // outputs (leading dimension d); Uf, xs may be null
  int* status;
};

__device__ __forceinline__ void flag(int* st) { atomicOr(st, ST_FWD_NOT_PD); }

// ---------------------------------------------------------------------------
// team helpers (all NT threads call them; every one ends synchronised)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double team_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// dst (LDS, D x D) <- a d x d array with leading dimension ld, zero padded.
// Every lane issues all of its loads before its first LDS write (a
// lane-strided loop stays rolled and waits out each load in turn); with
// SYNC = false the caller batches several loads under one barrier.
template <class T, int D, bool SYNC = true, class S>
__device__ __forceinline__ void ld_mat(T* dst, const S* src, int d, int ld) {
  constexpr int PER = (D * D + NT - 1) / NT;
  T v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * NT, i = e / D, j = e % D;
    v[k] = (e < D * D && i < d && j < d) ? (T)src[(int64_t)i * ld + j] : T(0);
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + k * NT;
    if (e < D * D) dst[(e / D) * Dm<D>::LM + e % D] = v[k];
  }
  if constexpr (SYNC) __syncthreads();
}

// global dense D x D <- LDS matrix
template <class T, int D>
__device__ __forceinline__ void st_mat(T* dst, const T* src) {
  for (int e = threadIdx.x; e < D * D; e += NT) dst[e] = src[(e / D) * Dm<D>::LM + e % D];
}

template <class T, int D>
__device__ __forceinline__ void set_eye(T* dst, int d, T diag) {
  for (int e = threadIdx.x; e < D * D; e += NT) {
    const int i = e / D, j = e % D;
    dst[i * Dm<D>::LM + j] = (i == j && i < d) ? diag : T(0);
  }
  __syncthreads();
}

template <class T, int D>
__device__ __forceinline__ void cp_mat(T* dst, const T* src) {
  for (int e = threadIdx.x; e < Dm<D>::MAT; e += NT) dst[e] = src[e];
  __syncthreads();
}

// C = op(A) op(B) (+ Cadd, which may be C itself); C must not alias A or B.
template <class T, int D, bool TA, bool TB>
__device__ __forceinline__ void mm(T* __restrict__ C, const T* __restrict__ A, const T* __restrict__ B, int d,
                   const T* Cadd = nullptr, T sign = T(1)) {
  constexpr int L = Dm<D>::LM;
  for (int e = threadIdx.x; e < D * D; e += NT) {
    const int i = e / D, j = e % D;
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {  // the zero padding makes the padded width exact
      const T a = TA ? A[k * L + i] : A[i * L + k];
      const T b = TB ? B[j * L + k] : B[k * L + j];
      acc = fma(a, b, acc);
    }
    C[i * L + j] = (Cadd ? Cadd[i * L + j] : T(0)) + sign * acc;
  }
  __syncthreads();
}

// y = op(A) x (+ y0, which may be y); y must not alias x.
template <class T, int D, bool TA>
__device__ __forceinline__ void mv(T* __restrict__ y, const T* __restrict__ A, const T* __restrict__ x, int d,
                   const T* y0 = nullptr, T sign = T(1)) {
  constexpr int L = Dm<D>::LM;
  const int i = threadIdx.x;
  if (i < D) {
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) acc = fma(TA ? A[k * L + i] : A[i * L + k], x[k], acc);
    y[i] = (i < d) ? ((y0 ? y0[i] : T(0)) + sign * acc) : T(0);
  }
  __syncthreads();
}

// Lanes per column of a triangular solve over ncols columns: a power of two,
// at most one wave, with all columns' groups fitting in the team.
__device__ __forceinline__ int solve_group(int ncols) {
  int g = 64;
  while (g > 1 && g * ncols > NT) g >>= 1;
  return g;
}

// X <- L^{-1} X over ncols columns of X (entry (i, j) at X[i*rs + j*cs]); L lower
// (LDS, stride LM).  Forward substitution by columns of L: each column of X has
// a group of lanes, lane r owning the rows i = r mod group; x_i is formed by its
// owner, broadcast across the group by a shuffle, and every lane updates its
// rows below i.  Returns false on a non-positive pivot.
template <class T, int D>
__device__ __forceinline__ bool solve_l(T* X, int rs, int cs, const T* L, int ncols, int d) {
  constexpr int LM = Dm<D>::LM;
  const int gs = solve_group(ncols), tid = threadIdx.x, j = tid / gs, r = tid % gs;
  bool ok = true;
  if (j < ncols) {
    for (int i = 0; i < d; ++i) {
      T xi = T(0);
      if (r == i % gs) {
        const T p = L[i * LM + i];
        ok = ok && (p > T(0));
        xi = X[i * rs + j * cs] / p;
        X[i * rs + j * cs] = xi;
      }
      xi = __shfl(xi, i % gs, gs);
      for (int k = i + 1 + ((r - i - 1) % gs + gs) % gs; k < d; k += gs)
        X[k * rs + j * cs] = fma(-L[k * LM + i], xi, X[k * rs + j * cs]);
    }
  }
  __syncthreads();
  return __syncthreads_and(ok);
}

// X <- L^{-T} X over ncols columns (backward substitution with the upper L^T),
// laid out as solve_l.
template <class T, int D>
__device__ __forceinline__ bool solve_lt(T* X, int rs, int cs, const T* L, int ncols, int d) {
  constexpr int LM = Dm<D>::LM;
  const int gs = solve_group(ncols), tid = threadIdx.x, j = tid / gs, r = tid % gs;
  bool ok = true;
  if (j < ncols) {
    for (int i = d - 1; i >= 0; --i) {
      T xi = T(0);
      if (r == i % gs) {
        const T p = L[i * LM + i];
        ok = ok && (p > T(0));
        xi = X[i * rs + j * cs] / p;
        X[i * rs + j * cs] = xi;
      }
      xi = __shfl(xi, i % gs, gs);
      for (int k = r; k < i; k += gs) X[k * rs + j * cs] = fma(-L[i * LM + k], xi, X[k * rs + j * cs]);
    }
  }
  __syncthreads();
  return __syncthreads_and(ok);
}

// Rows of X (D x D in LDS): X <- X L^{-T} and X <- X L^{-1}.
template <class T, int D>
__device__ __forceinline__ bool rows_times_linvT(T* X, const T* L, int nrows, int d) {
  return solve_l<T, D>(X, 1, Dm<D>::LM, L, nrows, d);
}
template <class T, int D>
__device__ __forceinline__ bool rows_times_linv(T* X, const T* L, int nrows, int d) {
  return solve_lt<T, D>(X, 1, Dm<D>::LM, L, nrows, d);
}

// sum of log of the first d diagonal entries of an LDS factor, in double
template <class T, int D>
__device__ __forceinline__ double logdiag(const T* L, int d, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < d; i += NT) v += log((double)L[i * Dm<D>::LM + i]);
  return team_sum(v, red);
}

template <class T, int D>
__device__ __forceinline__ double dot(const T* x, const T* y, int d, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < d; i += NT) v += (double)x[i] * (double)y[i];
  return team_sum(v, red);
}

// ---------------------------------------------------------------------------
// tria: in-place triangularisation of the r x c block M (c >= r) at the top
// left of W (double, row stride LW).  On return W[0:r][0:r] is the lower-
// triangular L with non-negative diagonal and L L^T = M M^T.  L is computed in
// double as the Cholesky factor of the Gram matrix M M^T, itself formed in
// double: for matrices held in FP32 this is as accurate as a Householder
// reduction (the squared condition number of M, at most ~1e8 on these models,
// stays far below 1/eps of double), and it replaces a chain of r dependent
// reflections by one product and a Cholesky with two barriers per column.
// The factorisation is for a positive semi-definite matrix: a pivot <= 0 (an
// exactly singular direction, e.g. a zero block, or its rounding) gives a zero
// column.  Each thread keeps its 4 x 4 share of the Gram matrix in registers
// until every thread has read M, then writes it over M.
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ void tria(double* W, int r, int c, double* dv) {
  constexpr int LW = Dm<D>::LW, R = 2 * D, NB = R / 16;
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  // Gram matrix: thread (ti, tj) accumulates rows ti + 16 u and columns
  // tj + 16 v (consecutive threads read consecutive rows: no bank conflicts)
  double gv[NB][NB];
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int v = 0; v < NB; ++v) gv[u][v] = 0.0;
#pragma unroll 2
  for (int k = 0; k < c; ++k) {
    double a[NB], b[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      a[u] = (ti + 16 * u < r) ? W[(ti + 16 * u) * LW + k] : 0.0;
      b[u] = (tj + 16 * u < r) ? W[(tj + 16 * u) * LW + k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
#pragma unroll
      for (int v = 0; v < NB; ++v) gv[u][v] = fma(a[u], b[v], gv[u][v]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int v = 0; v < NB; ++v) {
      const int i = ti + 16 * u, j = tj + 16 * v;
      if (i < r && j < r) W[i * LW + j] = (j <= i) ? gv[u][v] : 0.0;
    }
  __syncthreads();
  // right-looking Cholesky; thread (ti, tj) updates rows ti + 16 a and
  // columns tj + 16 b of the trailing block
  for (int k = 0; k < r; ++k) {
    const double p = W[k * LW + k];
    const double dk = (p > 0.0) ? sqrt(p) : 0.0;
    const double inv = (dk > 0.0) ? 1.0 / dk : 0.0;
    for (int i = k + 1 + tid; i < r; i += NT) W[i * LW + k] *= inv;
    __syncthreads();
    if (tid == 0) W[k * LW + k] = dk;
#pragma unroll
    for (int a = 0; a < R / 16; ++a) {
      const int i = k + 1 + ti + 16 * a;
      if (i < r) {
        const double lik = W[i * LW + k];
#pragma unroll
        for (int b = 0; b < R / 16; ++b) {
          const int j = k + 1 + tj + 16 * b;
          if (j <= i) W[i * LW + j] = fma(-lik, W[j * LW + k], W[i * LW + j]);
        }
      }
    }
    __syncthreads();
  }
  (void)dv;
}

// W block (roff, coff) of size d x d <- an LDS matrix (optionally transposed)
template <class T, int D, bool TR>
__device__ __forceinline__ void to_w(double* W, int roff, int coff, const T* M, int d) {
  constexpr int LW = Dm<D>::LW, LM = Dm<D>::LM;
  for (int e = threadIdx.x; e < d * d; e += NT) {
    const int i = e / d, j = e % d;
    W[(roff + i) * LW + coff + j] = (double)(TR ? M[j * LM + i] : M[i * LM + j]);
  }
}

template <int D>
__device__ __forceinline__ void w_fill(double* W, int roff, int coff, int d, double diag) {
  constexpr int LW = Dm<D>::LW;
  for (int e = threadIdx.x; e < d * d; e += NT) {
    const int i = e / d, j = e % d;
    W[(roff + i) * LW + coff + j] = (i == j) ? diag : 0.0;
  }
}

// LDS matrix (zero padded) <- W block (roff, coff), d x d
template <class T, int D>
__device__ __forceinline__ void from_w(T* M, const double* W, int roff, int coff, int d) {
  constexpr int LW = Dm<D>::LW, LM = Dm<D>::LM;
  for (int e = threadIdx.x; e < D * D; e += NT) {
    const int i = e / D, j = e % D;
    M[i * LM + j] = (i < d && j < d) ? (T)W[(roff + i) * LW + coff + j] : T(0);
  }
}

// Measurement update of a predictive (m_p, U_p) by omega = x + N(0, diag Om):
// tria([[Om^1/2, U_p], [0, U_p]]) -> P11 (factor of S), P21, P22 (updated
// factor, written to Uo).  s = P11^{-1} (omega - m_p).  Returns the predictive
// log density of omega, in double, through *lpred.
template <class T, int D>
__device__ __forceinline__ bool sqrt_update(double* W, double* dv, const T* Up, const double* Om_t, int d, T* P11,
                            T* P21, T* Uo, T* vs, const T* vmp, const double* om_t, double* red,
                            double* lpred) {
  for (int e = threadIdx.x; e < d * d; e += NT) {
    const int i = e / d, j = e % d;
    W[i * Dm<D>::LW + j] = (i == j) ? sqrt(Om_t[i]) : 0.0;
  }
  to_w<T, D, false>(W, 0, d, Up, d);
  w_fill<D>(W, d, 0, d, 0.0);
  to_w<T, D, false>(W, d, d, Up, d);
  __syncthreads();
  tria<D>(W, 2 * d, 2 * d, dv);
  from_w<T, D>(P11, W, 0, 0, d);
  from_w<T, D>(P21, W, d, 0, d);
  from_w<T, D>(Uo, W, d, d, d);
  if (threadIdx.x < D) vs[threadIdx.x] = (threadIdx.x < d) ? (T)(om_t[threadIdx.x]) - vmp[threadIdx.x] : T(0);
  __syncthreads();
  const bool ok = solve_l<T, D>(vs, 1, 0, P11, 1, d);
  const double ld = logdiag<T, D>(P11, d, red);
  const double q = dot<T, D>(vs, vs, d, red);
  *lpred = -0.5 * (d * LOG2PI + 2.0 * ld + q);
  return ok;
}

// Prediction factor U_p = tria([F U, L_Q]) into Up (FU: scratch matrix).
template <class T, int D>
__device__ __forceinline__ void sqrt_predict(double* W, double* dv, const T* sF, const T* U, const T* sLQ, int d,
                             T* FU, T* Up) {
  mm<T, D, false, false>(FU, sF, U, d);
  to_w<T, D, false>(W, 0, 0, FU, d);
  to_w<T, D, false>(W, 0, d, sLQ, d);
  __syncthreads();
  tria<D>(W, d, 2 * d, dv);
  from_w<T, D>(Up, W, 0, 0, d);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// set-up: L_Q = chol(Q), L_0 = chol(P0) (double), F in T
// ---------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ bool chol_lds(double* A, int d) {
  constexpr int LM = Dm<D>::LM;
  __shared__ int okf;
  if (threadIdx.x == 0) okf = 1;
  __syncthreads();
  for (int k = 0; k < d; ++k) {
    if (threadIdx.x == 0) {
      const double p = A[k * LM + k];
      if (!(p > 0.0)) okf = 0;
      A[k * LM + k] = (p > 0.0) ? sqrt(p) : 1.0;
    }
    __syncthreads();
    for (int i = k + 1 + threadIdx.x; i < d; i += NT) A[i * LM + k] /= A[k * LM + k];
    __syncthreads();
    for (int e = threadIdx.x; e < d * d; e += NT) {
      const int i = e / d, j = e % d;
      if (j > k && i >= j) A[i * LM + j] -= A[i * LM + k] * A[j * LM + k];
    }
    __syncthreads();
  }
  return okf != 0;
}

__global__ void k_sq_init(int* status) {
  if (threadIdx.x < 2) status[threadIdx.x] = 0;
}

template <class T, int D>
__global__ void __launch_bounds__(NT) k_sq_prep(SqArgs<T> P) {
  __shared__ double A[Dm<D>::MAT];
  const int d = P.d;
  for (int which = 0; which < 2; ++which) {
    ld_mat<double, D>(A, which ? P.P0 : P.Q, d, d);
    const bool ok = chol_lds<D>(A, d);
    if (!ok && threadIdx.x == 0) flag(P.status);
    T* out = which ? P.L0 : P.LQ;
    for (int e = threadIdx.x; e < D * D; e += NT) {
      const int i = e / D, j = e % D;
      out[e] = (i < d && j <= i) ? (T)A[i * Dm<D>::LM + j] : T(0);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < D * D; e += NT) {
    const int i = e / D, j = e % D;
    P.Fs[e] = (i < d && j < d) ? (T)P.F[i * d + j] : T(0);
  }
}

// LDS carve-up shared by the kernels: nm matrices of T, nv vectors of T (D
// each), then the double areas (W, dv, red).
template <class T, int D>
struct Carve {
  T* m[14];
  T* v[10];
  double *W, *dv, *red;
  __device__ __forceinline__ Carve(unsigned char* base, int nm, int nv) {
    T* p = reinterpret_cast<T*>(base);
    for (int i = 0; i < nm; ++i) m[i] = p + i * Dm<D>::MAT;
    p += nm * Dm<D>::MAT;
    for (int i = 0; i < nv; ++i) v[i] = p + i * D;
    // the double areas start at a 16-byte multiple; plain pointer arithmetic on
    // the LDS base (no integer round trip) lets the compiler keep LDS accesses
    W = reinterpret_cast<double*>(base + tbytes(nm, nv));
    dv = W + Dm<D>::WSZ;
    red = dv + Dm<D>::DV;
  }
  static constexpr size_t tbytes(int nm, int nv) {
    return (((size_t)(nm * Dm<D>::MAT + nv * D) * sizeof(T)) + 15) & ~size_t(15);
  }
  static constexpr size_t bytes(int nm, int nv) {
    return tbytes(nm, nv) + (size_t)(Dm<D>::WSZ + Dm<D>::DV + NT / 64) * sizeof(double);
  }
};

constexpr int FOLD_M = 10, FOLD_V = 6;
constexpr int HS_M = 12, HS_V = 8;
constexpr int FIN_M = 6, FIN_V = 3;
constexpr int SB_M = 6, SB_V = 4;
constexpr int PF_M = 3, PF_V = 3;

// ---------------------------------------------------------------------------
// fold: block element of steps s0..s1-1, appending one step at a time:
//   T = F A, mu = F b + b_dyn, U_p = tria([F U, L_Q]);
//   update by omega_t: P11, P21, P22;  w = omega_t - mu, s = P11^{-1} w;
//   G = P11^{-1} T:  eta += G^T s,  Z = tria([Z, G^T])  (J += T^T S^{-1} T);
//   K = P21 P11^{-1}:  A = T - K T,  b = mu + K w,  U = P22;
//   lc += log N(omega_t; mu, S).
// Block 0 starts from the prior (t = 0: mu = m0, U_p = L_0, no x_prev
// dependence, so A, eta, Z stay 0); other blocks start from the identity
// element (A = I).
// ---------------------------------------------------------------------------
template <class T, int D>
__global__ void __launch_bounds__(NT) k_sq_fold(SqArgs<T> P) {
  extern __shared__ unsigned char smem[];
  Carve<T, D> c(smem, FOLD_M, FOLD_V);
  T *sF = c.m[0], *sLQ = c.m[1], *sA = c.m[2], *sU = c.m[3], *sZ = c.m[4], *sT = c.m[5],
    *sG = c.m[6], *sP11 = c.m[7], *sP21 = c.m[8], *sX = c.m[9];
  T *vb = c.v[0], *veta = c.v[1], *vmu = c.v[2], *vw = c.v[3], *vs = c.v[4], *vt = c.v[5];
  const int d = P.d, blk = blockIdx.x, tid = threadIdx.x;
  const int s0 = blk * P.B, s1 = min(P.N, s0 + P.B);
  ld_mat<T, D, false>(sF, P.Fs, D, D);
  ld_mat<T, D>(sLQ, P.LQ, D, D);
  set_eye<T, D>(sA, d, blk == 0 ? T(0) : T(1));
  set_eye<T, D>(sU, d, T(0));
  set_eye<T, D>(sZ, d, T(0));
  if (tid < D) {
    vb[tid] = T(0);
    veta[tid] = T(0);
  }
  __syncthreads();
  double lc = 0.0;
  bool ok = true;
  for (int t = s0; t < s1; ++t) {
    const bool prior = (t == 0);
    const bool dep = (blk != 0);  // the element depends on x_prev
    if (prior) {
      ld_mat<T, D>(sX, P.L0, D, D);
      if (tid < D) vmu[tid] = (tid < d) ? (T)P.m0[tid] : T(0);
      __syncthreads();
    } else {
      if (dep) mm<T, D, false, false>(sT, sF, sA, d);
      mv<T, D, false>(vmu, sF, vb, d);
      if (tid < d && P.b) vmu[tid] += (T)P.b[tid];
      sqrt_predict<T, D>(c.W, c.dv, sF, sU, sLQ, d, sG, sX);
    }
    double lp;
    ok = sqrt_update<T, D>(c.W, c.dv, sX, P.Om + (int64_t)t * d, d, sP11, sP21, sU, vs, vmu,
                           P.om + (int64_t)t * d, c.red, &lp) && ok;
    lc += lp;
    // vw = w = omega - mu (sqrt_update left s = P11^{-1} w in vs)
    if (tid < D) vw[tid] = (tid < d) ? (T)P.om[(int64_t)t * d + tid] - vmu[tid] : T(0);
    __syncthreads();
    if (dep && !prior) {
      cp_mat<T, D>(sG, sT);
      ok = solve_l<T, D>(sG, Dm<D>::LM, 1, sP11, d, d) && ok;  // G = P11^{-1} T
      mv<T, D, true>(veta, sG, vs, d, veta);                   // eta += G^T s
      to_w<T, D, false>(c.W, 0, 0, sZ, d);
      to_w<T, D, true>(c.W, 0, d, sG, d);
      __syncthreads();
      tria<D>(c.W, d, 2 * d, c.dv);
      from_w<T, D>(sZ, c.W, 0, 0, d);
      __syncthreads();
    }
    ok = rows_times_linv<T, D>(sP21, sP11, d, d) && ok;  // K = P21 P11^{-1}
    mv<T, D, false>(vt, sP21, vw, d);
    if (tid < D) vb[tid] = (tid < d) ? vmu[tid] + vt[tid] : T(0);
    __syncthreads();
    if (dep && !prior) {
      mm<T, D, false, false>(sA, sP21, sT, d, sT, T(-1));  // A = T - K T
    }
  }
  if (!ok && tid == 0) flag(P.status);
  T* out = P.el_out + (int64_t)blk * El<D>::SIZE;
  st_mat<T, D>(out + El<D>::A, sA);
  st_mat<T, D>(out + El<D>::U, sU);
  st_mat<T, D>(out + El<D>::Z, sZ);
  if (tid < D) {
    out[El<D>::b + tid] = vb[tid];
    out[El<D>::eta + tid] = veta[tid];
  }
  if (tid == 0) P.lc_out[blk] = lc;
}

// ---------------------------------------------------------------------------
// Hillis-Steele level: out[k] = in[k - s] (x) in[k] for k >= s, else in[k].
// ---------------------------------------------------------------------------
template <class T, int D>
__global__ void __launch_bounds__(NT) k_sq_hs(SqArgs<T> P) {
  extern __shared__ unsigned char smem[];
  const int k = blockIdx.x, tid = threadIdx.x, d = P.d, s = P.hs;
  const T* ej = P.el_in + (int64_t)k * El<D>::SIZE;
  T* out = P.el_out + (int64_t)k * El<D>::SIZE;
  if (k < s) {
    for (int base = 0; base < El<D>::SIZE; base += 8 * NT) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * NT + tid;
        v[u] = e < El<D>::SIZE ? ej[e] : T(0);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = base + u * NT + tid;
        if (e < El<D>::SIZE) out[e] = v[u];
      }
    }
    if (tid == 0) P.lc_out[k] = P.lc_in[k];
    return;
  }
  const T* ei = P.el_in + (int64_t)(k - s) * El<D>::SIZE;
  Carve<T, D> c(smem, HS_M, HS_V);
  T *Ui = c.m[0], *Zj = c.m[1], *Ai = c.m[2], *Aj = c.m[3], *Uj = c.m[4], *Zi = c.m[5],
    *X11 = c.m[6], *X21 = c.m[7], *X22 = c.m[8], *G = c.m[9], *Mm = c.m[10], *Tm = c.m[11];
  T *bi = c.v[0], *eti = c.v[1], *bj = c.v[2], *etj = c.v[3], *vc = c.v[4], *v1 = c.v[5],
    *v2 = c.v[6], *v3 = c.v[7];
  ld_mat<T, D, false>(Ui, ei + El<D>::U, D, D);
  ld_mat<T, D, false>(Zj, ej + El<D>::Z, D, D);
  ld_mat<T, D, false>(Ai, ei + El<D>::A, D, D);
  ld_mat<T, D, false>(Aj, ej + El<D>::A, D, D);
  ld_mat<T, D, false>(Uj, ej + El<D>::U, D, D);
  ld_mat<T, D>(Zi, ei + El<D>::Z, D, D);
  if (tid < D) {
    bi[tid] = ei[El<D>::b + tid];
    eti[tid] = ei[El<D>::eta + tid];
    bj[tid] = ej[El<D>::b + tid];
    etj[tid] = ej[El<D>::eta + tid];
  }
  __syncthreads();
  bool ok = true;
  // tria([[U_i^T Z_j, I], [Z_j, 0]])
  mm<T, D, true, false>(Tm, Ui, Zj, d);
  to_w<T, D, false>(c.W, 0, 0, Tm, d);
  w_fill<D>(c.W, 0, d, d, 1.0);
  to_w<T, D, false>(c.W, d, 0, Zj, d);
  w_fill<D>(c.W, d, d, d, 0.0);
  __syncthreads();
  tria<D>(c.W, 2 * d, 2 * d, c.dv);
  from_w<T, D>(X11, c.W, 0, 0, d);
  from_w<T, D>(X21, c.W, d, 0, d);
  from_w<T, D>(X22, c.W, d, d, d);
  __syncthreads();
  cp_mat<T, D>(G, Ui);
  ok = rows_times_linvT<T, D>(G, X11, d, d) && ok;  // G = U_i X11^{-T}
  mm<T, D, false, true>(Mm, G, X21, d);
  for (int e = tid; e < D * D; e += NT) {
    const int i = e / D, j = e % D;
    const T v = (i == j && i < d) ? T(1) : T(0);
    Mm[i * Dm<D>::LM + j] = v - Mm[i * Dm<D>::LM + j];
  }
  __syncthreads();
  // c = eta_j - Z_j Z_j^T b_i;  h = X11^{-1} U_i^T c
  mv<T, D, true>(v1, Zj, bi, d);
  mv<T, D, false>(vc, Zj, v1, d, etj, T(-1));
  mv<T, D, true>(v2, Ui, vc, d);
  ok = solve_l<T, D>(v2, 1, 0, X11, 1, d) && ok;
  double lc = P.lc_in[k - s] + P.lc_in[k] - logdiag<T, D>(X11, d, c.red);
  if (tid < D) v3[tid] = etj[tid] + vc[tid];
  __syncthreads();
  lc += 0.5 * dot<T, D>(bi, v3, d, c.red) + 0.5 * dot<T, D>(v2, v2, d, c.red);
  // A = A_j M A_i
  mm<T, D, false, false>(Tm, Mm, Ai, d);
  mm<T, D, false, false>(X21, Aj, Tm, d);  // X21 is free now
  st_mat<T, D>(out + El<D>::A, X21);
  // b = A_j M (b_i + U_i U_i^T eta_j) + b_j
  mv<T, D, true>(v1, Ui, etj, d);
  mv<T, D, false>(v2, Ui, v1, d, bi);
  mv<T, D, false>(v3, Mm, v2, d);
  mv<T, D, false>(v1, Aj, v3, d, bj);
  if (tid < D) out[El<D>::b + tid] = v1[tid];
  // eta = A_i^T M^T c + eta_i
  mv<T, D, true>(v2, Mm, vc, d);
  mv<T, D, true>(v3, Ai, v2, d, eti);
  if (tid < D) out[El<D>::eta + tid] = v3[tid];
  // U = tria([A_j G, U_j])
  mm<T, D, false, false>(Tm, Aj, G, d);
  to_w<T, D, false>(c.W, 0, 0, Tm, d);
  to_w<T, D, false>(c.W, 0, d, Uj, d);
  __syncthreads();
  tria<D>(c.W, d, 2 * d, c.dv);
  from_w<T, D>(Tm, c.W, 0, 0, d);
  __syncthreads();
  st_mat<T, D>(out + El<D>::U, Tm);
  // Z = tria([A_i^T X22, Z_i])
  mm<T, D, true, false>(G, Ai, X22, d);
  to_w<T, D, false>(c.W, 0, 0, G, d);
  to_w<T, D, false>(c.W, 0, d, Zi, d);
  __syncthreads();
  tria<D>(c.W, d, 2 * d, c.dv);
  from_w<T, D>(Tm, c.W, 0, 0, d);
  __syncthreads();
  st_mat<T, D>(out + El<D>::Z, Tm);
  if (tid == 0) {
    P.lc_out[k] = lc;
    if (!ok) flag(P.status);
  }
}

// ---------------------------------------------------------------------------
// re-scan: each block runs a square-root Kalman filter over its steps from the
// filtering moments entering it (block 0: the prior at t = 0):
//   predict  m_p = F m + b_dyn, U_p = tria([F U, L_Q]);
//   update   P11, P21, P22;  s = P11^{-1} (omega - m_p);  m = m_p + P21 s;  U = P22;
//   ell_t = -1/2 (d log 2 pi + 2 sum log diag P11 + s^T s).
// ---------------------------------------------------------------------------
template <class T, int D>
__global__ void __launch_bounds__(NT) k_sq_final(SqArgs<T> P) {
  extern __shared__ unsigned char smem[];
  Carve<T, D> c(smem, FIN_M, FIN_V);
  T *sF = c.m[0], *sLQ = c.m[1], *sU = c.m[2], *sP11 = c.m[3], *sP21 = c.m[4], *sX = c.m[5];
  T *vm = c.v[0], *vmp = c.v[1], *vs = c.v[2];
  const int d = P.d, blk = blockIdx.x, tid = threadIdx.x;
  const int s0 = blk * P.B, s1 = min(P.N, s0 + P.B);
  ld_mat<T, D, false>(sF, P.Fs, D, D);
  ld_mat<T, D>(sLQ, P.LQ, D, D);
  if (blk > 0) {
    const T* pre = P.el_in + (int64_t)(blk - 1) * El<D>::SIZE;  // prefix through block blk-1
    ld_mat<T, D>(sU, pre + El<D>::U, D, D);
    if (tid < D) vm[tid] = pre[El<D>::b + tid];
  } else {
    set_eye<T, D>(sU, d, T(0));
    if (tid < D) vm[tid] = T(0);
  }
  __syncthreads();
  bool ok = true;
  for (int t = s0; t < s1; ++t) {
    if (t == 0) {
      ld_mat<T, D>(sX, P.L0, D, D);
      if (tid < D) vmp[tid] = (tid < d) ? (T)P.m0[tid] : T(0);
      __syncthreads();
    } else {
      mv<T, D, false>(vmp, sF, vm, d);
      if (tid < d && P.b) vmp[tid] += (T)P.b[tid];
      sqrt_predict<T, D>(c.W, c.dv, sF, sU, sLQ, d, sP21, sX);
    }
    double lp;
    ok = sqrt_update<T, D>(c.W, c.dv, sX, P.Om + (int64_t)t * d, d, sP11, sP21, sU, vs, vmp,
                           P.om + (int64_t)t * d, c.red, &lp) && ok;
    mv<T, D, false>(vm, sP21, vs, d, vmp);
    // outputs: means and factors (boundary arrays in double, the sampler's copy in T)
    if (tid < d) {
      P.mf[(int64_t)t * d + tid] = (double)vm[tid];
    }
    if (tid < D) P.mfT[(int64_t)t * D + tid] = vm[tid];
    st_mat<T, D>(P.UfT + (int64_t)t * D * D, sU);
    if (P.Uf)
      for (int e = tid; e < d * d; e += NT)
        P.Uf[(int64_t)t * d * d + e] = (double)sU[(e / d) * Dm<D>::LM + e % d];
    if (tid == 0) P.ell[t] = lp;
    __syncthreads();
  }
  if (!ok && tid == 0) flag(P.status);
}

// ---------------------------------------------------------------------------
// sampler elements, one team per t:
//   tria([[L_Q, F U^f_t], [0, U^f_t]]) -> P11 (factor of P^p_{t+1}), P21, P22;
//   E_t = P21 P11^{-1},  U_t = m^f_t - E_t (F m^f_t + b_dyn) + P22 xi_t;
// the last step: E = 0, U = m^f + U^f xi.
// ---------------------------------------------------------------------------
template <class T, int D>
__global__ void __launch_bounds__(NT) k_sq_sbuild(SqArgs<T> P) {
  extern __shared__ unsigned char smem[];
  Carve<T, D> c(smem, SB_M, SB_V);
  T *sF = c.m[0], *sLQ = c.m[1], *sU = c.m[2], *sP11 = c.m[3], *sP21 = c.m[4], *sX = c.m[5];
  T *vm = c.v[0], *vmp = c.v[1], *vxi = c.v[2], *vo = c.v[3];
  const int d = P.d, t = blockIdx.x, tid = threadIdx.x;
  ld_mat<T, D>(sU, P.UfT + (int64_t)t * D * D, D, D);
  if (tid < D) {
    vm[tid] = P.mfT[(int64_t)t * D + tid];
    vxi[tid] = (tid < d) ? (T)P.xi[(int64_t)t * d + tid] : T(0);
  }
  __syncthreads();
  T* Eo = P.E + (int64_t)t * D * D;
  if (t == P.N - 1) {
    mv<T, D, false>(vo, sU, vxi, d, vm);
    for (int e = tid; e < D * D; e += NT) Eo[e] = T(0);
    if (tid < D) P.Ut[(int64_t)t * D + tid] = vo[tid];
    return;
  }
  ld_mat<T, D, false>(sF, P.Fs, D, D);
  ld_mat<T, D>(sLQ, P.LQ, D, D);
  mm<T, D, false, false>(sX, sF, sU, d);
  to_w<T, D, false>(c.W, 0, 0, sLQ, d);
  to_w<T, D, false>(c.W, 0, d, sX, d);
  w_fill<D>(c.W, d, 0, d, 0.0);
  to_w<T, D, false>(c.W, d, d, sU, d);
  __syncthreads();
  tria<D>(c.W, 2 * d, 2 * d, c.dv);
  from_w<T, D>(sP11, c.W, 0, 0, d);
  from_w<T, D>(sP21, c.W, d, 0, d);
  from_w<T, D>(sX, c.W, d, d, d);
  __syncthreads();
  const bool ok = rows_times_linv<T, D>(sP21, sP11, d, d);  // E = P21 P11^{-1}
  mv<T, D, false>(vmp, sF, vm, d);
  if (tid < d && P.b) vmp[tid] += (T)P.b[tid];
  __syncthreads();
  mv<T, D, false>(vo, sP21, vmp, d, vm, T(-1));  // g = m - E m_p
  mv<T, D, false>(vmp, sX, vxi, d, vo);          // U = g + chol(L) xi
  st_mat<T, D>(Eo, sP21);
  if (tid < D) P.Ut[(int64_t)t * D + tid] = vmp[tid];
  if (!ok && tid == 0) flag(P.status);
}

// per block: suffix aggregate (E_a, U_a) = e_s0 o ... o e_{s1-1}, with
// (E_i, U_i) o (E_j, U_j) = (E_i E_j, E_i U_j + U_i)
template <class T, int D>
__global__ void __launch_bounds__(NT) k_sq_pfold(SqArgs<T> P) {
  extern __shared__ unsigned char smem[];
  Carve<T, D> c(smem, PF_M, PF_V);
  T *Ea = c.m[0], *Et = c.m[1], *Tm = c.m[2];
  T *ua = c.v[0], *ut = c.v[1], *tv = c.v[2];
  const int d = P.d, blk = blockIdx.x, tid = threadIdx.x;
  const int s0 = blk * P.B, s1 = min(P.N, s0 + P.B);
  ld_mat<T, D>(Ea, P.E + (int64_t)(s1 - 1) * D * D, D, D);
  if (tid < D) ua[tid] = P.Ut[(int64_t)(s1 - 1) * D + tid];
  __syncthreads();
  for (int t = s1 - 2; t >= s0; --t) {
    ld_mat<T, D>(Et, P.E + (int64_t)t * D * D, D, D);
    if (tid < D) ut[tid] = P.Ut[(int64_t)t * D + tid];
    __syncthreads();
    mm<T, D, false, false>(Tm, Et, Ea, d);
    mv<T, D, false>(tv, Et, ua, d, ut);
    cp_mat<T, D>(Ea, Tm);
    if (tid < D) ua[tid] = tv[tid];
    __syncthreads();
  }
  T* o = P.agg + (int64_t)blk * (D * D + D);
  st_mat<T, D>(o, Ea);
  if (tid < D) o[D * D + tid] = ua[tid];
}

// one team, blocks from last to first: the state entering block k from the
// right (x*_{s1}) is xin[k]; x*_{s0} = E_a x + U_a
template <class T, int D>
__global__ void __launch_bounds__(NT) k_sq_pscan(SqArgs<T> P) {
  extern __shared__ unsigned char smem[];
  Carve<T, D> c(smem, PF_M, PF_V);
  T *Ea = c.m[0];
  T *x = c.v[0], *y = c.v[1], *ua = c.v[2];
  const int d = P.d, tid = threadIdx.x;
  if (tid < D) x[tid] = T(0);
  __syncthreads();
  for (int k = P.nb - 1; k >= 0; --k) {
    const T* a = P.agg + (int64_t)k * (D * D + D);
    if (tid < D) P.xin[(int64_t)k * D + tid] = x[tid];
    ld_mat<T, D>(Ea, a, D, D);
    if (tid < D) ua[tid] = a[D * D + tid];
    __syncthreads();
    mv<T, D, false>(y, Ea, x, d, ua);
    if (tid < D) x[tid] = y[tid];
    __syncthreads();
  }
}

// per block: x*_t = E_t x*_{t+1} + U_t from the state entering on the right
template <class T, int D>
__global__ void __launch_bounds__(NT) k_sq_pfinal(SqArgs<T> P) {
  extern __shared__ unsigned char smem[];
  Carve<T, D> c(smem, PF_M, PF_V);
  T* Et = c.m[0];
  T *x = c.v[0], *y = c.v[1], *ut = c.v[2];
  const int d = P.d, blk = blockIdx.x, tid = threadIdx.x;
  const int s0 = blk * P.B, s1 = min(P.N, s0 + P.B);
  if (tid < D) x[tid] = P.xin[(int64_t)blk * D + tid];
  __syncthreads();
  for (int t = s1 - 1; t >= s0; --t) {
    ld_mat<T, D>(Et, P.E + (int64_t)t * D * D, D, D);
    if (tid < D) ut[tid] = P.Ut[(int64_t)t * D + tid];
    __syncthreads();
    mv<T, D, false>(y, Et, x, d, ut);
    if (tid < d) P.xs[(int64_t)t * d + tid] = (double)y[tid];
    if (tid < D) x[tid] = y[tid];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <class T, int D>
hipError_t set_limits() {
  hipError_t e;
  const int lim[] = {(int)Carve<T, D>::bytes(FOLD_M, FOLD_V), (int)Carve<T, D>::bytes(HS_M, HS_V),
                     (int)Carve<T, D>::bytes(FIN_M, FIN_V), (int)Carve<T, D>::bytes(SB_M, SB_V),
                     (int)Carve<T, D>::bytes(PF_M, PF_V)};
  if ((e = hipFuncSetAttribute((const void*)k_sq_fold<T, D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lim[0])) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_sq_hs<T, D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lim[1])) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_sq_final<T, D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, lim[2])) != hipSuccess)
    return e;
  return hipFuncSetAttribute((const void*)k_sq_sbuild<T, D>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, lim[3]);
}

hipError_t set_limits_all() {
  hipError_t e;
  if ((e = set_limits<float, 16>()) != hipSuccess) return e;
  if ((e = set_limits<float, 32>()) != hipSuccess) return e;
  if ((e = set_limits<double, 16>()) != hipSuccess) return e;
  return set_limits<double, 32>();
}

struct SqLayout {
  int D, B, nb;
  size_t LQ, L0, Fs, el[2], lc[2], mfT, UfT, E, Ut, agg, xin, ell, status, total;
};

inline size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

void sq_layout(SqLayout& L, int N, int d, int block, size_t tsz) {
  L.D = d <= 16 ? 16 : 32;
  L.B = block > 0 ? block : std::max(4, (N + 255) / 256);
  L.nb = (N + L.B - 1) / L.B;
  const size_t DD = (size_t)L.D * L.D, ES = 3 * DD + 2 * L.D;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = up256(o + bytes);
    return at;
  };
  L.LQ = take(DD * tsz);
  L.L0 = take(DD * tsz);
  L.Fs = take(DD * tsz);
  L.el[0] = take(L.nb * ES * tsz);
  L.el[1] = take(L.nb * ES * tsz);
  L.lc[0] = take(L.nb * sizeof(double));
  L.lc[1] = take(L.nb * sizeof(double));
  L.mfT = take((size_t)N * L.D * tsz);
  L.UfT = take((size_t)N * DD * tsz);
  L.E = take((size_t)N * DD * tsz);
  L.Ut = take((size_t)N * L.D * tsz);
  L.agg = take(L.nb * (DD + L.D) * tsz);
  L.xin = take(L.nb * (size_t)L.D * tsz);
  L.ell = take((size_t)N * sizeof(double));
  L.status = take(2 * sizeof(int));
  L.total = o;
}

template <class T>
T* atp(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

template <class T, int D>
akf_status run(const akf_model* m, const SqLayout& L, const double* om, const double* Om,
               const double* xi, double* xs, double* mf, double* Uf, double* ell, double* logZ,
               int32_t* status, void* ws, hipStream_t st) {
  SqArgs<T> P{};
  P.N = m->N;
  P.d = m->dx;
  P.B = L.B;
  P.nb = L.nb;
  P.m0 = m->m0;
  P.F = m->F;
  P.b = m->b;
  P.Q = m->Q;
  P.P0 = m->P0;
  P.om = om;
  P.Om = Om;
  P.xi = xi;
  P.Fs = atp<T>(ws, L.Fs);
  P.LQ = atp<T>(ws, L.LQ);
  P.L0 = atp<T>(ws, L.L0);
  P.mfT = atp<T>(ws, L.mfT);
  P.UfT = atp<T>(ws, L.UfT);
  P.E = atp<T>(ws, L.E);
  P.Ut = atp<T>(ws, L.Ut);
  P.agg = atp<T>(ws, L.agg);
  P.xin = atp<T>(ws, L.xin);
  P.mf = mf;
  P.Uf = Uf;
  P.ell = ell ? ell : atp<double>(ws, L.ell);
  P.xs = xs;
  P.status = atp<int>(ws, L.status);
  akf_status s;
  k_sq_init<<<dim3(1), dim3(64), 0, st>>>(P.status);
  k_sq_prep<T, D><<<dim3(1), dim3(NT), 0, st>>>(P);
  P.el_out = atp<T>(ws, L.el[0]);
  P.lc_out = atp<double>(ws, L.lc[0]);
  k_sq_fold<T, D><<<dim3(L.nb), dim3(NT), Carve<T, D>::bytes(FOLD_M, FOLD_V), st>>>(P);
  int cur = 0;
  for (int sdist = 1; sdist < L.nb; sdist *= 2) {
    P.el_in = atp<T>(ws, L.el[cur]);
    P.lc_in = atp<double>(ws, L.lc[cur]);
    P.el_out = atp<T>(ws, L.el[1 - cur]);
    P.lc_out = atp<double>(ws, L.lc[1 - cur]);
    P.hs = sdist;
    k_sq_hs<T, D><<<dim3(L.nb), dim3(NT), Carve<T, D>::bytes(HS_M, HS_V), st>>>(P);
    cur = 1 - cur;
  }
  P.el_in = atp<T>(ws, L.el[cur]);
  P.lc_in = atp<double>(ws, L.lc[cur]);
  k_sq_final<T, D><<<dim3(L.nb), dim3(NT), Carve<T, D>::bytes(FIN_M, FIN_V), st>>>(P);
  if ((s = hip_check(hipGetLastError(), "square-root filter launch")) != AKF_OK) return s;
  if (logZ && (s = hip_check(launch_sum(P.ell, P.N, logZ, P.status, st), "sum launch")) != AKF_OK)
    return s;
  if (xs) {
    k_sq_sbuild<T, D><<<dim3(P.N), dim3(NT), Carve<T, D>::bytes(SB_M, SB_V), st>>>(P);
    k_sq_pfold<T, D><<<dim3(L.nb), dim3(NT), Carve<T, D>::bytes(PF_M, PF_V), st>>>(P);
    k_sq_pscan<T, D><<<dim3(1), dim3(NT), Carve<T, D>::bytes(PF_M, PF_V), st>>>(P);
    k_sq_pfinal<T, D><<<dim3(L.nb), dim3(NT), Carve<T, D>::bytes(PF_M, PF_V), st>>>(P);
    if ((s = hip_check(hipGetLastError(), "square-root sampler launch")) != AKF_OK) return s;
  }
  if (status)
    return hip_check(hipMemcpyAsync(status, P.status, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy");
  return AKF_OK;
}

}  // namespace sq
}  // namespace akf

using namespace akf;

extern "C" {

size_t akf_sqrt_workspace_bytes(const akf_model* model, int32_t block) {
  if (check_model(model, false, true) != AKF_OK || model->dx > 32 || block < 0 ||
      check_linear(model, "the square-root filter") != AKF_OK)
    return 0;
  sq::SqLayout L;
  sq::sq_layout(L, model->N, model->dx, block,
                model->dtype == AKF_F32 ? sizeof(float) : sizeof(double));
  return L.total;
}

akf_status akf_sqrt_filter_sample(const akf_model* model, const double* om, const double* Om,
                                  const double* xi, double* x_out, double* mf, double* Uf,
                                  double* ell, double* logZ, int32_t* status, void* ws,
                                  size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_model(model, false, true)) != AKF_OK) return s;
  if ((s = check_linear(model, "the square-root filter")) != AKF_OK) return s;
  if (model->dx > 32)
    return fail(AKF_ERR_SHAPE, "the square-root filter takes dx <= 32 (got %d)", model->dx);
  if (!om || !Om || !mf) return fail(AKF_ERR_INVALID, "om, Om and mf must be non-NULL");
  if (x_out && !xi) return fail(AKF_ERR_INVALID, "a path sample (x_out) needs xi");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  sq::SqLayout L;
  const bool f32 = model->dtype == AKF_F32;
  sq::sq_layout(L, model->N, model->dx, block, f32 ? sizeof(float) : sizeof(double));
  if (!ws) return fail(AKF_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(AKF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total)
    return fail(AKF_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  static std::once_flag once;
  static hipError_t lim_err = hipSuccess;
  std::call_once(once, [] { lim_err = sq::set_limits_all(); });
  if (lim_err != hipSuccess)
    return fail(AKF_ERR_HIP, "setting LDS limits failed: %s", hipGetErrorString(lim_err));
  hipStream_t st = (hipStream_t)stream;
  if (f32)
    return L.D == 16 ? sq::run<float, 16>(model, L, om, Om, xi, x_out, mf, Uf, ell, logZ, status,
                                          ws, st)
                     : sq::run<float, 32>(model, L, om, Om, xi, x_out, mf, Uf, ell, logZ, status,
                                          ws, st);
  return L.D == 16 ? sq::run<double, 16>(model, L, om, Om, xi, x_out, mf, Uf, ell, logZ, status,
                                         ws, st)
                   : sq::run<double, 32>(model, L, om, Om, xi, x_out, mf, Uf, ell, logZ, status,
                                         ws, st);
}

}  // extern "C"
