// akf_dyn.hip -- nonlinear dynamics x_t = f(x_{t-1}) + N(0, Q), with f one
// Euler-Maruyama step x + dt beta(x) of the Lorenz-63 or Lorenz-96 SDE.
//
// Each MH step linearises f around the current path (Alg. "General Auxiliary
// Kalman sampler", dynamics line; Example "gslr-example", extended
// linearisation): F_t = J(a_{t-1}), b_t = f(a_{t-1}) - F_t a_{t-1}, which the
// filter and sampler kernels read per step.  The reverse linearisation (at x*)
// also forms the terms of log r that no longer cancel:
//   sum_{t>=1} [log N(x*_t; f(x*_{t-1}), Q) - log N(x*_t; F^x_t x*_{t-1} + b^x_t, Q)]
// - sum_{t>=1} [log N(x_t;  f(x_{t-1}),  Q) - log N(x_t;  F^x*_t x_{t-1} + b^x*_t, Q)].
// One wave per time step (lane i = coordinate i), DW waves per workgroup.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "akf_internal.h"
#include "akf_team.hpp"

namespace akf {

namespace {

constexpr int DW = 4;

__device__ __forceinline__ double dyn_dt(const KModel& M) {
  return M.dyn == DYN_LORENZ63 ? M.dyn_par[3] : M.dyn_par[1];
}

// drift beta_i(x), x in LDS
__device__ __forceinline__ double dyn_beta(const KModel& M, const double* x, int i) {
  if (M.dyn == DYN_LORENZ63) {
    const double t1 = M.dyn_par[0], t2 = M.dyn_par[1], t3 = M.dyn_par[2];
    if (i == 0) return t1 * (x[1] - x[0]);
    if (i == 1) return t2 * x[0] - x[1] - x[0] * x[2];
    return x[0] * x[1] - t3 * x[2];
  }
  const int d = M.d;
  const int ip = (i + 1) % d, im = (i + d - 1) % d, im2 = (i + d - 2) % d;
  return (x[ip] - x[im2]) * x[im] - x[i] + M.dyn_par[0];
}

// d beta_i / d x_j
__device__ __forceinline__ double dyn_dbeta(const KModel& M, const double* x, int i, int j) {
  if (M.dyn == DYN_LORENZ63) {
    const double t1 = M.dyn_par[0], t2 = M.dyn_par[1], t3 = M.dyn_par[2];
    if (i == 0) return j == 0 ? -t1 : (j == 1 ? t1 : 0.0);
    if (i == 1) return j == 0 ? t2 - x[2] : (j == 1 ? -1.0 : -x[0]);
    return j == 0 ? x[1] : (j == 1 ? x[0] : -t3);
  }
  const int d = M.d;
  const int ip = (i + 1) % d, im = (i + d - 1) % d, im2 = (i + d - 2) % d;
  double v = 0.0;
  if (j == ip) v += x[im];
  if (j == im2) v -= x[im];
  if (j == im) v += x[ip] - x[im2];
  if (j == i) v -= 1.0;
  return v;
}

// (J(x) w)_i with J = I + dt d beta / dx
__device__ __forceinline__ double dyn_jvp(const KModel& M, const double* x, const double* w,
                                          int i) {
  double s = 0.0;
  if (M.dyn == DYN_LORENZ63) {
    for (int j = 0; j < 3; ++j) s += dyn_dbeta(M, x, i, j) * w[j];
  } else {
    const int d = M.d;
    const int ip = (i + 1) % d, im = (i + d - 1) % d, im2 = (i + d - 2) % d;
    s = x[im] * (w[ip] - w[im2]) + (x[ip] - x[im2]) * w[im] - w[i];
  }
  return w[i] + dyn_dt(M) * s;
}

__global__ void __launch_bounds__(64 * DW) k_dyn_lin(KModel M, DynArgs A) {
  __shared__ double sQ[64 * 64];
  __shared__ double sa[DW][64], sz[DW][64], sdel[DW][64], sp1[DW][64], sp2[DW][64];
  __shared__ double sh2[DW][64];
  __shared__ double red[DW];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, d = M.d;
  const int t = blockIdx.x * DW + w;
  const bool active = t >= 1 && t < M.N;
  const bool mis = A.z != nullptr;
  if (mis)
    team_move<64 * DW, 64 * 64>(
        d * d, [&](int e) { return A.Qinv[e]; },
        [&](int e, double v) { sQ[(e / d) * 64 + e % d] = v; });
  if (lane < 64) {
    sa[w][lane] = (active && lane < d) ? A.a[(int64_t)(t - 1) * d + lane] : 0.0;
    sz[w][lane] = (active && mis && lane < d) ? A.z[(int64_t)(t - 1) * d + lane] : 0.0;
    sdel[w][lane] = sa[w][lane] - sz[w][lane];
  }
  __syncthreads();
  const double dt = dyn_dt(M);
  double term = 0.0;
  if (active) {
    // F_t, coalesced over its d*d entries
    double* Ft = A.Ft + (int64_t)t * d * d;
    for (int e = lane; e < d * d; e += 64) {
      const int i = e / d, j = e % d;
      Ft[e] = (i == j ? 1.0 : 0.0) + dt * dyn_dbeta(M, sa[w], i, j);
    }
    double f = 0.0;
    if (lane < d) {
      f = sa[w][lane] + dt * dyn_beta(M, sa[w], lane);
      A.bt[(int64_t)t * d + lane] = f - dyn_jvp(M, sa[w], sa[w], lane);
    }
    if (mis && lane < d) {
      // a = x*, z = x: r1 = x*_t - f(x*_{t-1}), r2 = x*_t - f(x_{t-1}) - J(x_{t-1})(x*_{t-1} - x_{t-1}),
      // r3 = x_t - f(x_{t-1}), r4 = x_t - f(x*_{t-1}) + J(x*_{t-1})(x*_{t-1} - x_{t-1})
      const double fz = sz[w][lane] + dt * dyn_beta(M, sz[w], lane);
      const double at = A.a[(int64_t)t * d + lane], zt = A.z[(int64_t)t * d + lane];
      const double r1 = at - f;
      const double r2 = at - fz - dyn_jvp(M, sz[w], sdel[w], lane);
      const double r3 = zt - fz;
      const double r4 = zt - f + dyn_jvp(M, sa[w], sdel[w], lane);
      sp1[w][lane] = r1 + r2;
      sp2[w][lane] = r3 + r4;
      term = -0.5 * (r1 - r2);  // times (Q^{-1} p1)_i below
      sh2[w][lane] = 0.5 * (r3 - r4);
    } else if (mis) {
      sp1[w][lane] = 0.0;
      sp2[w][lane] = 0.0;
    }
  } else if (mis) {
    sp1[w][lane] = 0.0;
    sp2[w][lane] = 0.0;
  }
  if (!mis) return;
  __syncthreads();
  double part = 0.0;
  if (active && lane < d) {
    double q1 = 0.0, q2 = 0.0;
    for (int j = 0; j < d; ++j) {
      const double qij = sQ[j * 64 + lane];  // Q^{-1} is symmetric
      q1 += qij * sp1[w][j];
      q2 += qij * sp2[w][j];
    }
    part = term * q1 + sh2[w][lane] * q2;
  }
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
  if (lane == 0) red[w] = part;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int k = 0; k < DW; ++k) s += red[k];
    A.part[blockIdx.x] = s;
  }
}

// Q^{-1} by in-place Gauss-Jordan elimination in LDS (Q symmetric positive
// definite, no pivoting), symmetrised.  One workgroup of 64 threads, thread j
// owns column j; at step k the unit column k takes the place of column k.
__global__ void __launch_bounds__(64) k_qinv(KModel M, double* Qinv) {
  constexpr int LD = 65;
  __shared__ double sA[64 * LD], colk[64];
  const int tid = threadIdx.x, d = M.d;
  for (int e = tid; e < d * d; e += 64) sA[(e / d) * LD + e % d] = M.Q[e];
  __syncthreads();
  for (int k = 0; k < d; ++k) {
    if (tid < d) colk[tid] = sA[tid * LD + k];
    __syncthreads();
    const double inv = 1.0 / colk[k];
    if (tid < d) {
      const double akj = (tid == k ? 1.0 : sA[k * LD + tid]) * inv;
      for (int i = 0; i < d; ++i) {
        if (i == k) continue;
        sA[i * LD + tid] = (tid == k ? 0.0 : sA[i * LD + tid]) - colk[i] * akj;
      }
      sA[k * LD + tid] = akj;
    }
    __syncthreads();
  }
  for (int e = tid; e < d * d; e += 64) {
    const int i = e / d, j = e % d;
    Qinv[e] = 0.5 * (sA[i * LD + j] + sA[j * LD + i]);
  }
}

}  // namespace

hipError_t launch_qinv(const KModel& M, double* Qinv, hipStream_t st) {
  hipLaunchKernelGGL(k_qinv, dim3(1), dim3(64), 0, st, M, Qinv);
  return hipGetLastError();
}

hipError_t launch_dyn_lin(const KModel& M, DynArgs A, int* n_part, hipStream_t st) {
  const int nblk = (M.N + DW - 1) / DW;
  if (n_part) *n_part = nblk;
  timing_mark(FAM_LIN, 1, st);
  hipLaunchKernelGGL(k_dyn_lin, dim3(nblk), dim3(64 * DW), 0, st, M, A);
  timing_mark(FAM_LIN, 0, st);
  return hipGetLastError();
}

}  // namespace akf
