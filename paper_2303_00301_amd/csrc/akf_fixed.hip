// akf_fixed.hip -- MH steps whose auxiliary model keeps the same covariances
// from step to step.
//
// Under first-order proposals Omega_t = delta/2 I for every t and every path
// (eq. gaussian-FK-proposal with Sigma_t = I), so every covariance of the
// auxiliary LGSSM -- P^p_t, P^f_t, S_t, the sampler's E_t and L_t -- is the same
// at every step and for the forward and reverse proposals alike: they depend on
// the path only through Omega_t.  A run forms them once (the full filter and
// sampler element build, keeping S_t^{-1}, log det S_t, E_t and chol(L_t)); each
// proposal then needs matrix-vector work only:
//   cmean : c_t = omega_t - Omega S_t^{-1} (omega_t - b) (t = 0: with m0), so
//           that m^f_t = Phi_t m^f_{t-1} + c_t with Phi_t = Omega S_t^{-1} F;
//   scan  : that affine recursion, run in reversed time through the pathwise
//           sampler's suffix scan (Phi_0 = 0 is its terminal element);
//   ell   : ell_t = log N(omega_t; F m^f_{t-1} + b, S_t) from S_t^{-1} and
//           log det S_t, and for the forward proposal the sampler elements
//           U_t = m^f_t - E_t (F m^f_t + b) + chol(L_t) xi_t.
// One team per time step.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "akf_team.hpp"
#include "akf_internal.h"

namespace akf {

namespace {

constexpr double LOG2PI_X = 1.8378770664093454835606594728112;

template <int D>
__device__ __forceinline__ void xload_pad(double* s, const double* __restrict__ g) {
  for (int e = threadIdx.x; e < D * D; e += Cfg<D>::NT) s[(e / D) * Cfg<D>::LD + (e % D)] = g[e];
}

template <int D>
__device__ __forceinline__ void xload_user(double* s, const double* __restrict__ g, int d) {
  for (int e = threadIdx.x; e < D * D; e += Cfg<D>::NT) {
    const int i = e / D, j = e % D;
    s[i * Cfg<D>::LD + j] = (i < d && j < d) ? g[i * d + j] : 0.0;
  }
}

// LDS doubles of each kernel: phi two matrices; cmean one matrix and two
// vectors; ell two matrices and its vectors, two more matrices with the
// sampler elements
template <int D>
constexpr int lds_phi() {
  return 2 * Cfg<D>::MAT;
}
template <int D>
constexpr int lds_cmean() {
  return Cfg<D>::MAT + 2 * D;
}
template <int D>
constexpr int lds_ell(bool samp) {
  return (samp ? 4 : 2) * Cfg<D>::MAT + 8 * D + 16;
}

// Phi_t = Omega S_t^{-1} F, stored at reversed index N - 1 - t; Phi_0 = 0.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_fixed_phi(KModel M, FixedArgs A) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  const int t = blockIdx.x, d = M.d;
  double* out = A.Ephi + (int64_t)(M.N - 1 - t) * D * D;
  RM<D> R;
  if (t == 0) {
    rm_zero<D>(R);
    rm_store<D>(R, out, D, D);
    return;
  }
  xload_pad<D>(B1, A.Sinv + (int64_t)t * D * D);
  xload_user<D>(B2, M.F, d);
  team_sync();
  gemm<D, false, false, false>(R, B1, B2);  // S^{-1} F
#pragma unroll
  for (int q = 0; q < Cfg<D>::TPW; ++q) R.t[q] *= A.ovar;
  rm_store<D>(R, out, D, D);
}

// c_t (reversed index) from this proposal's pseudo-observations.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_fixed_cmean(KModel M, FixedArgs A) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* vw = B1 + C::MAT;
  double* vv = vw + D;
  const int t = blockIdx.x, tid = threadIdx.x, d = M.d;
  if (t == 0 && tid == 0 && *A.setup_status) atomicOr(A.status, *A.setup_status);
  xload_pad<D>(B1, A.Sinv + (int64_t)t * D * D);
  const double* om = A.om + (int64_t)t * d;
  if (tid < D) {
    const double mu = (tid < d) ? (t == 0 ? M.m0[tid] : (M.b ? M.b[tid] : 0.0)) : 0.0;
    vw[tid] = (tid < d) ? om[tid] - mu : 0.0;
  }
  team_sync();
  matvec<D, false>(vv, B1, vw);  // S^{-1} (omega - mu)
  if (tid < D) A.U[(int64_t)(M.N - 1 - t) * D + tid] = (tid < d) ? om[tid] - A.ovar * vv[tid] : 0.0;
}

// ell_t, and (with xi_x) the sampler elements U_t.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_fixed_ell(KModel M, FixedArgs A) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* sF = lds;
  double* B1 = sF + C::MAT;
  double* vm = B1 + C::MAT;  // m^f_t
  double* vq = vm + D;       // m^f_{t-1}
  double* vp = vq + D;       // m^p_t, then F m^f_t + b
  double* vr = vp + D;       // residual
  double* vs = vr + D;       // S^{-1} r
  double* vx = vs + D;       // xi_t
  double* vu = vx + D;
  double* vb = vu + D;       // b, zero-padded
  double* red = vb + D;
  double* B2 = red + 16;     // E_t and chol(L_t): sampler elements only
  double* B3 = B2 + C::MAT;
  const int t = blockIdx.x, tid = threadIdx.x, d = M.d, N = M.N;
  const bool samp = A.xi_x != nullptr;
  xload_user<D>(sF, M.F, d);
  xload_pad<D>(B1, A.Sinv + (int64_t)t * D * D);
  if (samp) {
    if (t < N - 1) xload_pad<D>(B2, A.Ec + (int64_t)t * D * D);
    xload_pad<D>(B3, A.Lc + (int64_t)t * D * D);
  }
  if (tid < D) {
    vm[tid] = A.mfr[(int64_t)(N - 1 - t) * D + tid];
    vq[tid] = (t > 0) ? A.mfr[(int64_t)(N - t) * D + tid] : 0.0;
    vx[tid] = (samp && tid < d) ? A.xi_x[(int64_t)t * d + tid] : 0.0;
    vb[tid] = (M.b && tid < d) ? M.b[tid] : 0.0;
  }
  team_sync();
  if (t > 0) {
    matvec<D, false>(vp, sF, vq, vb);  // F m^f_{t-1} + b
  } else if (tid < D) {
    vp[tid] = (tid < d) ? M.m0[tid] : 0.0;
  }
  team_sync();
  if (tid < D) vr[tid] = (tid < d) ? A.om[(int64_t)t * d + tid] - vp[tid] : 0.0;
  team_sync();
  matvec<D, false>(vs, B1, vr);
  const double q = team_sum<D>(tid < D ? vr[tid] * vs[tid] : 0.0, red);
  if (tid == 0) A.ell[t] = -0.5 * (d * LOG2PI_X + A.ldS[t] + q);
  if (!samp) return;
  matvec<D, false>(vu, B3, vx, vm);  // m^f + chol(L) xi
  if (t < N - 1) {
    matvec<D, false>(vp, sF, vm, vb);  // F m^f_t + b
    matvec<D, false>(vr, B2, vp);       // E_t (F m^f_t + b)
    if (tid < D) vu[tid] -= vr[tid];
  }
  if (tid < D) A.U[(int64_t)t * D + tid] = (tid < d) ? vu[tid] : 0.0;
}

template <int D>
hipError_t set_limits() {
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_fixed_phi<D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               lds_phi<D>() * (int)sizeof(double))) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_fixed_cmean<D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               lds_cmean<D>() * (int)sizeof(double))) != hipSuccess)
    return e;
  return hipFuncSetAttribute((const void*)k_fixed_ell<D>,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             lds_ell<D>(true) * (int)sizeof(double));
}

template <int D>
hipError_t launch_k(int which, const KModel& M, FixedArgs A, hipStream_t st) {
  static const hipError_t lim = set_limits<D>();  // once per process
  if (lim != hipSuccess) return lim;
  const dim3 g(M.N), b(Cfg<D>::NT);
  const size_t dbl = sizeof(double);
  if (which == 0) hipLaunchKernelGGL(k_fixed_phi<D>, g, b, lds_phi<D>() * dbl, st, M, A);
  if (which == 1) hipLaunchKernelGGL(k_fixed_cmean<D>, g, b, lds_cmean<D>() * dbl, st, M, A);
  if (which == 2)
    hipLaunchKernelGGL(k_fixed_ell<D>, g, b, lds_ell<D>(A.xi_x != nullptr) * dbl, st, M, A);
  return hipGetLastError();
}

hipError_t launch_any(int which, int D, const KModel& M, FixedArgs A, hipStream_t st) {
  switch (D) {
    case 16: return launch_k<16>(which, M, A, st);
    case 32: return launch_k<32>(which, M, A, st);
    case 64: return launch_k<64>(which, M, A, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_fixed_phi_any(int D, const KModel& M, FixedArgs A, hipStream_t st) {
  return launch_any(0, D, M, A, st);
}
hipError_t launch_fixed_cmean_any(int D, const KModel& M, FixedArgs A, hipStream_t st) {
  return launch_any(1, D, M, A, st);
}
hipError_t launch_fixed_ell_any(int D, const KModel& M, FixedArgs A, hipStream_t st) {
  return launch_any(2, D, M, A, st);
}

}  // namespace akf
