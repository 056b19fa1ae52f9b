// akf_adjoint.hip -- (E, g, L) suffix scans, the RTS smoother, and the
// reverse-mode adjoint of the Kalman log marginal likelihood.
//
// (E, g, L) scan (eq. EgL_comb): elements e_t = (E_t, g_t, L_t) with the
// operator (earlier i, later j)  (E_i E_j, E_i g_j + g_i, E_i L_j E_i' + L_i).
// The suffix scan e_t o ... o e_{N-1} with a terminal element of E = 0 yields,
// for the RTS smoother elements, the smoothing moments (m^s_t, P^s_t).  Blocked
// like the other scans: fold per block (backwards), tree over block
// aggregates (up: combine; down: propagate the suffix state (g, L) entering
// each node from the right), final per block.
//
// Adjoint.  For the LGSSM x_t = F x_{t-1} + N(0, Q), y_t = H x_t + N(0, R)
// (App. A, eq. lgssm-app) the log-likelihood L = sum_t ell_t of the Kalman
// filter (Alg. "Kalman filter", predictive form) has the reverse-mode adjoint
//   mbar_t = Phi_t' mbar_{t+1} + H' w_t,
//   Pbar_t = Phi_t' Pbar_{t+1} Phi_t + G_t,
//   G_t    = -1/2 H'(S^{-1} - w w')H + sym((mbar_t - H'w_t)(H'w_t)'),
// where mbar_t = dL/dm^p_t, Pbar_t = dL/dP^p_t (symmetric), Phi_t = F (I - K_t H),
// S_t = H P^p_t H' + R, K_t = P^p_t H' S_t^{-1}, w_t = S_t^{-1}(y_t - H m^p_t).
// Both are suffix scans: mbar with path elements (E, U) = (Phi', H'w) and
// Pbar with (E, L) = (Phi', G).  Parameter gradients are sums of local terms:
//   dL/dF = sum_{t<N-1} [mbar_{t+1} m^f_t' + 2 Pbar_{t+1} F P^f_t]
//   dL/dQ = sum_{t>=1} Pbar_t
//   dL/dH = sum_t [w m^p' - Sig H P^p + w (P^f fbar)' - (K' fbar) m^f' - 2 K' Fbar P^f]
//   dL/dR = sum_t [-Sig/2 - sym(K' fbar w') + K' Fbar K]
// with Sig = S^{-1} - w w', fbar = F' mbar_{t+1}, Fbar = F' Pbar_{t+1} F (zero at
// t = N-1).  The forward filtering moments (m^f, P^f) are the checkpoint; every
// other per-step quantity is recomputed from them.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "akf_team.hpp"
#include "akf_internal.h"

namespace akf {

__device__ __forceinline__ void flag_status2(int* st, int bit) { atomicOr(st, bit); }

template <int D>
__device__ __forceinline__ void lds_load_pad2(double* s, const double* __restrict__ g) {
  lds_fill<D>(s, [=](int i, int j) { return g[i * D + j]; });
}

template <int D>
__device__ __forceinline__ void lds_load_user(double* s, const double* __restrict__ g, int rows,
                                              int cols) {
  lds_fill<D>(s, [=](int i, int j) { return (i < rows && j < cols) ? g[i * cols + j] : 0.0; });
}

template <int D>
__device__ __forceinline__ void rm_store_t(const RM<D>& a, double* __restrict__ g, int ld, int d) {
  AKF_RM_FOR(D, q, r, i, j) if (i < d && j < d) g[(size_t)j * ld + i] = a.t[q][r];
}

// ---------------------------------------------------------------------------
// (E, g, L) scan
// ---------------------------------------------------------------------------
template <int D>
struct EglLayout {
  static constexpr int E = 0, L = D * D, g = 2 * D * D;
  static constexpr int SIZE = 2 * D * D + D;
};
template <int D>
struct EglState {  // suffix state entering a node from the right
  static constexpr int L = 0, g = D * D;
  static constexpr int SIZE = D * D + D;
};

// The GEMMs of the scan kernels, the smoother's and the adjoint's element
// builds are fully unrolled (U = D / 4); in the gradient kernel every product
// but one (K, the last to fit, would spill) is.
//
// acc <- e_t o acc for t = s1-2 .. s0, starting from acc = e_{s1-1}.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_egl_fold(EglArgs A) {
  using C = Cfg<D>;
  using EL = EglLayout<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* B3 = B2 + C::MAT;
  double* vg = B3 + C::MAT;
  double* vn = vg + D;
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int s0 = blk * A.B, s1 = min(A.N, s0 + A.B);
  RM<D> Et, Lt, T;
  rm_load<D>(Et, A.E + (int64_t)(s1 - 1) * D * D, D, D);
  rm_load<D>(Lt, A.L + (int64_t)(s1 - 1) * D * D, D, D);
  if (tid < D) vg[tid] = A.g ? A.g[(int64_t)(s1 - 1) * D + tid] : 0.0;
  for (int t = s1 - 2; t >= s0; --t) {
    lds_load_pad2<D>(B1, A.E + (int64_t)t * D * D);
    rm_stage<D>(Et, B2);
    rm_stage<D>(Lt, B3);
    team_sync();
    gemm<D, false, false, false, D / 4>(Et, B1, B2);  // E_t E~
    gemm<D, false, false, false, D / 4>(T, B1, B3);   // E_t L~
    matvec<D, false>(vn, B1, vg);
    team_sync();
    rm_stage<D>(T, B3);
    if (tid < D) vg[tid] = vn[tid] + (A.g ? A.g[(int64_t)t * D + tid] : 0.0);
    team_sync();
    gemm<D, false, true, false, D / 4>(Lt, B3, B1);  // (E_t L~) E_t'
    rm_add_load<D>(Lt, A.L + (int64_t)t * D * D, D, D);
    rm_symmetrise<D>(Lt, B2);
  }
  double* out = A.agg + (int64_t)blk * EL::SIZE;
  rm_store<D>(Et, out + EL::E, D, D);
  rm_store<D>(Lt, out + EL::L, D, D);
  if (tid < D) out[EL::g + tid] = vg[tid];
}

template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_egl_up(EglTree T) {
  using C = Cfg<D>;
  using EL = EglLayout<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* B3 = B2 + C::MAT;
  double* vg = B3 + C::MAT;
  double* vn = vg + D;
  const int k = blockIdx.x, tid = threadIdx.x;
  const double* el = T.src + (int64_t)(2 * k) * EL::SIZE;
  double* out = T.dst + (int64_t)k * EL::SIZE;
  if (2 * k + 1 >= T.n_src) {
    team_copy<C::NT>(out, el, EL::SIZE);
    return;
  }
  const double* er = el + EL::SIZE;
  lds_load_pad2<D>(B1, el + EL::E);
  lds_load_pad2<D>(B2, er + EL::E);
  lds_load_pad2<D>(B3, er + EL::L);
  if (tid < D) vg[tid] = er[EL::g + tid];
  team_sync();
  RM<D> R1, R2;
  gemm<D, false, false, false, D / 4>(R1, B1, B2);  // E_l E_r
  gemm<D, false, false, false, D / 4>(R2, B1, B3);  // E_l L_r
  matvec<D, false>(vn, B1, vg);
  rm_store<D>(R1, out + EL::E, D, D);
  team_sync();
  rm_stage<D>(R2, B3);
  if (tid < D) out[EL::g + tid] = vn[tid] + el[EL::g + tid];
  team_sync();
  gemm<D, false, true, false, D / 4>(R1, B3, B1);  // E_l L_r E_l'
  rm_add_load<D>(R1, el + EL::L, D, D);
  rm_symmetrise<D>(R1, B2);
  rm_store<D>(R1, out + EL::L, D, D);
}

// State entering node k of level l (pre_src) -> its children at level l-1:
// right child inherits; left child gets e_right o state = (E_r g + g_r, E_r L E_r' + L_r).
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_egl_down(EglTree T) {
  using C = Cfg<D>;
  using EL = EglLayout<D>;
  using ES = EglState<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* vg = B2 + C::MAT;
  double* vn = vg + D;
  const int k = blockIdx.x, tid = threadIdx.x;
  const double* sin = T.pre_src + (int64_t)k * ES::SIZE;
  const bool has_right = (2 * k + 1 < T.n_dst);
  double* sl = T.pre_dst + (int64_t)(2 * k) * ES::SIZE;
  if (!has_right) {
    team_copy<C::NT>(sl, sin, ES::SIZE);
    return;
  }
  double* sr = T.pre_dst + (int64_t)(2 * k + 1) * ES::SIZE;
  team_copy<C::NT>(sr, sin, ES::SIZE);
  const double* er = T.src + (int64_t)(2 * k + 1) * EL::SIZE;
  lds_load_pad2<D>(B1, er + EL::E);
  lds_load_pad2<D>(B2, sin + ES::L);
  if (tid < D) vg[tid] = sin[ES::g + tid];
  team_sync();
  RM<D> R1;
  gemm<D, false, false, false, D / 4>(R1, B1, B2);  // E_r L
  matvec<D, false>(vn, B1, vg);
  team_sync();
  rm_stage<D>(R1, B2);
  if (tid < D) sl[ES::g + tid] = vn[tid] + er[EL::g + tid];
  team_sync();
  gemm<D, false, true, false, D / 4>(R1, B2, B1);  // E_r L E_r'
  rm_add_load<D>(R1, er + EL::L, D, D);
  rm_symmetrise<D>(R1, B2);
  rm_store<D>(R1, sl + ES::L, D, D);
}

// Final: state = incoming; for t = s1-1 .. s0: state = e_t o state; write it.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_egl_final(EglArgs A) {
  using C = Cfg<D>;
  using ES = EglState<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* vg = B2 + C::MAT;
  double* vn = vg + D;
  const int blk = blockIdx.x, tid = threadIdx.x;
  const int s0 = blk * A.B, s1 = min(A.N, s0 + A.B);
  const double* sin = A.state + (int64_t)blk * ES::SIZE;
  RM<D> Lm, T;
  rm_load<D>(Lm, sin + ES::L, D, D);
  if (tid < D) vg[tid] = sin[ES::g + tid];
  for (int t = s1 - 1; t >= s0; --t) {
    lds_load_pad2<D>(B1, A.E + (int64_t)t * D * D);
    rm_stage<D>(Lm, B2);
    team_sync();
    gemm<D, false, false, false, D / 4>(T, B1, B2);
    matvec<D, false>(vn, B1, vg);
    team_sync();
    rm_stage<D>(T, B2);
    if (tid < D) vg[tid] = vn[tid] + (A.g ? A.g[(int64_t)t * D + tid] : 0.0);
    team_sync();
    gemm<D, false, true, false, D / 4>(Lm, B2, B1);
    rm_add_load<D>(Lm, A.L + (int64_t)t * D * D, D, D);
    rm_symmetrise<D>(Lm, B2);
    rm_store<D>(Lm, A.outL + (int64_t)t * A.ldo * A.ldo, A.ldo, A.dout);
    if (A.outg && tid < A.dout) A.outg[(int64_t)t * A.ldo + tid] = vg[tid];
  }
}

// ---------------------------------------------------------------------------
// RTS smoother elements (eq. init-dnc): E_t = P^f_t F' (P^p_{t+1})^{-1},
// g_t = m^f_t - E_t (F m^f_t + b), L_t = P^f_t - E_t F P^f_t; terminal (0, m^f, P^f).
// ---------------------------------------------------------------------------
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_smooth_build(KModel M, SmoothArgs S) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* sF = lds;
  double* B1 = sF + C::MAT;
  double* B2 = B1 + C::MAT;
  double* B3 = B2 + C::MAT;
  double* vm = B3 + C::MAT;
  double* vmp = vm + D;
  double* vg = vmp + D;
  const int t = blockIdx.x, tid = threadIdx.x, d = M.d;
  RM<D> Pf, R1, R2;
  rm_load<D>(Pf, S.Pf + (int64_t)t * S.ldm * S.ldm, S.ldm, d);
  if (tid < D) vm[tid] = (tid < d) ? S.mf[(int64_t)t * S.ldm + tid] : 0.0;
  if (t == M.N - 1) {
    rm_zero<D>(R1);
    rm_store<D>(R1, S.E + (int64_t)t * D * D, D, D);
    rm_store<D>(Pf, S.L + (int64_t)t * D * D, D, D);
    if (tid < D) S.g[(int64_t)t * D + tid] = vm[tid];
    return;
  }
  bool ok = true;
  double ld;
  rm_load<D>(R2, M.Q, d, d);  // issued early: its latency overlaps G = F P^f
  lds_load_user<D>(sF, M.F, d, d);
  rm_stage<D>(Pf, B1);
  team_sync();
  gemm<D, false, false, false, D / 4>(R1, sF, B1);  // G = F P^f
  team_sync();
  rm_stage<D>(R1, B1);
  team_sync();
  gemm<D, false, true, true, D / 4>(R2, B1, sF);  // Q + G F'
  matvec<D, false>(vmp, sF, vm);
  if (tid < d && M.b) vmp[tid] += M.b[tid];
  {
    const RM<D> Pp = R2;
    ok = spd_inv<D>(R2, d, B3, &ld) && ok;  // (P^p)^{-1}
    inv_refine<D>(R2, Pp, d, B2, B3);       // P^p inherits the conditioning of Q
  }
  rm_stage<D>(R2, B2);
  team_sync();
  gemm<D, true, false, false, D / 4>(R1, B1, B2);  // E = G' (P^p)^{-1}
  rm_store<D>(R1, S.E + (int64_t)t * D * D, D, D);
  rm_stage<D>(R1, B3);
  team_sync();
  gemm<D, false, false, false, D / 4>(R2, B3, B1);  // E G
  rm_rsub<D>(R2, Pf);                        // L = P^f - E G
  matvec<D, false>(vg, B3, vmp);
  if (tid < D) S.g[(int64_t)t * D + tid] = vm[tid] - vg[tid];
  rm_symmetrise<D>(R2, B2);
  rm_store<D>(R2, S.L + (int64_t)t * D * D, D, D);
  if (!ok && tid == 0) flag_status2(S.status, ST_FWD_NOT_PD);
}

// ---------------------------------------------------------------------------
// LGSSM helpers
// ---------------------------------------------------------------------------
// Q = diag(exp(logq)), R = diag(exp(logr)) (dense, user dims)
__global__ void k_lgssm_prep(LgArgs G) {
  const int tid = threadIdx.x + blockIdx.x * blockDim.x;
  const int nq = G.dx * G.dx, nr = G.dy * G.dy;
  if (tid < nq) {
    const int i = tid / G.dx, j = tid % G.dx;
    G.Q[tid] = (i == j) ? exp(G.logq[i]) : 0.0;
  } else if (tid < nq + nr) {
    const int e = tid - nq, i = e / G.dy, j = e % G.dy;
    G.R[e] = (i == j) ? exp(G.logr[i]) : 0.0;
  }
}

// sum of ell (fixed-order tree within one team); NaN when the filter that
// wrote ell set a status bit (status may be null)
__global__ void __launch_bounds__(256) k_sum(const double* __restrict__ a, int n, double* out,
                                             const int* status) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += a[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = red[0] + red[1] + red[2] + red[3];
    *out = (status && *status != 0) ? __builtin_nan("") : t;
  }
}

// Recompute the filter quantities of step t from the checkpoint:
// Pp, mp (registers / LDS), B_HP <- H Pp, B_Si <- S^{-1} (Gauss-Jordan in
// registers), vw <- w = S^{-1} v, vv <- v.  scr: a free D x D LDS buffer.  Team-wide;
// ends synchronised.
template <int D>
__device__ void adj_step_quantities(const KModel& M, const LgArgs& G, int t, const double* sF,
                                    const double* sH, double* B_HP, double* B_Si, double* Btmp,
                                    RM<D>& Pp, double* vmp, double* vv, double* vw, double* scr,
                                    bool& ok) {
  const int tid = threadIdx.x, d = G.dx, p = G.dy;
  RM<D> R1;
  if (t == 0) {
    rm_load<D>(Pp, M.P0, d, d);
    if (tid < D) vmp[tid] = (tid < d) ? M.m0[tid] : 0.0;
  } else {
    rm_load<D>(R1, G.Pf + (int64_t)(t - 1) * D * D, D, D);
    rm_stage<D>(R1, Btmp);
    if (tid < D) vv[tid] = G.mf[(int64_t)(t - 1) * D + tid];
    team_sync();
    gemm<D, false, false, false, D / 4>(R1, sF, Btmp);  // F P^f
    matvec<D, false>(vmp, sF, vv);
    team_sync();
    rm_stage<D>(R1, Btmp);
    team_sync();
    gemm<D, false, true, false, D / 4>(Pp, Btmp, sF);
    rm_add_load<D>(Pp, G.Q, d, d);
  }
  team_sync();
  rm_stage<D>(Pp, Btmp);
  team_sync();
  gemm<D, false, false, false, D / 4>(R1, sH, Btmp);  // H Pp
  team_sync();
  rm_stage<D>(R1, B_HP);
  team_sync();
  gemm<D, false, true, false, D / 4>(R1, B_HP, sH);  // S = H Pp H' + R
  rm_add_load<D>(R1, G.R, p, p);
  matvec<D, false>(vv, sH, vmp);
  if (tid < D) vv[tid] = (tid < p) ? G.y[(int64_t)t * p + tid] - vv[tid] : 0.0;
  double ld;
  ok = spd_inv<D>(R1, p, scr, &ld) && ok;  // S^{-1} (zero outside p x p)
  rm_stage<D>(R1, B_Si);
  team_sync();
  matvec<D, false>(vw, B_Si, vv);  // w = S^{-1} v
  team_sync();
}

// Adjoint elements of step t: E_t = Phi_t' (0 at t = N-1), U_t = h_t = H' w_t,
// Cm_t = -1/2 H' (S^{-1} - w w') H.  One team per t, D <= 32.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_adj_build(KModel M, LgArgs G) {
  // four LDS matrices (F, H and two work buffers X, Y; 35 KB at D = 32), so
  // that four one-wave teams share a CU.  Y serves in turn as staging, as the
  // inverse's scratch and as S^{-1}; K is formed into registers first, which
  // frees both work buffers for the rest.
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* sF = lds;
  double* sH = sF + C::MAT;
  double* X = sH + C::MAT;
  double* Y = X + C::MAT;
  double* vmp = Y + C::MAT;
  double* vv = vmp + D;
  double* vw = vv + D;
  const int t = blockIdx.x, tid = threadIdx.x, d = G.dx, p = G.dy;
  lds_load_user<D>(sF, M.F, d, d);
  lds_load_user<D>(sH, G.H, p, d);
  team_sync();
  bool ok = true;
  RM<D> Pp, R1, R2, K;
  adj_step_quantities<D>(M, G, t, sF, sH, X, Y, Y, Pp, vmp, vv, vw, Y, ok);  // X = H Pp, Y = S^{-1}
  // h = H' w
  matvec<D, true>(G.U + (int64_t)t * D, sH, vw);
  // K = (H Pp)' S^{-1};  Sig = S^{-1} - w w'
  gemm<D, true, false, false, D / 4>(K, X, Y);
  rm_unstage<D>(R1, Y);
  AKF_RM_FOR(D, q, r, i, j) R1.t[q][r] -= vw[i] * vw[j];
  team_sync();
  // Cm = -1/2 H' Sig H
  rm_stage<D>(R1, X);
  team_sync();
  gemm<D, false, false, false, D / 4>(R2, X, sH);  // Sig H
  rm_stage<D>(R2, Y);
  team_sync();
  gemm<D, true, false, false, D / 4>(R1, sH, Y);  // H' Sig H
  rm_axpy<D>(R1, -1.5, R1);                // -1/2 H' Sig H
  rm_store<D>(R1, G.Cm + (int64_t)t * D * D, D, D);
  if (t == M.N - 1) {
    rm_zero<D>(R1);
    rm_store<D>(R1, G.E + (int64_t)t * D * D, D, D);
  } else {
    // Phi = F - (F K) H;  E = Phi'
    rm_stage<D>(K, X);
    team_sync();
    gemm<D, false, false, false, D / 4>(R2, sF, X);  // F K
    rm_stage<D>(R2, Y);
    team_sync();
    gemm<D, false, false, false, D / 4>(R1, Y, sH);  // F K H
    RM<D> Fm;
    rm_load<D>(Fm, M.F, d, d);
    rm_rsub<D>(R1, Fm);  // Phi = F - F K H
    rm_store_t<D>(R1, G.E + (int64_t)t * D * D, D, D);
  }
  if (!ok && tid == 0) flag_status2(G.status, ST_FWD_NOT_PD);
}

// G_t = Cm_t + sym((mbar_t - h_t) h_t')   (in place over Cm)
template <int D>
__global__ void __launch_bounds__(256) k_adj_G(LgArgs G, int N) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * D * D) return;
  const int64_t t = e / (D * D);
  const int i = (int)((e / D) % D), j = (int)(e % D);
  const double* h = G.U + t * D;
  const double* mb = G.mbar + t * D;
  const double a = (mb[i] - h[i]) * h[j] + (mb[j] - h[j]) * h[i];
  G.Cm[e] += 0.5 * a;
}

// Per-block accumulation of the parameter gradients (one team per block of
// steps; partial sums [F (D*D) | H (D*D) | q (D) | r (D)] per block).
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_adj_grad(KModel M, LgArgs G) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  // six matrices and ten vectors (53 KB at D = 32), so that three one-wave
  // teams share a CU
  double* sF = lds;
  double* sH = sF + C::MAT;
  double* B_HP = sH + C::MAT;
  double* B_Si = B_HP + C::MAT;
  double* Bt = B_Si + C::MAT;
  double* Bu = Bt + C::MAT;
  double* vmp = Bu + C::MAT;
  double* vv = vmp + D;
  double* vw = vv + D;
  double* vmf = vw + D;
  double* vfb = vmf + D;   // fbar = F' mbar_{t+1}
  double* vk = vfb + D;    // K' fbar
  double* vpf = vk + D;    // P^f fbar
  double* vmb = vpf + D;   // mbar_{t+1}
  double* vq = vmb + D;    // accumulated dL/dQ_ii
  double* vr = vq + D;     // accumulated dL/dR_jj
  const int blk = blockIdx.x, tid = threadIdx.x, d = G.dx, p = G.dy, N = M.N;
  const int s0 = blk * G.B, s1 = min(N, s0 + G.B);
  lds_load_user<D>(sF, M.F, d, d);
  lds_load_user<D>(sH, G.H, p, d);
  if (tid < D) {
    vq[tid] = 0.0;
    vr[tid] = 0.0;
  }
  team_sync();
  RM<D> gF, gH, Pp, Pf, R1, R2, K;
  rm_zero<D>(gF);
  rm_zero<D>(gH);
  bool ok = true;
  for (int t = s0; t < s1; ++t) {
    // Bt is free while S is inverted: it serves as the inverse's scratch
    adj_step_quantities<D>(M, G, t, sF, sH, B_HP, B_Si, Bt, Pp, vmp, vv, vw, Bt, ok);
    const bool last = (t == N - 1);
    rm_load<D>(Pf, G.Pf + (int64_t)t * D * D, D, D);
    if (tid < D) {
      vmf[tid] = G.mf[(int64_t)t * D + tid];
      vmb[tid] = last ? 0.0 : G.mbar[(int64_t)(t + 1) * D + tid];
    }
    // dL/dQ_ii += Pbar_t,ii  (t >= 1)
    if (t >= 1 && tid < D) vq[tid] += G.Pbar[(int64_t)t * D * D + tid * D + tid];
    team_sync();
    // fbar = F' mbar_{t+1}
    matvec<D, true>(vfb, sF, vmb);
    // K = (H Pp)' S^{-1}
    gemm<D, true, false, false>(K, B_HP, B_Si);
    team_sync();
    // Fbar = F' Pbar_{t+1} F  -> R1 ; also F-gradient term Pbar_{t+1} F P^f
    RM<D> Fb;
    rm_zero<D>(Fb);
    if (!last) {
      lds_load_pad2<D>(Bu, G.Pbar + (int64_t)(t + 1) * D * D);
      team_sync();
      gemm<D, false, false, false, D / 4>(R1, Bu, sF);  // Pbar F
      team_sync();
      rm_stage<D>(R1, Bt);
      rm_stage<D>(Pf, Bu);
      team_sync();
      gemm<D, false, false, false, D / 4>(R2, Bt, Bu);  // Pbar F P^f
      rm_axpy<D>(gF, 2.0, R2);
      gemm<D, true, false, false, D / 4>(Fb, sF, Bt);  // F' Pbar F
      team_sync();
      // dF += mbar_{t+1} m^f_t'
      AKF_RM_FOR(D, q, r, i, j) gF.t[q][r] += vmb[i] * vmf[j];
    }
    // vectors: vk = K' fbar, vpf = P^f fbar
    rm_stage<D>(K, Bt);
    rm_stage<D>(Pf, Bu);
    team_sync();
    matvec<D, true>(vk, Bt, vfb);
    matvec<D, false>(vpf, Bu, vfb);
    team_sync();
    // H-gradient:  w mp' - Sig H Pp + w (P^f fbar)' - (K' fbar) m^f' - 2 K' Fbar P^f
    // Sig H Pp = S^{-1} (H Pp) - w (w' H Pp)
    gemm<D, false, false, false, D / 4>(R1, B_Si, B_HP);  // S^{-1} H Pp
    rm_axpy<D>(gH, -1.0, R1);
    // w' H Pp  (row vector) into vv
    matvec<D, true>(vv, B_HP, vw);
    AKF_RM_FOR(D, q, r, i, j)
    gH.t[q][r] += vw[i] * vmp[j] + vw[i] * vv[j] + vw[i] * vpf[j] - vk[i] * vmf[j];
    // R-gradient diag: -1/2 Sig_jj - (K' fbar)_j w_j + (K' Fbar K)_jj
    if (tid < p) vr[tid] += -0.5 * (B_Si[tid * C::LD + tid] - vw[tid] * vw[tid]) - vk[tid] * vw[tid];
    if (!last) {
      // K' Fbar -> R1 (Bt holds K)
      rm_stage<D>(Fb, Bu);
      team_sync();
      gemm<D, true, false, false, D / 4>(R1, Bt, Bu);  // K' Fbar
      team_sync();
      rm_stage<D>(R1, Bu);
      rm_stage<D>(Pf, B_HP);  // H Pp is no longer read in this step
      team_sync();
      gemm<D, false, false, false, D / 4>(R2, Bu, B_HP);  // K' Fbar P^f
      rm_axpy<D>(gH, -2.0, R2);
      // (K' Fbar K)_jj = sum_i (K' Fbar)_ji K_ij
      if (tid < p) {
        double s = 0.0;
        for (int i = 0; i < D; ++i) s = fma(Bu[tid * C::LD + i], Bt[i * C::LD + tid], s);
        vr[tid] += s;
      }
    }
    team_sync();
  }
  double* out = G.part + (int64_t)blk * (2 * D * D + 2 * D);
  rm_store<D>(gF, out, D, D);
  rm_store<D>(gH, out + D * D, D, D);
  if (tid < D) {
    out[2 * D * D + tid] = vq[tid];
    out[2 * D * D + D + tid] = vr[tid];
  }
  if (!ok && tid == 0) flag_status2(G.status, ST_FWD_NOT_PD);
}

// Sum the block partials in a fixed order and map to (dF, dlogq, dH, dlogr),
// scaled by the upstream gradient ll_bar.
template <int D>
__global__ void __launch_bounds__(256) k_adj_reduce(LgArgs G, int nblk, const double* ll_bar) {
  // 32 parameters per workgroup; thread row r (of 8) adds blocks r, r + 8, ...
  // and the rows are added in row order, so the result does not depend on timing
  __shared__ double acc[8][33];
  const int px = threadIdx.x & 31, gy = threadIdx.x >> 5;
  const int tid = blockIdx.x * 32 + px;
  const int d = G.dx, p = G.dy;
  const int tot = d * d + d + p * d + p;
  const bool valid = tid < tot;
  int off = 0;
  double* dst = nullptr;
  double mul = 1.0;
  if (!valid) {
  } else if (tid < d * d) {
    const int i = tid / d, j = tid % d;
    off = i * D + j;
    dst = G.dF + tid;
  } else if (tid < d * d + d) {
    const int i = tid - d * d;
    off = 2 * D * D + i;
    dst = G.dlogq + i;
    mul = exp(G.logq[i]);
  } else if (tid < d * d + d + p * d) {
    const int e = tid - d * d - d, k = e / d, j = e % d;
    off = D * D + k * D + j;
    dst = G.dH + e;
  } else {
    const int k = tid - d * d - d - p * d;
    off = 2 * D * D + D + k;
    dst = G.dlogr + k;
    mul = exp(G.logr[k]);
  }
  double s = 0.0;
  if (valid)
    for (int b = gy; b < nblk; b += 8) s += G.part[(int64_t)b * (2 * D * D + 2 * D) + off];
  acc[gy][px] = s;
  __syncthreads();
  if (gy == 0 && valid) {
    double t = acc[0][px];
#pragma unroll
    for (int r = 1; r < 8; ++r) t += acc[r][px];
    const double sc = ll_bar ? *ll_bar : 1.0;
    // a failed forward or adjoint pass (any status bit) leaves no gradient
    *dst = (*G.status != 0) ? __builtin_nan("") : sc * mul * t;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int D>
size_t lds_bytes_mats(int nmat, int nvec) {
  return (size_t)(nmat * Cfg<D>::MAT + nvec * D + 16) * sizeof(double);
}

template <int D>
hipError_t launch_egl_scan(EglArgs A, EglTree* up, EglTree* down, int n_levels, hipStream_t st) {
  const int nb = (A.N + A.B - 1) / A.B;
  hipLaunchKernelGGL(k_egl_fold<D>, dim3(nb), dim3(Cfg<D>::NT), lds_bytes_mats<D>(3, 2), st, A);
  for (int l = 0; l < n_levels; ++l)
    hipLaunchKernelGGL(k_egl_up<D>, dim3(up[l].n_dst), dim3(Cfg<D>::NT), lds_bytes_mats<D>(3, 2),
                       st, up[l]);
  for (int l = n_levels - 1; l >= 0; --l)
    hipLaunchKernelGGL(k_egl_down<D>, dim3(down[l].n_src), dim3(Cfg<D>::NT),
                       lds_bytes_mats<D>(2, 2), st, down[l]);
  hipLaunchKernelGGL(k_egl_final<D>, dim3(nb), dim3(Cfg<D>::NT), lds_bytes_mats<D>(2, 2), st, A);
  return hipGetLastError();
}

hipError_t launch_egl_scan_any(int D, EglArgs A, EglTree* up, EglTree* down, int nl,
                               hipStream_t st) {
  switch (D) {
    case 16: return launch_egl_scan<16>(A, up, down, nl, st);
    case 32: return launch_egl_scan<32>(A, up, down, nl, st);
    case 64: return launch_egl_scan<64>(A, up, down, nl, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_smooth_build_any(int D, const KModel& M, SmoothArgs S, hipStream_t st) {
  switch (D) {
    case 16:
      hipLaunchKernelGGL(k_smooth_build<16>, dim3(M.N), dim3(64), lds_bytes_mats<16>(4, 7), st, M, S);
      break;
    case 32:
      hipLaunchKernelGGL(k_smooth_build<32>, dim3(M.N), dim3(64), lds_bytes_mats<32>(4, 7), st, M, S);
      break;
    case 64:
      hipLaunchKernelGGL(k_smooth_build<64>, dim3(M.N), dim3(256), lds_bytes_mats<64>(4, 7), st, M,
                         S);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lgssm_prep(LgArgs G, hipStream_t st) {
  const int n = G.dx * G.dx + G.dy * G.dy;
  hipLaunchKernelGGL(k_lgssm_prep, dim3((n + 255) / 256), dim3(256), 0, st, G);
  return hipGetLastError();
}

hipError_t launch_sum(const double* a, int n, double* out, const int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, a, n, out, status);
  return hipGetLastError();
}

template <int D>
hipError_t launch_adj_build_t(const KModel& M, LgArgs G, hipStream_t st) {
  timing_mark(FAM_ADJ_BUILD, 1, st);
  hipLaunchKernelGGL(k_adj_build<D>, dim3(M.N), dim3(Cfg<D>::NT), lds_bytes_mats<D>(4, 3), st, M, G);
  timing_mark(FAM_ADJ_BUILD, 0, st);
  return hipGetLastError();
}
template <int D>
hipError_t launch_adj_finish_t(const KModel& M, LgArgs G, int nblk, const double* ll_bar,
                               hipStream_t st) {
  const int64_t n = (int64_t)M.N * D * D;
  timing_mark(FAM_ADJ_GRAD, 1, st);
  hipLaunchKernelGGL(k_adj_grad<D>, dim3(nblk), dim3(Cfg<D>::NT), lds_bytes_mats<D>(6, 10), st, M,
                     G);
  timing_mark(FAM_ADJ_GRAD, 0, st);
  const int tot = G.dx * G.dx + G.dx + G.dy * G.dx + G.dy;
  hipLaunchKernelGGL(k_adj_reduce<D>, dim3((tot + 31) / 32), dim3(256), 0, st, G, nblk, ll_bar);
  (void)n;
  return hipGetLastError();
}
template <int D>
hipError_t launch_adj_G_t(LgArgs G, int N, hipStream_t st) {
  const int64_t n = (int64_t)N * D * D;
  hipLaunchKernelGGL(k_adj_G<D>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, G, N);
  return hipGetLastError();
}

hipError_t launch_adj_build_any(int D, const KModel& M, LgArgs G, hipStream_t st) {
  if (D == 16) return launch_adj_build_t<16>(M, G, st);
  if (D == 32) return launch_adj_build_t<32>(M, G, st);
  return hipErrorInvalidValue;
}
hipError_t launch_adj_G_any(int D, LgArgs G, int N, hipStream_t st) {
  if (D == 16) return launch_adj_G_t<16>(G, N, st);
  if (D == 32) return launch_adj_G_t<32>(G, N, st);
  return hipErrorInvalidValue;
}
hipError_t launch_adj_finish_any(int D, const KModel& M, LgArgs G, int nblk, const double* ll_bar,
                                 hipStream_t st) {
  if (D == 16) return launch_adj_finish_t<16>(M, G, nblk, ll_bar, st);
  if (D == 32) return launch_adj_finish_t<32>(M, G, nblk, ll_bar, st);
  return hipErrorInvalidValue;
}

}  // namespace akf
