// akf_dnc.hip -- divide-and-conquer pathwise sampler (App. A,
// "Divide-and-conquer strategies"), an alternative to the prefix-sum sampler
// with the same inputs (filtering moments) and the same law.
//
// Bisection tree of [0, T] (T = N - 1): an interval [k, m] with m - k >= 2 is
// a node with midpoint l = (k + m) / 2 and children [k, l], [l, m]; every
// 0 < l < T is the midpoint of exactly one node.  Node slot i at depth j is
// reached from [0, T] by the bits of i (1 = right child), so no node table is
// needed.
//   leaves  : (E, g, L) of [t, t+1] (eq. init-dnc), one team per t;
//   up      : deepest level first, one team per node: the element of [k, m]
//             from its children (eq. EgL_comb) and the bridge
//             p(x_l | x_k, x_m) = N(G x_k + Gamma x_m + w, V) (eq.
//             recursive_params), with chol(V);
//   root    : x_T = m^f_T + chol(P^f_T) xi_T, x_0 = E_{0:T} x_T + g_{0:T} +
//             chol(L_{0:T}) xi_0;
//   down    : level by level from the root, x_l = G x_k + Gamma x_m + w +
//             chol(V) xi_l (matrix-vector products only).
// Elements and bridges are stored D-padded by midpoint (leaves by t).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "akf_team.hpp"
#include "akf_internal.h"

namespace akf {

namespace {

template <int D>
__device__ __forceinline__ void load_pad(double* s, const double* __restrict__ g) {
  lds_fill<D>(s, [=](int i, int j) { return g[i * D + j]; });
}

template <int D>
__device__ __forceinline__ void load_user(double* s, const double* __restrict__ g, int d) {
  lds_fill<D>(s, [=](int i, int j) { return (i < d && j < d) ? g[i * d + j] : 0.0; });
}

// Node slot i at depth j of the bisection tree of [0, T]; false when the slot
// holds no node (an interval on the way, or the slot's own, is shorter than 2).
__device__ __forceinline__ bool dnc_node(int T, int depth, int i, int& k, int& l, int& m) {
  k = 0;
  m = T;
  for (int b = depth - 1; b >= 0; --b) {
    if (m - k < 2) return false;
    const int mid = (k + m) / 2;
    if ((i >> b) & 1)
      k = mid;
    else
      m = mid;
  }
  if (m - k < 2) return false;
  l = (k + m) / 2;
  return true;
}

template <int D>
constexpr int dnc_lds_doubles() {
  return 4 * Cfg<D>::MAT + inv_scratch<D>() + 4 * D + 16;
}

// (E, g, L) of [t, t+1]: G = F P^f (F the transition into t+1), P^p = G F' + Q,
// E = G' (P^p)^{-1}, g = m^f - E (F m^f + b), L = P^f - E G.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_dnc_leaf(KModel M, DncArgs A) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* sF = lds;
  double* B1 = sF + C::MAT;
  double* B2 = B1 + C::MAT;
  double* B3 = B2 + C::MAT;
  double* scr = B3 + C::MAT;
  double* vm = scr + inv_scratch<D>();
  double* vmp = vm + D;
  double* vg = vmp + D;
  const int t = blockIdx.x, tid = threadIdx.x, d = M.d;
  RM<D> Pf, R1, R2;
  rm_load<D>(Pf, A.Pf + (int64_t)t * A.ldm * A.ldm, A.ldm, d);
  rm_load<D>(R2, M.Q, d, d);
  if (A.Ft)
    load_user<D>(sF, A.Ft + (int64_t)(t + 1) * d * d, d);
  else
    load_user<D>(sF, M.F, d);
  const double* bt = A.Ft ? A.bt + (int64_t)(t + 1) * d : M.b;
  if (tid < D) vm[tid] = (tid < d) ? A.mf[(int64_t)t * A.ldm + tid] : 0.0;
  rm_stage<D>(Pf, B1);
  team_sync();
  gemm<D, false, false, false, D / 4>(R1, sF, B1);  // G = F P^f
  team_sync();
  rm_stage<D>(R1, B1);  // B1 = G
  team_sync();
  gemm<D, false, true, true, D / 4>(R2, B1, sF);  // P^p = Q + G F'
  matvec<D, false>(vmp, sF, vm);
  if (tid < d && bt) vmp[tid] += bt[tid];
  bool ok;
  double ld;
  {
    const RM<D> Pp = R2;
    ok = spd_inv<D>(R2, d, scr, &ld);
    inv_refine<D>(R2, Pp, d, B2, B3);
  }
  rm_stage<D>(R2, B2);
  team_sync();
  gemm<D, true, false, false, D / 4>(R1, B1, B2);  // E = G' (P^p)^{-1}
  rm_store<D>(R1, A.Elf + (int64_t)t * D * D, D, D);
  rm_stage<D>(R1, B3);
  team_sync();
  gemm<D, false, false, false, D / 4>(R2, B3, B1);  // E G
  rm_rsub<D>(R2, Pf);                        // L = P^f - E G
  rm_symmetrise<D>(R2, B2);
  rm_store<D>(R2, A.Llf + (int64_t)t * D * D, D, D);
  matvec<D, false>(vg, B3, vmp);
  if (tid < D) A.glf[(int64_t)t * D + tid] = vm[tid] - vg[tid];
  if (!ok && tid == 0) atomicOr(A.status, ST_FWD_NOT_PD);
}

// One node: the element of [k, m] from [k, l] (E1, g1, L1) and [l, m]
// (E2, g2, L2): E = E1 E2, g = E1 g2 + g1, L = E1 L2 E1' + L1; the bridge
// G = L2 E1' L^{-1} = (E1 L2)' L^{-1}, Gamma = E2 - G E, w = g2 - G g,
// V = L2 - G (E1 L2), and chol(V).
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_dnc_up(KModel M, DncArgs A, int depth) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* B3 = B2 + C::MAT;
  double* B4 = B3 + C::MAT;
  double* scr = B4 + C::MAT;
  double* vg1 = scr + inv_scratch<D>();
  double* vg2 = vg1 + D;
  double* vg = vg2 + D;
  double* vw = vg + D;
  const int tid = threadIdx.x, d = M.d;
  int k, l, m;
  if (!dnc_node(A.T, depth, blockIdx.x, k, l, m)) return;
  // children: a leaf when the interval has length 1, else the node at its midpoint
  const bool lleaf = (l - k == 1), rleaf = (m - l == 1);
  const int li = lleaf ? k : (k + l) / 2, ri = rleaf ? l : (l + m) / 2;
  const double* E1p = (lleaf ? A.Elf : A.Eno) + (int64_t)li * D * D;
  const double* L1p = (lleaf ? A.Llf : A.Lno) + (int64_t)li * D * D;
  const double* g1p = (lleaf ? A.glf : A.gno) + (int64_t)li * D;
  const double* E2p = (rleaf ? A.Elf : A.Eno) + (int64_t)ri * D * D;
  const double* L2p = (rleaf ? A.Llf : A.Lno) + (int64_t)ri * D * D;
  const double* g2p = (rleaf ? A.glf : A.gno) + (int64_t)ri * D;
  RM<D> E2, L2, L, T1, R;
  rm_load<D>(E2, E2p, D, D);
  rm_load<D>(L2, L2p, D, D);
  rm_load<D>(L, L1p, D, D);
  load_pad<D>(B1, E1p);
  if (tid < D) {
    vg1[tid] = g1p[tid];
    vg2[tid] = g2p[tid];
  }
  rm_stage<D>(E2, B2);
  rm_stage<D>(L2, B3);
  team_sync();
  RM<D> E;
  gemm<D, false, false, false, D / 4>(E, B1, B2);   // E = E1 E2
  gemm<D, false, false, false, D / 4>(T1, B1, B3);  // T1 = E1 L2
  matvec<D, false>(vg, B1, vg2, vg1);        // g = E1 g2 + g1
  rm_stage<D>(T1, B4);
  team_sync();
  gemm<D, false, true, true, D / 4>(L, B4, B1);  // L = L1 + T1 E1'
  rm_symmetrise<D>(L, B2);
  rm_store<D>(E, A.Eno + (int64_t)l * D * D, D, D);
  rm_store<D>(L, A.Lno + (int64_t)l * D * D, D, D);
  if (tid < D) A.gno[(int64_t)l * D + tid] = vg[tid];
  // bridge
  bool ok;
  double ld;
  {
    R = L;
    ok = spd_inv<D>(R, d, scr, &ld);
    inv_refine<D>(R, L, d, B1, B2);  // L inherits the conditioning of Q
  }
  rm_stage<D>(R, B3);
  team_sync();
  RM<D> G;
  gemm<D, true, false, false, D / 4>(G, B4, B3);  // G = T1' L^{-1}
  team_sync();
  rm_stage<D>(G, B3);
  rm_stage<D>(E, B1);
  team_sync();
  gemm<D, false, false, false, D / 4>(R, B3, B1);  // G E
  rm_rsub<D>(R, E2);                        // Gamma = E2 - G E
  rm_store<D>(G, A.Gb + (int64_t)l * D * D, D, D);
  rm_store<D>(R, A.Gam + (int64_t)l * D * D, D, D);
  matvec<D, false>(vw, B3, vg);  // G g
  if (tid < D) A.wb[(int64_t)l * D + tid] = vg2[tid] - vw[tid];
  gemm<D, false, false, false, D / 4>(R, B3, B4);  // G T1
  rm_rsub<D>(R, L2);                        // V = L2 - G E1 L2
  rm_symmetrise<D>(R, B2);
  ok = chol_reg<D>(R, d, scr, &ld) && ok;
  rm_store<D>(R, A.Vc + (int64_t)l * D * D, D, D);
  if (!ok && tid == 0) atomicOr(A.status, ST_FWD_NOT_PD);
}

// x_T and x_0.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_dnc_root(KModel M, DncArgs A) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* scr = B2 + C::MAT;
  double* vx = scr + inv_scratch<D>();
  double* vt = vx + D;
  double* vz = vt + D;
  const int tid = threadIdx.x, d = M.d, T = A.T;
  RM<D> R;
  double ld;
  rm_load<D>(R, A.Pf + (int64_t)T * A.ldm * A.ldm, A.ldm, d);
  bool ok = chol_reg<D>(R, d, scr, &ld);
  rm_stage<D>(R, B1);
  if (tid < D) vt[tid] = (tid < d) ? A.xi[(int64_t)T * d + tid] : 0.0;
  team_sync();
  matvec<D, false>(vx, B1, vt);
  if (tid < D) vx[tid] = (tid < d) ? A.mf[(int64_t)T * A.ldm + tid] + vx[tid] : 0.0;
  if (tid < d) A.x[(int64_t)T * d + tid] = vx[tid];
  if (T >= 1) {
    const bool leaf = (T == 1);
    const double* Ep = (leaf ? A.Elf : A.Eno) + (int64_t)(leaf ? 0 : T / 2) * D * D;
    const double* Lp = (leaf ? A.Llf : A.Lno) + (int64_t)(leaf ? 0 : T / 2) * D * D;
    const double* gp = (leaf ? A.glf : A.gno) + (int64_t)(leaf ? 0 : T / 2) * D;
    rm_load<D>(R, Lp, D, D);
    ok = chol_reg<D>(R, d, scr, &ld) && ok;
    team_sync();
    load_pad<D>(B2, Ep);
    rm_stage<D>(R, B1);
    if (tid < D) vt[tid] = (tid < d) ? A.xi[tid] : 0.0;
    team_sync();
    matvec<D, false>(vz, B2, vx, gp);  // E x_T + g
    matvec<D, false>(vz, B1, vt, vz);  // + chol(L) xi_0
    if (tid < d) A.x[tid] = vz[tid];
  }
  if (!ok && tid == 0) atomicOr(A.status, ST_FWD_NOT_PD);
}

// Midpoints of the nodes at one depth.
template <int D>
__global__ void __launch_bounds__(Cfg<D>::NT) k_dnc_down(KModel M, DncArgs A, int depth) {
  using C = Cfg<D>;
  extern __shared__ double lds[];
  double* B1 = lds;
  double* B2 = B1 + C::MAT;
  double* B3 = B2 + C::MAT;
  double* vk = B3 + C::MAT;
  double* vm = vk + D;
  double* vxi = vm + D;
  double* vy = vxi + D;
  const int tid = threadIdx.x, d = M.d;
  int k, l, m;
  if (!dnc_node(A.T, depth, blockIdx.x, k, l, m)) return;
  load_pad<D>(B1, A.Gb + (int64_t)l * D * D);
  load_pad<D>(B2, A.Gam + (int64_t)l * D * D);
  load_pad<D>(B3, A.Vc + (int64_t)l * D * D);
  if (tid < D) {
    vk[tid] = (tid < d) ? A.x[(int64_t)k * d + tid] : 0.0;
    vm[tid] = (tid < d) ? A.x[(int64_t)m * d + tid] : 0.0;
    vxi[tid] = (tid < d) ? A.xi[(int64_t)l * d + tid] : 0.0;
  }
  team_sync();
  matvec<D, false>(vy, B1, vk, A.wb + (int64_t)l * D);  // w + G x_k
  matvec<D, false>(vy, B2, vm, vy);                     // + Gamma x_m
  matvec<D, false>(vy, B3, vxi, vy);                    // + chol(V) xi_l
  if (tid < d) A.x[(int64_t)l * d + tid] = vy[tid];
}

template <int D>
hipError_t set_dnc_lds_limits(size_t lds) {
  hipError_t e;
  if ((e = hipFuncSetAttribute((const void*)k_dnc_leaf<D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_dnc_up<D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds)) != hipSuccess)
    return e;
  if ((e = hipFuncSetAttribute((const void*)k_dnc_root<D>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
    return e;
  return hipFuncSetAttribute((const void*)k_dnc_down<D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

template <int D>
hipError_t launch_dnc(const KModel& M, DncArgs A, int depth, hipStream_t st) {
  const size_t lds = (size_t)dnc_lds_doubles<D>() * sizeof(double);
  // the LDS limit is a per-kernel attribute: set once per process
  static const hipError_t set_err = set_dnc_lds_limits<D>(lds);
  if (set_err != hipSuccess) return set_err;
  const dim3 nt(Cfg<D>::NT);
  timing_mark(FAM_DNC, 1, st);
  if (A.T >= 1) hipLaunchKernelGGL(k_dnc_leaf<D>, dim3(A.T), nt, lds, st, M, A);
  for (int j = depth - 1; j >= 0; --j)
    hipLaunchKernelGGL(k_dnc_up<D>, dim3(1u << j), nt, lds, st, M, A, j);
  hipLaunchKernelGGL(k_dnc_root<D>, dim3(1), nt, lds, st, M, A);
  for (int j = 0; j < depth; ++j)
    hipLaunchKernelGGL(k_dnc_down<D>, dim3(1u << j), nt, lds, st, M, A, j);
  timing_mark(FAM_DNC, 0, st);
  return hipGetLastError();
}

}  // namespace

// Levels of the bisection tree of [0, T] that hold nodes.
int dnc_depth(int T) {
  int depth = 0, len = T;
  while (len >= 2) {
    ++depth;
    len = (len + 1) / 2;
  }
  return depth;
}

hipError_t launch_dnc_any(int D, const KModel& M, DncArgs A, hipStream_t st) {
  const int depth = dnc_depth(A.T);
  switch (D) {
    case 16: return launch_dnc<16>(M, A, depth, st);
    case 32: return launch_dnc<32>(M, A, depth, st);
    case 64: return launch_dnc<64>(M, A, depth, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace akf
