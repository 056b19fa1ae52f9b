// akf_fact.hip -- the auxiliary LGSSM of a prior that factorises over
// coordinates: dx independent scalar LGSSMs.
//
// When P0, F and Q are diagonal and Omega_t is diagonal (first order, or
// second order with a diagonal emission Hessian), the auxiliary proposal is a
// product over coordinates even though the target is not (Sec.
// "Spatio-temporal model"): every Kalman quantity is a scalar, and the
// parallel-in-time filter and pathwise sampler of App. A ("Prefix-sums and the
// parallel Kalman filter", "Parallel Rauch--Tung--Striebel sampler") run on
// scalars.  One workgroup per coordinate, FT threads; time is cut into chunks
// of FT * S steps (S <= FS_MAX per thread), each chunk a blocked
// reduce-then-scan:
//   filter  : fold   -- each thread folds its S elements (A, b, C, eta, J);
//             scan   -- inclusive scan over the FT thread elements (wave
//                       shuffles, then the wave totals through LDS), with the
//                       previous chunk's last filtering moments in front;
//             final  -- each thread re-runs its steps from its prefix with the
//                       sequential Kalman update: m^f_t, P^f_t and the
//                       predictive log-likelihood terms.
//   sampler : chunks from the last to the first; x_t = E_t x_{t+1} + U_t with
//             E_t = G_t, U_t = m^f_t - G_t m^p_{t+1} + sqrt(Sigma_t) xi_t; fold
//             per thread, suffix scan of the affine maps, then each thread
//             walks its steps backward from the state entering from the right.
// Filtering moments are kept coordinate-major ([dx][N]) in the workspace
// between the filter and the sampler.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "akf_internal.h"

namespace akf {

namespace {

constexpr double LOG2PI_F = 1.8378770664093454835606594728112;
constexpr int FT = 256;      // threads per coordinate
constexpr int FW = FT / 64;  // waves per coordinate
constexpr int FS_MAX = 8;    // steps per thread and chunk

// Scalar filter element: p(x_t | x_s, y_{s+1:t}) = N(A x_s + b, C) and the
// information pair (eta, J) of p(y_{s+1:t} | x_s).  (1, 0, 0, 0, 0) is the
// identity of the combination.
struct SE {
  double A, b, C, eta, J;
};

// Element combination (App. A, eq. parallel filter operator) for scalars;
// `i` precedes `j` in time.
__device__ __forceinline__ SE se_combine(const SE& i, const SE& j) {
  const double iw = 1.0 / (1.0 + i.C * j.J);
  SE o;
  o.A = j.A * i.A * iw;
  o.b = j.A * (i.b + i.C * j.eta) * iw + j.b;
  o.C = j.A * j.A * i.C * iw + j.C;
  o.eta = i.A * (j.eta - j.J * i.b) * iw + i.eta;
  o.J = i.A * i.A * j.J * iw + i.J;
  return o;
}

__device__ __forceinline__ SE se_shfl_up(const SE& e, int s) {
  SE o;
  o.A = __shfl_up(e.A, s);
  o.b = __shfl_up(e.b, s);
  o.C = __shfl_up(e.C, s);
  o.eta = __shfl_up(e.eta, s);
  o.J = __shfl_up(e.J, s);
  return o;
}

// Affine map x -> E x + U (one backward sampling step or a composition).
struct AM {
  double E, U;
};

// a o b: apply b, then a (a holds the earlier time steps)
__device__ __forceinline__ AM am_compose(const AM& a, const AM& b) {
  return AM{a.E * b.E, a.E * b.U + a.U};
}

__device__ __forceinline__ double block_reduce(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < FW; ++w) s += red[w];
  return s;
}

__global__ void __launch_bounds__(FT) k_fact_scan(KModel M, FactArgs P) {
  __shared__ SE swave[FW];
  __shared__ AM samp[FW];
  __shared__ double red[FW];
  __shared__ double carry[2];
  const int i = blockIdx.x;  // coordinate
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int N = M.N, d = M.d;
  const double F = M.F[i], Q = M.Q[i], P0 = M.P0[i], m0 = M.m0[i];
  const double bb = M.b ? M.b[i] : 0.0;
  int S = (N + FT - 1) / FT;
  if (S > FS_MAX) S = FS_MAX;
  const int chunk = FT * S;
  const int n_chunks = (N + chunk - 1) / chunk;
  double* mfc = P.mf ? P.mf + (int64_t)i * N : nullptr;
  double* Pfc = P.Pf ? P.Pf + (int64_t)i * N : nullptr;
  bool bad = false;
  double lz = 0.0;
  double cm = 0.0, cP = 0.0;  // filtering moments at the end of the previous chunk

  // ---------------- filter ----------------
  for (int c = 0; c < n_chunks; ++c) {
    const int t0 = c * chunk + tid * S;
    int cnt = N - t0;
    cnt = cnt < 0 ? 0 : (cnt > S ? S : cnt);
    double om[FS_MAX], Om[FS_MAX];
#pragma unroll
    for (int s = 0; s < FS_MAX; ++s) {
      if (s < cnt) {
        om[s] = P.om[(int64_t)(t0 + s) * d + i];
        Om[s] = P.Om[(int64_t)(t0 + s) * d + i];
      }
    }
    // fold: this thread's elements, in time order
    SE acc{1.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < FS_MAX; ++s) {
      if (s < cnt) {
        SE e;
        if (t0 + s == 0) {
          const double iS = 1.0 / (P0 + Om[s]);
          e = SE{0.0, m0 + P0 * (om[s] - m0) * iS, P0 * Om[s] * iS, 0.0, 0.0};
        } else {
          const double iS = 1.0 / (Q + Om[s]);
          e = SE{F * Om[s] * iS, (Om[s] * bb + Q * om[s]) * iS, Q * Om[s] * iS,
                 F * (om[s] - bb) * iS, F * F * iS};
        }
        acc = se_combine(acc, e);
      }
    }
    // inclusive scan over the wave
    SE inc = acc;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
      const SE o = se_shfl_up(inc, s);
      if (lane >= s) inc = se_combine(o, inc);
    }
    if (lane == 63) swave[w] = inc;
    SE ex = se_shfl_up(inc, 1);
    if (lane == 0) ex = SE{1.0, 0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    // prefix entering this thread: previous chunk's moments, earlier waves, earlier lanes
    SE pre = (c == 0) ? SE{1.0, 0.0, 0.0, 0.0, 0.0} : SE{0.0, cm, cP, 0.0, 0.0};
    for (int k = 0; k < w; ++k) pre = se_combine(pre, swave[k]);
    pre = se_combine(pre, ex);
    // final: sequential Kalman update from the prefix moments (b, C); the
    // log det terms are accumulated as one product (frexp keeps it in range)
    double m = pre.b, Pv = pre.C, ell = 0.0, sprod = 1.0;
    int sexp = 0;
#pragma unroll
    for (int s = 0; s < FS_MAX; ++s) {
      if (s < cnt) {
        const int t = t0 + s;
        const double mp = (t == 0) ? m0 : F * m + bb;
        const double Pp = (t == 0) ? P0 : F * F * Pv + Q;
        const double Sv = Pp + Om[s];
        if (!(Sv > 0.0) || !(Pp >= 0.0)) bad = true;
        const double iS = 1.0 / Sv;
        const double r = om[s] - mp;
        int e2;
        sprod = frexp(sprod * Sv, &e2);
        sexp += e2;
        ell += -0.5 * (LOG2PI_F + r * r * iS);
        m = mp + Pp * iS * r;
        Pv = Pp * Om[s] * iS;
        if (mfc) {
          mfc[t] = m;
          Pfc[t] = Pv;
        }
      }
    }
    ell += -0.5 * (log(sprod) + sexp * 0.69314718055994530942);  // log det terms
    lz += block_reduce(ell, red);
    // moments at the chunk's last step for the next chunk
    if (c + 1 < n_chunks && tid == FT - 1) {
      carry[0] = m;
      carry[1] = Pv;
    }
    __syncthreads();
    cm = carry[0];
    cP = carry[1];
  }
  if (bad || !isfinite(lz)) atomicOr(P.status, P.fail_bit);
  if (tid == 0) P.lz[i] = lz;
  if (!P.xi_x) return;

  // ---------------- sampler ----------------
  // mf/Pf were written by this workgroup; make them visible to every thread
  __threadfence_block();
  __syncthreads();
  double xr = 0.0;  // x entering the current chunk from the right
  bool sbad = false;
  for (int c = n_chunks - 1; c >= 0; --c) {
    const int t0 = c * chunk + tid * S;
    int cnt = N - t0;
    cnt = cnt < 0 ? 0 : (cnt > S ? S : cnt);
    AM st[FS_MAX];
#pragma unroll
    for (int s = 0; s < FS_MAX; ++s) {
      if (s < cnt) {
        const int t = t0 + s;
        const double mf = mfc[t], Pf = Pfc[t];
        const double xi = P.xi_x[(int64_t)t * d + i];
        if (t == N - 1) {
          if (!(Pf > 0.0)) sbad = true;
          st[s] = AM{0.0, mf + sqrt(Pf) * xi};
        } else {
          const double Pp1 = F * F * Pf + Q;
          const double iP = 1.0 / Pp1;
          const double G = Pf * F * iP;
          const double Sig = Pf * Q * iP;
          if (!(Pp1 > 0.0) || !(Sig > 0.0)) sbad = true;
          st[s] = AM{G, mf - G * (F * mf + bb) + sqrt(Sig) * xi};
        }
      }
    }
    // fold: composition of this thread's steps (earliest first)
    AM agg{1.0, 0.0};
#pragma unroll
    for (int s = FS_MAX - 1; s >= 0; --s)
      if (s < cnt) agg = am_compose(st[s], agg);
    // inclusive suffix scan over the wave
    AM inc = agg;
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
      const AM o{__shfl_down(inc.E, s), __shfl_down(inc.U, s)};
      if (lane + s < 64) inc = am_compose(inc, o);
    }
    if (lane == 0) samp[w] = inc;
    AM ex{__shfl_down(inc.E, 1), __shfl_down(inc.U, 1)};
    if (lane == 63) ex = AM{1.0, 0.0};
    __syncthreads();
    // state entering this wave from the right, then this thread
    double xw = xr;
    for (int k = FW - 1; k > w; --k) xw = samp[k].E * xw + samp[k].U;
    double x = ex.E * xw + ex.U;
#pragma unroll
    for (int s = FS_MAX - 1; s >= 0; --s) {
      if (s < cnt) {
        x = st[s].E * x + st[s].U;
        P.xs[(int64_t)(t0 + s) * d + i] = x;
      }
    }
    // state at the chunk's first step enters the previous chunk
    if (tid == 0) carry[0] = x;
    __syncthreads();
    xr = carry[0];
    __syncthreads();
  }
  if (sbad) atomicOr(P.status, P.fail_bit);
}

}  // namespace

hipError_t launch_fact_scan(const KModel& M, FactArgs P, hipStream_t st) {
  timing_mark(FAM_FACT, 1, st);
  hipLaunchKernelGGL(k_fact_scan, dim3(M.d), dim3(FT), 0, st, M, P);
  timing_mark(FAM_FACT, 0, st);
  return hipGetLastError();
}

}  // namespace akf
