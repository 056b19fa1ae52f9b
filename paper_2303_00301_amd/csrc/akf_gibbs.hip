// akf_gibbs.hip -- one Gibbs sweep over (theta, x) of the linear-Gaussian model
// (theta = (F, log diag Q, H, log diag R), App. A eq. lgssm-app; parameter
// estimation alternating with path updates as in Sec. "Parameter estimation in
// a continuous-discrete diffusion smoothing problem").  One sweep:
//   1. MALA on log p(theta) + log p(y | theta): the log-likelihood and its
//      gradient at the proposal come from the parallel filter and the adjoint
//      scans (akf_lgssm_loglik / akf_lgssm_loglik_grad); the accept decision
//      is taken on the device (k_gibbs_decide), so nothing returns to the host;
//   2. x ~ p(x | theta, y) exactly: the filtering moments of the chosen theta
//      (the proposal's, copied when it is accepted, else those kept from
//      before) feed the parallel RTS sampler;
//   3. k auxiliary Kalman MH steps on x at theta (akf_mh_run, order 2).
// The theta move targets the theta-marginal, so step 2 must re-draw x from its
// full conditional before any step that conditions on x.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "../../include/akf.h"
#include "akf_internal.h"
#include "akf_layout.h"

using namespace akf;

namespace {

constexpr int kRedThreads = 1024;

// theta' = theta + (eps^2 / 2) g + eps xi
__global__ void k_gibbs_propose(int p, const double* __restrict__ th, const double* __restrict__ g,
                                const double* __restrict__ xi, double eps,
                                double* __restrict__ thp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p) thp[i] = th[i] + 0.5 * eps * eps * g[i] + eps * xi[i];
}

// Sum over one workgroup of kRedThreads threads in a fixed order (each
// thread's strided partial, then a tree), so results do not depend on timing.
__device__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double log_prior_const(int p, double sd) {
  return -0.5 * p * log(2.0 * M_PI * sd * sd);
}

// Log posterior and gradient at a starting theta: lp = ll + log N(theta; 0,
// sd^2 I), g <- g - theta / sd^2 (g holds d ll / d theta on entry).
__global__ void __launch_bounds__(kRedThreads) k_gibbs_post(int p, const double* th,
                                                            const double* ll, double sd,
                                                            double* lp, double* g) {
  __shared__ double sh[kRedThreads];
  const double iv = 1.0 / (sd * sd);
  double s = 0.0;
  for (int i = threadIdx.x; i < p; i += kRedThreads) {
    s += th[i] * th[i];
    g[i] -= th[i] * iv;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) *lp = *ll - 0.5 * s * iv + log_prior_const(p, sd);
}

struct DecideArgs {
  int p;
  double sd, eps;
  double* th;          // current theta (replaced by the proposal on acceptance)
  double* g;           // its gradient of the log posterior
  double* lp;          // its log posterior
  const double* thp;   // proposal
  double* gp;          // in: d ll / d theta at the proposal; out: d log posterior
  const double* llp;   // log-likelihood at the proposal (NaN if its filter failed)
  const int* statp;    // status of the proposal's filter and adjoint
  const double* u;     // uniform in (0, 1)
  int* flag;           // 1 = accepted (read by the moment copy)
  int* acc_out;        // optional
  double* la_out;      // optional
};

// MALA decision on one workgroup:
//   log alpha = lp' - lp + log q(theta | theta') - log q(theta' | theta),
//   log q(a | b) = -|a - b - (eps^2/2) grad(b)|^2 / (2 eps^2) (constants cancel);
// accept iff the proposal's status is clear, log alpha is finite and
// log u < log alpha.  On acceptance theta, its gradient and log posterior are
// replaced by the proposal's.
__global__ void __launch_bounds__(kRedThreads) k_gibbs_decide(DecideArgs A) {
  __shared__ double sh[kRedThreads];
  __shared__ int acc_sh;
  const double iv = 1.0 / (A.sd * A.sd);
  const double h = 0.5 * A.eps * A.eps;
  double s_th = 0.0, s_fwd = 0.0, s_rev = 0.0;
  for (int i = threadIdx.x; i < A.p; i += kRedThreads) {
    const double tp = A.thp[i], t = A.th[i];
    const double gpi = A.gp[i] - tp * iv;
    A.gp[i] = gpi;
    s_th += tp * tp;
    const double rf = tp - t - h * A.g[i];
    const double rr = t - tp - h * gpi;
    s_fwd += rf * rf;
    s_rev += rr * rr;
  }
  s_th = block_sum(s_th, sh);
  s_fwd = block_sum(s_fwd, sh);
  s_rev = block_sum(s_rev, sh);
  if (threadIdx.x == 0) {
    const double lpp = *A.llp - 0.5 * s_th * iv + log_prior_const(A.p, A.sd);
    const double inv2e2 = 0.5 / (A.eps * A.eps);
    const double la = lpp - *A.lp - s_rev * inv2e2 + s_fwd * inv2e2;
    const int acc = (*A.statp == 0) && isfinite(la) && (log(*A.u) < la);
    acc_sh = acc;
    *A.flag = acc;
    if (A.acc_out) *A.acc_out = acc;
    if (A.la_out) *A.la_out = la;
    if (acc) *A.lp = lpp;
  }
  __syncthreads();
  if (acc_sh) {
    for (int i = threadIdx.x; i < A.p; i += kRedThreads) {
      A.th[i] = A.thp[i];
      A.g[i] = A.gp[i];
    }
  }
}

// Filtering moments of the chosen theta into the state (leading dimension ld
// -> d), when *flag is set (always when flag is null).
__global__ void k_gibbs_moments(const int* flag, const double* __restrict__ mf_src,
                                const double* __restrict__ Pf_src, int ld, double* __restrict__ mf,
                                double* __restrict__ Pf, int N, int d) {
  if (flag && !*flag) return;
  const int64_t nP = (int64_t)N * d * d, nm = (int64_t)N * d;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nP + nm; e += stride) {
    if (e < nP) {
      const int64_t t = e / (d * d);
      const int r = (int)(e % (d * d));
      const int i = r / d, j = r % d;
      Pf[e] = Pf_src[(t * ld + i) * ld + j];
    } else {
      const int64_t f = e - nP;
      const int64_t t = f / d;
      const int i = (int)(f % d);
      mf[f] = mf_src[t * ld + i];
    }
  }
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int n_params(const akf_lgssm* m) { return m->dx * m->dx + m->dx + m->dy * m->dx + m->dy; }

// The model of the sweep at a flat theta (F, logq, H, logr views into it).
akf_lgssm at_theta(const akf_lgssm* m, const double* th) {
  akf_lgssm s = *m;
  s.F = th;
  s.logq = th + m->dx * m->dx;
  s.H = s.logq + m->dx;
  s.logr = s.H + m->dy * m->dx;
  return s;
}

// akf_model of the same linear-Gaussian model for the sampler and the path
// steps: F, H from theta, Q, R dense from the state.
akf_model as_model(const akf_lgssm* m, const double* th, const double* Q, const double* R) {
  akf_model s{};
  s.N = m->N;
  s.dx = m->dx;
  s.dy = m->dy;
  s.m0 = m->m0;
  s.P0 = m->P0;
  s.F = th;
  s.b = nullptr;
  s.Q = Q;
  s.emit = AKF_EMIT_GAUSSIAN;
  s.H = th + m->dx * m->dx + m->dx;
  s.R = R;
  s.dyn = AKF_DYN_LINEAR;
  s.dtype = AKF_F64;
  return s;
}

struct StateLayout {
  size_t mf, Pf, Q, R, total;
};

StateLayout state_layout(const akf_lgssm* m) {
  StateLayout S{};
  size_t o = 0;
  S.mf = o;
  o = align_up(o + sizeof(double) * (size_t)m->N * m->dx);
  S.Pf = o;
  o = align_up(o + sizeof(double) * (size_t)m->N * m->dx * m->dx);
  S.Q = o;
  o = align_up(o + sizeof(double) * (size_t)m->dx * m->dx);
  S.R = o;
  o = align_up(o + sizeof(double) * (size_t)m->dy * m->dy);
  S.total = o;
  return S;
}

struct WsLayout {
  size_t inner;  // shared by the likelihood/adjoint, the sampler and the path steps
  size_t thp, gp, llp, statp, flag, total;
};

// Placeholder (never dereferenced) pointers for the size queries of the inner calls.
const double* kNoPtr = reinterpret_cast<const double*>(kAlign);

bool ws_layout(const akf_lgssm* m, int block, WsLayout& W) {
  const akf_lgssm lg = at_theta(m, kNoPtr);
  const akf_model mod = as_model(m, kNoPtr, kNoPtr, kNoPtr);
  const size_t a = akf_lgssm_workspace_bytes(&lg, block);
  const size_t b = akf_sampler_workspace_bytes(&mod, block);
  const size_t c = akf_mh_workspace_bytes(&mod, 2, block);
  if (!a || !b || !c) return false;
  const int p = n_params(m);
  size_t o = align_up(std::max(a, std::max(b, c)));
  W.inner = 0;
  W.thp = o;
  o = align_up(o + sizeof(double) * p);
  W.gp = o;
  o = align_up(o + sizeof(double) * p);
  W.llp = o;
  o = align_up(o + sizeof(double));
  W.statp = o;
  o = align_up(o + sizeof(int));
  W.flag = o;
  o = align_up(o + sizeof(int));
  W.total = o;
  return true;
}

akf_status check_gibbs(const akf_lgssm* m, double prior_sd) {
  if (!m) return fail(AKF_ERR_INVALID, "lgssm is NULL");
  if (m->N < 1) return fail(AKF_ERR_SHAPE, "N must be >= 1 (got %d)", m->N);
  if (m->dx < 1 || m->dx > 32)
    return fail(AKF_ERR_SHAPE, "dx must be in [1, 32] for the Gibbs sweep (got %d)", m->dx);
  if (m->dy < 1 || m->dy > 32)
    return fail(AKF_ERR_SHAPE, "dy must be in [1, 32] for the Gibbs sweep (got %d)", m->dy);
  if (!m->m0 || !m->P0 || !m->y) return fail(AKF_ERR_INVALID, "m0, P0 and y must be non-NULL");
  if (!(prior_sd > 0.0) || !isfinite(prior_sd))
    return fail(AKF_ERR_INVALID, "prior_sd must be finite and > 0");
  return AKF_OK;
}

akf_status check_buffers(const akf_lgssm* m, void* state, size_t state_bytes, void* ws,
                         size_t ws_bytes, int block, WsLayout& W) {
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  if (!ws_layout(m, block, W)) return fail(AKF_ERR_SHAPE, "unsupported sizes for the Gibbs sweep");
  if (!ws || reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(AKF_ERR_WORKSPACE, "workspace must be non-NULL and %zu-byte aligned", kAlign);
  if (ws_bytes < W.total)
    return fail(AKF_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, W.total);
  const StateLayout S = state_layout(m);
  if (!state || reinterpret_cast<uintptr_t>(state) % kAlign)
    return fail(AKF_ERR_WORKSPACE, "state must be non-NULL and %zu-byte aligned", kAlign);
  if (state_bytes < S.total)
    return fail(AKF_ERR_WORKSPACE, "state too small: %zu < %zu bytes", state_bytes, S.total);
  return AKF_OK;
}

// Filtering moments (from the likelihood call's workspace, under `flag`) and
// the dense Q, R of theta into the state.
akf_status keep_theta(const akf_lgssm* m, const double* th, const int* flag, void* state,
                      void* ws, int block, hipStream_t st) {
  Layout Lo;
  const akf_lgssm lg = at_theta(m, th);
  lgssm_layout(Lo, &lg, block);
  const StateLayout S = state_layout(m);
  const int64_t n = (int64_t)m->N * m->dx * (m->dx + 1);
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_gibbs_moments, dim3(grid), dim3(256), 0, st, flag,
                     at<double>(ws, Lo.mf), at<double>(ws, Lo.Pf), Lo.D, at<double>(state, S.mf),
                     at<double>(state, S.Pf), m->N, m->dx);
  akf_status s;
  if ((s = hip_check(hipGetLastError(), "moment copy launch")) != AKF_OK) return s;
  LgArgs G{};
  G.dx = m->dx;
  G.dy = m->dy;
  G.logq = lg.logq;
  G.logr = lg.logr;
  G.Q = at<double>(state, S.Q);
  G.R = at<double>(state, S.R);
  return hip_check(launch_lgssm_prep(G, st), "Q, R launch");
}

// log p(y | theta) and its gradient into ll [1] and g [p] (flat layout), with
// the status of both passes in *stat.
akf_status loglik_and_grad(const akf_lgssm* m, const double* th, double* ll, double* g, int* stat,
                           void* ws, size_t ws_bytes, int block, hipStream_t st) {
  const akf_lgssm lg = at_theta(m, th);
  akf_status s;
  if ((s = akf_lgssm_loglik(&lg, ll, nullptr, nullptr, ws, ws_bytes, block, st)) != AKF_OK)
    return s;
  double* dF = g;
  double* dq = dF + m->dx * m->dx;
  double* dH = dq + m->dx;
  double* dr = dH + m->dy * m->dx;
  return akf_lgssm_loglik_grad(&lg, nullptr, dF, dq, dH, dr, stat, ws, ws_bytes, block, st);
}

}  // namespace

extern "C" {

size_t akf_gibbs_state_bytes(const akf_lgssm* m) {
  if (check_gibbs(m, 1.0) != AKF_OK) return 0;
  return state_layout(m).total;
}

size_t akf_gibbs_workspace_bytes(const akf_lgssm* m, int32_t block) {
  if (check_gibbs(m, 1.0) != AKF_OK || block < 0) return 0;
  WsLayout W;
  return ws_layout(m, block, W) ? W.total : 0;
}

akf_status akf_gibbs_init(const akf_lgssm* m, const double* theta, double prior_sd,
                          double* logpost, double* grad, void* state, size_t state_bytes,
                          int32_t* status, void* ws, size_t ws_bytes, int32_t block,
                          void* stream) {
  akf_status s;
  if ((s = check_gibbs(m, prior_sd)) != AKF_OK) return s;
  if (!theta || !logpost || !grad)
    return fail(AKF_ERR_INVALID, "theta, logpost and grad must be non-NULL");
  WsLayout W;
  if ((s = check_buffers(m, state, state_bytes, ws, ws_bytes, block, W)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  double* ll = at<double>(ws, W.llp);
  int* stat = at<int>(ws, W.statp);
  if ((s = loglik_and_grad(m, theta, ll, grad, stat, ws, W.thp, block, st)) != AKF_OK) return s;
  hipLaunchKernelGGL(k_gibbs_post, dim3(1), dim3(kRedThreads), 0, st, n_params(m), theta, ll,
                     prior_sd, logpost, grad);
  if ((s = hip_check(hipGetLastError(), "posterior launch")) != AKF_OK) return s;
  if ((s = keep_theta(m, theta, nullptr, state, ws, block, st)) != AKF_OK) return s;
  if (status)
    return hip_check(hipMemcpyAsync(status, stat, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy");
  return AKF_OK;
}

akf_status akf_gibbs_sweep(const akf_lgssm* m, double* theta, double* logpost, double* grad,
                           double* x, void* state, size_t state_bytes, double prior_sd, double eps,
                           const double* xi_theta, const double* u_theta, const double* xi_x,
                           double delta, int32_t n_path, const double* xi_path,
                           const double* u_path, int32_t* accepted_theta, double* log_alpha,
                           double* path_log_ratio, int32_t* path_accepted, int32_t* path_status,
                           int32_t* status, void* ws, size_t ws_bytes, int32_t block,
                           void* stream) {
  akf_status s;
  if ((s = check_gibbs(m, prior_sd)) != AKF_OK) return s;
  if (!theta || !logpost || !grad || !x || !xi_theta || !u_theta || !xi_x)
    return fail(AKF_ERR_INVALID,
                "theta, logpost, grad, x, xi_theta, u_theta and xi_x must be non-NULL");
  if (!(eps > 0.0) || !isfinite(eps)) return fail(AKF_ERR_INVALID, "eps must be finite and > 0");
  if (n_path < 0) return fail(AKF_ERR_INVALID, "n_path must be >= 0");
  if (n_path > 0 && (!xi_path || !u_path || !(delta > 0.0)))
    return fail(AKF_ERR_INVALID, "path steps need xi_path, u_path and delta > 0");
  WsLayout W;
  if ((s = check_buffers(m, state, state_bytes, ws, ws_bytes, block, W)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int p = n_params(m);
  double* thp = at<double>(ws, W.thp);
  double* gp = at<double>(ws, W.gp);
  double* llp = at<double>(ws, W.llp);
  int* statp = at<int>(ws, W.statp);
  int* flag = at<int>(ws, W.flag);
  const size_t inner = W.thp;  // bytes of the shared region at the start of ws
  // 1. MALA proposal, its log-likelihood and gradient, the decision
  hipLaunchKernelGGL(k_gibbs_propose, dim3((p + 255) / 256), dim3(256), 0, st, p, theta, grad,
                     xi_theta, eps, thp);
  if ((s = hip_check(hipGetLastError(), "proposal launch")) != AKF_OK) return s;
  if ((s = loglik_and_grad(m, thp, llp, gp, statp, ws, inner, block, st)) != AKF_OK) return s;
  DecideArgs A{};
  A.p = p;
  A.sd = prior_sd;
  A.eps = eps;
  A.th = theta;
  A.g = grad;
  A.lp = logpost;
  A.thp = thp;
  A.gp = gp;
  A.llp = llp;
  A.statp = statp;
  A.u = u_theta;
  A.flag = flag;
  A.acc_out = accepted_theta;
  A.la_out = log_alpha;
  hipLaunchKernelGGL(k_gibbs_decide, dim3(1), dim3(kRedThreads), 0, st, A);
  if ((s = hip_check(hipGetLastError(), "decision launch")) != AKF_OK) return s;
  if (status &&
      (s = hip_check(hipMemcpyAsync(status, statp, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy")) != AKF_OK)
    return s;
  // 2. the state follows the chosen theta; exact draw of x given it
  if ((s = keep_theta(m, theta, flag, state, ws, block, st)) != AKF_OK) return s;
  const StateLayout S = state_layout(m);
  const akf_model mod =
      as_model(m, theta, at<double>(state, S.Q), at<double>(state, S.R));
  if ((s = akf_rts_sample(&mod, at<double>(state, S.mf), at<double>(state, S.Pf), xi_x, x,
                          status ? status + 1 : nullptr, ws, inner, block, stream)) != AKF_OK)
    return s;
  // 3. auxiliary Kalman path steps at theta
  if (n_path > 0)
    return akf_mh_run(&mod, m->y, x, delta, 2, n_path, xi_path, u_path, path_log_ratio,
                      path_accepted, nullptr, nullptr, path_status, ws, inner, block, stream);
  return AKF_OK;
}

}  // extern "C"
