// akf_capi.cpp -- C ABI of libauxkf: argument validation, workspace layout and
// the launch sequence of one auxiliary Kalman MH step (see include/akf.h).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "../../include/akf.h"
#include "akf_internal.h"

using namespace akf;

namespace {

thread_local char g_err[512] = "";

akf_status fail(akf_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int pick_D(int d) { return d <= 16 ? 16 : (d <= 32 ? 32 : (d <= 64 ? 64 : 0)); }

// Default scan block: enough blocks to give every CU (256) its resident teams
// (LDS-limited: 1 team of 4 waves at D = 64, several single-wave teams below),
// and at least 4 steps per block so that small problems do not pay for a deep
// tree of tiny launches.
int auto_block(int N, int D) {
  const int teams_per_cu = D == 64 ? 1 : (D == 32 ? 4 : 8);
  const int target = 256 * teams_per_cu;
  int B = (N + target - 1) / target;
  if (B < 4) B = 4;
  if (B > N) B = N;
  return B;
}

constexpr int kMaxLevels = 32;

struct Layout {
  int N = 0, d = 0, dy = 0, D = 0, B = 0, nb = 0, L = 0;
  int n_lvl[kMaxLevels + 1] = {0};
  int n_part = 0;
  // byte offsets
  size_t u = 0, om = 0, Om = 0, om2 = 0, Om2 = 0, xs = 0, ell = 0, ell2 = 0;
  size_t plhx = 0, plhxs = 0, pterms = 0;
  size_t gG = 0, gRinv = 0, gOmd = 0, gOmdinv = 0, gscal = 0;
  size_t elem[kMaxLevels + 1] = {0};
  size_t pre[kMaxLevels + 1] = {0};
  size_t mf = 0, Pf = 0, E = 0, U = 0;
  size_t sagg[kMaxLevels + 1] = {0};
  size_t xin[kMaxLevels + 1] = {0};
  size_t status = 0, accept = 0;
  size_t total = 0;
};

enum LayoutKind { LAYOUT_STEP = 0, LAYOUT_FILTER = 1, LAYOUT_SAMPLER = 2 };

void make_layout(Layout& Lo, int N, int d, int dy, int block, int kind) {
  Lo.N = N;
  Lo.d = d;
  Lo.dy = dy;
  Lo.D = pick_D(d);
  const int D = Lo.D;
  Lo.B = block > 0 ? (block > N ? N : block) : auto_block(N, D);
  Lo.nb = (N + Lo.B - 1) / Lo.B;
  Lo.n_lvl[0] = Lo.nb;
  Lo.L = 0;
  while (Lo.n_lvl[Lo.L] > 1 && Lo.L < kMaxLevels) {
    Lo.n_lvl[Lo.L + 1] = (Lo.n_lvl[Lo.L] + 1) / 2;
    ++Lo.L;
  }
  const size_t dbl = sizeof(double);
  const size_t vn = (size_t)N * d * dbl;
  const size_t ES = (size_t)(3 * D * D + 2 * D) * dbl;
  const size_t PS = (size_t)(D * D + D + 2) * dbl;
  const size_t SS = (size_t)(D * D + D) * dbl;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes == 0 ? 1 : bytes);
    return o;
  };
  const int nparts_diag = (int)(((int64_t)N * d + 255) / 256);
  const int nparts_gauss = (N + 63) / 64;
  Lo.n_part = nparts_diag > nparts_gauss ? nparts_diag : nparts_gauss;
  if (kind == LAYOUT_STEP) {
    Lo.u = take(vn);
    Lo.om = take(vn);
    Lo.Om = take(vn);
    Lo.om2 = take(vn);
    Lo.Om2 = take(vn);
    Lo.xs = take(vn);
    Lo.ell2 = take((size_t)N * dbl);
    Lo.plhx = take((size_t)Lo.n_part * dbl);
    Lo.plhxs = take((size_t)Lo.n_part * dbl);
    Lo.pterms = take((size_t)Lo.n_part * dbl);
    Lo.gG = take((size_t)d * (dy > 0 ? dy : 1) * dbl);
    Lo.gRinv = take((size_t)(dy > 0 ? dy * dy : 1) * dbl);
    Lo.gOmd = take((size_t)d * d * dbl);
    Lo.gOmdinv = take((size_t)d * d * dbl);
    Lo.gscal = take(8 * dbl);
    Lo.accept = take(sizeof(int));
  }
  if (kind == LAYOUT_STEP || kind == LAYOUT_FILTER) {
    Lo.ell = take((size_t)N * dbl);
    for (int l = 0; l <= Lo.L; ++l) Lo.elem[l] = take((size_t)Lo.n_lvl[l] * ES);
    for (int l = 0; l <= Lo.L; ++l) Lo.pre[l] = take((size_t)Lo.n_lvl[l] * PS);
  }
  if (kind == LAYOUT_STEP) {
    Lo.mf = take((size_t)N * D * dbl);
    Lo.Pf = take((size_t)N * D * D * dbl);
  }
  if (kind == LAYOUT_STEP || kind == LAYOUT_SAMPLER) {
    Lo.E = take((size_t)N * D * D * dbl);
    Lo.U = take((size_t)N * D * dbl);
    for (int l = 0; l <= Lo.L; ++l) Lo.sagg[l] = take((size_t)Lo.n_lvl[l] * SS);
    for (int l = 0; l <= Lo.L; ++l) Lo.xin[l] = take((size_t)Lo.n_lvl[l] * D * dbl);
  }
  Lo.status = take(sizeof(int));
  Lo.total = off;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

akf_status check_model(const akf_model* m, bool need_emission) {
  if (!m) return fail(AKF_ERR_INVALID, "model is NULL");
  if (m->N < 1) return fail(AKF_ERR_SHAPE, "N must be >= 1 (got %d)", m->N);
  if (m->dx < 1 || m->dx > 64) return fail(AKF_ERR_SHAPE, "dx must be in [1, 64] (got %d)", m->dx);
  if (!m->m0 || !m->P0 || !m->F || !m->Q)
    return fail(AKF_ERR_INVALID, "m0, P0, F and Q must be non-NULL");
  if (!need_emission) return AKF_OK;
  if (m->dy < 1 || m->dy > 64) return fail(AKF_ERR_SHAPE, "dy must be in [1, 64] (got %d)", m->dy);
  switch (m->emit) {
    case AKF_EMIT_GAUSSIAN:
      if (!m->H || !m->R) return fail(AKF_ERR_INVALID, "Gaussian emission needs H and R");
      break;
    case AKF_EMIT_POISSON_LOG:
      if (!m->site) return fail(AKF_ERR_INVALID, "Poisson emission needs site");
      break;
    case AKF_EMIT_STUDENT_T:
      if (!m->site) return fail(AKF_ERR_INVALID, "Student-t emission needs site");
      if (!(m->nu > 0.0) || !(m->scale > 0.0))
        return fail(AKF_ERR_INVALID, "Student-t emission needs nu > 0 and scale > 0");
      break;
    default:
      return fail(AKF_ERR_INVALID, "unknown emission family %d", m->emit);
  }
  return AKF_OK;
}

KModel to_kmodel(const akf_model* m) {
  KModel M;
  M.N = m->N;
  M.d = m->dx;
  M.dy = m->dy;
  M.emit = m->emit;
  M.m0 = m->m0;
  M.P0 = m->P0;
  M.F = m->F;
  M.b = m->b;
  M.Q = m->Q;
  M.H = m->H;
  M.R = m->R;
  M.site = m->site;
  M.nu = m->nu;
  M.scale = m->scale;
  return M;
}

akf_status prepare_device() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] { err = set_lds_limits_all(); });
  if (err != hipSuccess)
    return fail(AKF_ERR_HIP, "setting LDS limits failed: %s", hipGetErrorString(err));
  return AKF_OK;
}

akf_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(AKF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return AKF_OK;
}

void fill_tree(const Layout& Lo, void* ws, size_t elem_size, const size_t* lvl_elem,
               const size_t* lvl_pre, int* status, int fail_bit, TreeArgs* up, TreeArgs* down) {
  for (int l = 1; l <= Lo.L; ++l) {
    TreeArgs u{};
    u.src = at<double>(ws, lvl_elem[l - 1]);
    u.dst = at<double>(ws, lvl_elem[l]);
    u.n_src = Lo.n_lvl[l - 1];
    u.n_dst = Lo.n_lvl[l];
    u.status = status;
    u.fail_bit = fail_bit;
    up[l - 1] = u;
    TreeArgs d{};
    d.src = at<double>(ws, lvl_elem[l - 1]);
    d.pre_src = at<double>(ws, lvl_pre[l]);
    d.pre_dst = at<double>(ws, lvl_pre[l - 1]);
    d.n_src = Lo.n_lvl[l];
    d.n_dst = Lo.n_lvl[l - 1];
    d.status = status;
    d.fail_bit = fail_bit;
    down[l - 1] = d;
  }
  (void)elem_size;
}

// root prefix flag (identity) of the filter tree
double* root_flag(const Layout& Lo, void* ws) {
  return at<double>(ws, Lo.pre[Lo.L]) + (Lo.D * Lo.D + Lo.D);
}

akf_status run_filter(const Layout& Lo, const KModel& M, void* ws, const double* om,
                      const double* Om, const double* Omd, double* mf, double* Pf, int ldm,
                      double* ell, int* status, int fail_bit, hipStream_t st) {
  FilterArgs P{};
  P.B = Lo.B;
  P.om = om;
  P.Om = Om;
  P.Omd = Omd;
  P.elem = at<double>(ws, Lo.elem[0]);
  P.pre = at<double>(ws, Lo.pre[0]);
  P.mf = mf;
  P.Pf = Pf;
  P.ldm = ldm;
  P.ell = ell;
  P.status = status;
  P.fail_bit = fail_bit;
  TreeArgs up[kMaxLevels], down[kMaxLevels];
  fill_tree(Lo, ws, 0, Lo.elem, Lo.pre, status, fail_bit, up, down);
  return hip_check(launch_filter_any(Lo.D, M, P, up, down, Lo.L, st), "filter launch");
}

akf_status run_sampler(const Layout& Lo, const KModel& M, void* ws, const double* mf,
                       const double* Pf, int ldm, const double* xi_x, double* xs, int* status,
                       hipStream_t st) {
  SampArgs S{};
  S.B = Lo.B;
  S.mf = mf;
  S.Pf = Pf;
  S.ldm = ldm;
  S.xi_x = xi_x;
  S.E = at<double>(ws, Lo.E);
  S.U = at<double>(ws, Lo.U);
  S.agg = at<double>(ws, Lo.sagg[0]);
  S.xin = at<double>(ws, Lo.xin[0]);
  S.xs = xs;
  S.status = status;
  TreeArgs up[kMaxLevels], down[kMaxLevels];
  fill_tree(Lo, ws, 0, Lo.sagg, Lo.xin, status, ST_FWD_NOT_PD, up, down);
  return hip_check(launch_sampler_any(Lo.D, M, S, up, down, Lo.L, st), "sampler launch");
}

akf_status mh_step_impl(const Layout& Lo, const KModel& M, const double* y, const double* x_in,
                        double delta, int order, const double* xi, const double* unif,
                        double* x_out, double* log_ratio, int32_t* accepted, double* logZ_fwd,
                        double* logZ_rev, int32_t* status_out, void* ws, hipStream_t st) {
  const size_t vn = (size_t)M.N * M.d;
  int* status = at<int>(ws, Lo.status);
  StepArgs A{};
  A.y = y;
  A.x = x_in;
  A.xi_u = xi;
  A.delta = delta;
  A.order = order;
  A.u = at<double>(ws, Lo.u);
  A.om = at<double>(ws, Lo.om);
  A.Om = at<double>(ws, Lo.Om);
  A.om2 = at<double>(ws, Lo.om2);
  A.Om2 = at<double>(ws, Lo.Om2);
  A.xs = at<double>(ws, Lo.xs);
  A.ell = at<double>(ws, Lo.ell);
  A.ell2 = at<double>(ws, Lo.ell2);
  A.part_lh_x = at<double>(ws, Lo.plhx);
  A.part_lh_xs = at<double>(ws, Lo.plhxs);
  A.part_terms = at<double>(ws, Lo.pterms);
  A.g_G = at<double>(ws, Lo.gG);
  A.g_Rinv = at<double>(ws, Lo.gRinv);
  A.g_Omd = at<double>(ws, Lo.gOmd);
  A.g_Omd_inv = at<double>(ws, Lo.gOmdinv);
  A.g_scal = at<double>(ws, Lo.gscal);
  A.status = status;
  A.accept_flag = at<int>(ws, Lo.accept);
  akf_status s;
  if ((s = hip_check(launch_step_init(status, root_flag(Lo, ws), at<double>(ws, Lo.xin[Lo.L]),
                                      Lo.D, st),
                     "init launch")) != AKF_OK)
    return s;
  int n_part_fwd = 0, n_part_rev = 0;
  if ((s = hip_check(launch_lin(M, A, 0, &n_part_fwd, st), "linearise launch")) != AKF_OK) return s;
  const double* Omd = (M.emit == EMIT_GAUSSIAN && order == 2) ? A.g_Omd : nullptr;
  double* mf = at<double>(ws, Lo.mf);
  double* Pf = at<double>(ws, Lo.Pf);
  if ((s = run_filter(Lo, M, ws, A.om, A.Om, Omd, mf, Pf, Lo.D, A.ell, status, ST_FWD_NOT_PD,
                      st)) != AKF_OK)
    return s;
  if ((s = run_sampler(Lo, M, ws, mf, Pf, Lo.D, xi + vn, A.xs, status, st)) != AKF_OK) return s;
  if ((s = hip_check(launch_lin(M, A, 1, &n_part_rev, st), "linearise launch")) != AKF_OK) return s;
  if ((s = run_filter(Lo, M, ws, A.om2, A.Om2, Omd, nullptr, nullptr, Lo.D, A.ell2, status,
                      ST_REV_NOT_PD, st)) != AKF_OK)
    return s;
  FinalArgs F{};
  F.unif = unif;
  F.log_ratio = log_ratio;
  F.accepted = accepted;
  F.logZ_fwd = logZ_fwd;
  F.logZ_rev = logZ_rev;
  F.status_out = status_out;
  F.n_part_fwd = n_part_fwd;
  F.n_part_rev = n_part_rev;
  return hip_check(launch_finalize(M, A, F, x_in, x_out, st), "finalize launch");
}

// ---- kernel timing hook -------------------------------------------------
struct TimingState {
  std::mutex mu;
  int family = -1;
  int capacity = 0;
  int used = 0;
  int open = 0;  // a begin event is pending
  hipEvent_t* ev = nullptr;  // 2 * capacity
};
TimingState g_timing;

void timing_release_locked() {
  for (int i = 0; i < 2 * g_timing.capacity; ++i) (void)hipEventDestroy(g_timing.ev[i]);
  delete[] g_timing.ev;
  g_timing.ev = nullptr;
  g_timing.capacity = g_timing.used = g_timing.open = 0;
  g_timing.family = -1;
}

akf_status check_ws(const Layout& Lo, void* ws, size_t ws_bytes) {
  if (!ws) return fail(AKF_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % kAlign)
    return fail(AKF_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
  if (ws_bytes < Lo.total)
    return fail(AKF_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, Lo.total);
  return AKF_OK;
}

}  // namespace

namespace akf {
void timing_mark(int family, int begin, hipStream_t st) {
  if (g_timing.family != family) return;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (g_timing.family != family || !g_timing.ev) return;
  if (begin) {
    if (g_timing.used >= g_timing.capacity) return;
    (void)hipEventRecord(g_timing.ev[2 * g_timing.used], st);
    g_timing.open = 1;
  } else if (g_timing.open) {
    (void)hipEventRecord(g_timing.ev[2 * g_timing.used + 1], st);
    g_timing.open = 0;
    ++g_timing.used;
  }
}
}  // namespace akf

extern "C" {

akf_status akf_timing_enable(int32_t family, int32_t capacity) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  timing_release_locked();
  if (family < 0) return AKF_OK;
  if (family >= FAM_COUNT) return fail(AKF_ERR_INVALID, "unknown kernel family %d", family);
  if (capacity < 1 || capacity > (1 << 20))
    return fail(AKF_ERR_INVALID, "capacity must be in [1, 2^20]");
  g_timing.ev = new hipEvent_t[2 * capacity];
  for (int i = 0; i < 2 * capacity; ++i) {
    hipError_t e = hipEventCreate(&g_timing.ev[i]);
    if (e != hipSuccess) {
      g_timing.capacity = i / 2;
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(g_timing.ev[j]);
      delete[] g_timing.ev;
      g_timing.ev = nullptr;
      g_timing.capacity = 0;
      return fail(AKF_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
  }
  g_timing.capacity = capacity;
  g_timing.family = family;
  return AKF_OK;
}

akf_status akf_timing_collect(int32_t* n_launches, double* total_ms) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (!n_launches || !total_ms) return fail(AKF_ERR_INVALID, "outputs must be non-NULL");
  double tot = 0.0;
  for (int i = 0; i < g_timing.used; ++i) {
    hipError_t e = hipEventSynchronize(g_timing.ev[2 * i + 1]);
    if (e != hipSuccess) return fail(AKF_ERR_HIP, "hipEventSynchronize: %s", hipGetErrorString(e));
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, g_timing.ev[2 * i], g_timing.ev[2 * i + 1]);
    if (e != hipSuccess) return fail(AKF_ERR_HIP, "hipEventElapsedTime: %s", hipGetErrorString(e));
    tot += ms;
  }
  *n_launches = g_timing.used;
  *total_ms = tot;
  g_timing.used = 0;
  g_timing.open = 0;
  return AKF_OK;
}

const char* akf_last_error(void) { return g_err; }

size_t akf_mh_workspace_bytes(const akf_model* model, int32_t order, int32_t block) {
  if (check_model(model, true) != AKF_OK || (order != 1 && order != 2)) return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP);
  return Lo.total;
}

akf_status akf_mh_step(const akf_model* model, const double* y, const double* x_in, double delta,
                       int32_t order, const double* xi, const double* unif, double* x_out,
                       double* log_ratio, int32_t* accepted, double* logZ_fwd, double* logZ_rev,
                       int32_t* status, void* ws, size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_model(model, true)) != AKF_OK) return s;
  if (!y || !x_in || !xi || !unif || !x_out)
    return fail(AKF_ERR_INVALID, "y, x_in, xi, unif and x_out must be non-NULL");
  if (!(delta > 0.0)) return fail(AKF_ERR_INVALID, "delta must be > 0");
  if (order != 1 && order != 2) return fail(AKF_ERR_INVALID, "order must be 1 or 2");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  return mh_step_impl(Lo, to_kmodel(model), y, x_in, delta, order, xi, unif, x_out, log_ratio,
                      accepted, logZ_fwd, logZ_rev, status, ws, (hipStream_t)stream);
}

akf_status akf_mh_run(const akf_model* model, const double* y, double* x, double delta,
                      int32_t order, int32_t n_steps, const double* xi, const double* unif,
                      double* log_ratio, int32_t* accepted, double* logZ_fwd, double* logZ_rev,
                      int32_t* status, void* ws, size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_model(model, true)) != AKF_OK) return s;
  if (!y || !x || !xi || !unif) return fail(AKF_ERR_INVALID, "y, x, xi and unif must be non-NULL");
  if (n_steps < 0) return fail(AKF_ERR_INVALID, "n_steps must be >= 0");
  if (!(delta > 0.0)) return fail(AKF_ERR_INVALID, "delta must be > 0");
  if (order != 1 && order != 2) return fail(AKF_ERR_INVALID, "order must be 1 or 2");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  const KModel M = to_kmodel(model);
  const size_t vn = (size_t)M.N * M.d;
  for (int k = 0; k < n_steps; ++k) {
    s = mh_step_impl(Lo, M, y, x, delta, order, xi + (size_t)k * 2 * vn, unif + k, x,
                     log_ratio ? log_ratio + k : nullptr, accepted ? accepted + k : nullptr,
                     logZ_fwd ? logZ_fwd + k : nullptr, logZ_rev ? logZ_rev + k : nullptr,
                     status ? status + k : nullptr, ws, (hipStream_t)stream);
    if (s != AKF_OK) return s;
  }
  return AKF_OK;
}

size_t akf_filter_workspace_bytes(const akf_model* model, int32_t block) {
  if (check_model(model, false) != AKF_OK) return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, block, LAYOUT_FILTER);
  return Lo.total;
}

akf_status akf_aux_filter(const akf_model* model, const double* omega, const double* Omega,
                          double* mf, double* Pf, double* ell, int32_t* status, void* ws,
                          size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_model(model, false)) != AKF_OK) return s;
  if (!omega || !Omega || !ell) return fail(AKF_ERR_INVALID, "omega, Omega and ell must be non-NULL");
  if ((mf == nullptr) != (Pf == nullptr))
    return fail(AKF_ERR_INVALID, "mf and Pf must both be given or both be NULL");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, block, LAYOUT_FILTER);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  int* dstat = at<int>(ws, Lo.status);
  if ((s = hip_check(launch_step_init(dstat, root_flag(Lo, ws), nullptr, 0, st), "init launch")) !=
      AKF_OK)
    return s;
  const KModel M = to_kmodel(model);
  if ((s = run_filter(Lo, M, ws, omega, Omega, nullptr, mf, Pf, M.d, ell, dstat, ST_FWD_NOT_PD,
                      st)) != AKF_OK)
    return s;
  if (status)
    return hip_check(hipMemcpyAsync(status, dstat, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy");
  return AKF_OK;
}

size_t akf_sampler_workspace_bytes(const akf_model* model, int32_t block) {
  if (check_model(model, false) != AKF_OK) return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, block, LAYOUT_SAMPLER);
  return Lo.total;
}

akf_status akf_rts_sample(const akf_model* model, const double* mf, const double* Pf,
                          const double* xi, double* x, int32_t* status, void* ws,
                          size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_model(model, false)) != AKF_OK) return s;
  if (!mf || !Pf || !xi || !x) return fail(AKF_ERR_INVALID, "mf, Pf, xi and x must be non-NULL");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, block, LAYOUT_SAMPLER);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  int* dstat = at<int>(ws, Lo.status);
  if ((s = hip_check(launch_step_init(dstat, nullptr, at<double>(ws, Lo.xin[Lo.L]), Lo.D, st),
                     "init launch")) != AKF_OK)
    return s;
  if ((s = run_sampler(Lo, to_kmodel(model), ws, mf, Pf, model->dx, xi, x, dstat, st)) != AKF_OK)
    return s;
  if (status)
    return hip_check(hipMemcpyAsync(status, dstat, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy");
  return AKF_OK;
}

}  // extern "C"
