// akf_capi.cpp -- C ABI of libauxkf: argument validation, workspace layout and
// the launch sequence of one auxiliary Kalman MH step (see include/akf.h).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "../../include/akf.h"
#include "akf_internal.h"
#include "akf_layout.h"

using namespace akf;

namespace {

// Step `step` of a run uses status word step & 1 (see k_step_init).
StepArgs make_step_args(const Layout& Lo, void* ws, const double* y, const double* x_in,
                        double delta, int order, const double* xi, int step) {
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
  A.g_Ht = at<double>(ws, Lo.gHt);
  A.g_Rinv = at<double>(ws, Lo.gRinv);
  A.g_Omd = at<double>(ws, Lo.gOmd);
  A.g_Omd_inv = at<double>(ws, Lo.gOmdinv);
  A.g_scal = at<double>(ws, Lo.gscal);
  A.status = at<int>(ws, Lo.status) + (step & 1);
  A.accept_flag = at<int>(ws, Lo.accept);
  return A;
}

// Step `step` (0 = the first of a call) of a run on one workspace.
akf_status mh_step_impl(const Layout& Lo, const KModel& M, const double* y, const double* x_in,
                        double delta, int order, const double* xi, const double* unif,
                        double* x_out, double* log_ratio, int32_t* accepted, double* logZ_fwd,
                        double* logZ_rev, int32_t* status_out, void* ws, hipStream_t st,
                        int step) {
  const size_t vn = (size_t)M.N * M.d;
  const StepArgs A = make_step_args(Lo, ws, y, x_in, delta, order, xi, step);
  int* status = A.status;
  akf_status s;
  if (step == 0 &&
      (s = hip_check(launch_step_init(at<int>(ws, Lo.status), root_flag(Lo, ws),
                                      at<double>(ws, Lo.xin[Lo.L]), Lo.D, st),
                     "init launch")) != AKF_OK)
    return s;
  int n_part_fwd = 0, n_part_rev = 0, n_part_dyn = 0;
  if ((s = hip_check(launch_lin(M, A, 0, &n_part_fwd, st), "linearise launch")) != AKF_OK) return s;
  // nonlinear dynamics: F_t, b_t of the extended linearisation, at x here and
  // at x* (with the mismatch terms of log r) before the reverse filter
  const bool nl = M.dyn != DYN_LINEAR;
  double* Ft = nl ? at<double>(ws, Lo.Ft) : nullptr;
  double* bt = nl ? at<double>(ws, Lo.bt) : nullptr;
  DynArgs Dy{};
  Dy.Ft = Ft;
  Dy.bt = bt;
  Dy.Qinv = nl ? at<double>(ws, Lo.Qinv) : nullptr;
  if (nl) {
    Dy.a = x_in;
    if ((s = hip_check(launch_dyn_lin(M, Dy, nullptr, st), "dynamics launch")) != AKF_OK) return s;
  }
  const double* Omd = (M.emit == EMIT_GAUSSIAN && order == 2) ? A.g_Omd : nullptr;
  double* mf = at<double>(ws, Lo.mf);
  double* Pf = at<double>(ws, Lo.Pf);
  if ((s = run_filter(Lo, M, ws, A.om, A.Om, Omd, mf, Pf, Lo.D, A.ell, status, ST_FWD_NOT_PD,
                      st, nullptr, nullptr, nullptr, 0, Ft, bt)) != AKF_OK)
    return s;
  if ((s = run_sampler(Lo, M, ws, mf, Pf, Lo.D, xi + vn, A.xs, status, st, Ft, bt)) != AKF_OK)
    return s;
  if ((s = hip_check(launch_lin(M, A, 1, &n_part_rev, st), "linearise launch")) != AKF_OK) return s;
  if (nl) {
    Dy.a = A.xs;
    Dy.z = x_in;
    Dy.part = at<double>(ws, Lo.pdyn);
    if ((s = hip_check(launch_dyn_lin(M, Dy, &n_part_dyn, st), "dynamics launch")) != AKF_OK)
      return s;
  }
  // the reverse proposal needs log Z(x*) only: element normalisers reduced up
  // the block tree, no re-scan
  const double* lz_rev = nullptr;
  if ((s = run_filter_logz(Lo, M, ws, A.om2, A.Om2, Omd, status, ST_REV_NOT_PD, st, Ft, bt,
                           &lz_rev)) != AKF_OK)
    return s;
  FinalArgs F{};
  F.status_next = at<int>(ws, Lo.status) + ((step + 1) & 1);
  F.lz_rev = lz_rev;
  F.part_dyn = Dy.part;
  F.n_part_dyn = n_part_dyn;
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

// One step with a factorising prior: the same linearisation and MH decision
// as mh_step_impl, with the dense filter and sampler replaced by dx scalar
// ones (one workgroup per coordinate).
akf_status fact_step_impl(const Layout& Lo, const KModel& M, const double* y, const double* x_in,
                          double delta, int order, const double* xi, const double* unif,
                          double* x_out, double* log_ratio, int32_t* accepted, double* logZ_fwd,
                          double* logZ_rev, int32_t* status_out, void* ws, hipStream_t st,
                          int step) {
  const size_t vn = (size_t)M.N * M.d;
  const StepArgs A = make_step_args(Lo, ws, y, x_in, delta, order, xi, step);
  int* status = A.status;
  akf_status s;
  if (step == 0 && (s = hip_check(launch_step_init(at<int>(ws, Lo.status), nullptr, nullptr, 0, st),
                                  "init launch")) != AKF_OK)
    return s;
  int n_part_fwd = 0, n_part_rev = 0;
  if ((s = hip_check(launch_lin(M, A, 0, &n_part_fwd, st), "linearise launch")) != AKF_OK) return s;
  FactArgs P{};
  P.om = A.om;
  P.Om = A.Om;
  P.xi_x = xi + vn;
  P.xs = A.xs;
  P.mf = at<double>(ws, Lo.mf);
  P.Pf = at<double>(ws, Lo.Pf);
  P.lz = A.ell;
  P.status = status;
  P.fail_bit = ST_FWD_NOT_PD;
  if ((s = hip_check(launch_fact_scan(M, P, st), "factorised scan launch")) != AKF_OK) return s;
  if ((s = hip_check(launch_lin(M, A, 1, &n_part_rev, st), "linearise launch")) != AKF_OK) return s;
  FactArgs R{};
  R.om = A.om2;
  R.Om = A.Om2;
  R.lz = A.ell2;
  R.status = status;
  R.fail_bit = ST_REV_NOT_PD;
  if ((s = hip_check(launch_fact_scan(M, R, st), "factorised scan launch")) != AKF_OK) return s;
  FinalArgs F{};
  F.status_next = at<int>(ws, Lo.status) + ((step + 1) & 1);
  F.n_ell = M.d;
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

// First-order steps with the auxiliary model's matrices formed once per call.
// Under order 1, Omega_t = delta/2 I whatever the path, so the forward and
// reverse auxiliary models of every step share P^p_t, S_t, P^f_t and the
// sampler's E_t and L_t.  Step 0 runs the full filter and sampler, keeping
// S_t^{-1}, log det S_t, E_t and chol(L_t), and forms the node products of two
// affine scans (the filtering means in reversed time with Phi_t =
// Omega S_t^{-1} F, the sampled path with E_t).  Every proposal after that is
// matrix-vector work: the means and log-likelihood terms in one kept scan,
// the path in another.  Set-up failures go to a third status word that each
// proposal folds into its step's own.
struct KeptTree {
  double* Tm[kMaxLevels + 1];
  double* Uagg[kMaxLevels + 1];
  double* xin[kMaxLevels + 1];
};

KeptTree kept_tree(const Layout& Lo, void* ws, const size_t* tm) {
  KeptTree K{};
  for (int l = 0; l <= Lo.L; ++l) {
    K.Tm[l] = at<double>(ws, tm[l]);
    K.Uagg[l] = at<double>(ws, Lo.vagg[l]);
    K.xin[l] = at<double>(ws, Lo.xin[l]);
  }
  return K;
}

// Kept-matrix state of a run: the workspace pointers of the kept matrices and
// trees.
struct Kept {
  FixedArgs X;
  KeptTree phi, e;
  double *Pf;
  double *Sinv, *ldS, *Et, *Lc;  // written by the plain forward pass that keeps them
};

Kept kept_state(const Layout& Lo, void* ws, const StepArgs& A, const double* xi_x,
                int* setup_status) {
  Kept K{};
  K.X.B = Lo.B;
  K.X.Sinv = at<double>(ws, Lo.Sinv);
  K.X.ldS = at<double>(ws, Lo.ldS);
  K.X.Et = at<double>(ws, Lo.Et);
  K.X.Lc = at<double>(ws, Lo.Lc);
  K.X.Phi = at<double>(ws, Lo.Phi);
  K.X.Fp = at<double>(ws, Lo.Fp);
  K.X.mf = at<double>(ws, Lo.mf);
  K.X.W = at<double>(ws, Lo.U);
  K.X.G = at<double>(ws, Lo.Gs);
  K.X.xs = A.xs;
  K.X.xi_x = xi_x;
  K.X.setup_status = setup_status;
  K.X.status = A.status;
  K.phi = kept_tree(Lo, ws, Lo.tphi);
  K.e = kept_tree(Lo, ws, Lo.te);
  K.Pf = at<double>(ws, Lo.Pf);
  K.Sinv = at<double>(ws, Lo.Sinv);
  K.ldS = at<double>(ws, Lo.ldS);
  K.Et = at<double>(ws, Lo.Et);
  K.Lc = at<double>(ws, Lo.Lc);
  return K;
}

// The plain forward filter and sampler at omega/Omega, keeping S^{-1}, log det
// S, E and chol(L); failures go to `status`.
akf_status forward_keep(const Layout& Lo, const KModel& M, void* ws, const StepArgs& A,
                        const Kept& K, int* status, hipStream_t st) {
  akf_status s;
  const double* xi_x = K.X.xi_x;
  if ((s = run_filter(Lo, M, ws, A.om, A.Om, nullptr, K.X.mf, K.Pf, Lo.D, A.ell, status,
                      ST_FWD_NOT_PD, st, nullptr, nullptr, nullptr, 0, nullptr, nullptr, K.Sinv,
                      K.ldS)) != AKF_OK)
    return s;
  return run_sampler(Lo, M, ws, K.X.mf, K.Pf, Lo.D, xi_x, A.xs, status, st, nullptr, nullptr,
                     K.Lc, K.Et);
}

// Phi_t = Omega_t S_t^{-1} F and the node products of both kept scans.
akf_status form_trees(const Layout& Lo, const KModel& M, const Kept& K, const double* Om,
                      hipStream_t st) {
  akf_status s;
  FixedArgs X = K.X;
  X.Om = Om;
  if ((s = hip_check(launch_fixed_phi_any(Lo.D, M, X, st), "Phi launch")) != AKF_OK) return s;
  const VScanArgs Vphi{M.N, Lo.B, X.Phi, M.gate}, Ve{M.N, Lo.B, X.Et, M.gate};
  if ((s = hip_check(launch_vtree_mats_any(Lo.D, Vphi, K.phi.Tm, Lo.n_lvl, Lo.L, st),
                     "scan products launch")) != AKF_OK)
    return s;
  return hip_check(launch_vtree_mats_any(Lo.D, Ve, K.e.Tm, Lo.n_lvl, Lo.L, st),
                   "scan products launch");
}

// A proposal's means and log-likelihood terms (and with `path` its sampled
// path) from the kept matrices.
akf_status kept_proposal(const Layout& Lo, const KModel& M, const Kept& K, const double* om,
                         const double* Om, double* ell, bool path, hipStream_t st) {
  akf_status s;
  FixedArgs X = K.X;
  X.om = om;
  X.Om = Om;
  X.ell = ell;
  if ((s = hip_check(launch_fixed_scan_any(Lo.D, 0, M, X, K.phi.Tm, K.phi.Uagg, K.phi.xin,
                                           Lo.n_lvl, Lo.L, st),
                     "mean scan launch")) != AKF_OK)
    return s;
  if (!path) return AKF_OK;
  return hip_check(launch_fixed_scan_any(Lo.D, 1, M, X, K.e.Tm, K.e.Uagg, K.e.xin, Lo.n_lvl, Lo.L,
                                         st),
                   "sampler scan launch");
}

akf_status kept_finalize(const Layout& Lo, const KModel& M, void* ws, const StepArgs& A,
                         int step, const double* lz_rev, int n_part_fwd, int n_part_rev,
                         const double* x_in, double* x_out, const double* unif,
                         double* log_ratio, int32_t* accepted, double* logZ_fwd,
                         double* logZ_rev, int32_t* status_out, hipStream_t st) {
  FinalArgs F{};
  F.status_next = at<int>(ws, Lo.status) + ((step + 1) & 1);
  F.lz_rev = lz_rev;
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

// the reuse gate (see k_reuse_gate), zero (a fresh pass) at the first step
int* reuse_gate_word(const Layout& Lo, void* ws) { return at<int>(ws, Lo.status) + 4; }

akf_status init_kept_status(const Layout& Lo, void* ws, hipStream_t st) {
  akf_status s;
  if ((s = hip_check(launch_step_init(at<int>(ws, Lo.status), root_flag(Lo, ws),
                                      at<double>(ws, Lo.xin[Lo.L]), Lo.D, st),
                     "init launch")) != AKF_OK)
    return s;
  if ((s = hip_check(launch_step_init(at<int>(ws, Lo.status) + 2, nullptr, nullptr, 0, st),
                     "init launch")) != AKF_OK)
    return s;
  return hip_check(launch_step_init(reuse_gate_word(Lo, ws), nullptr, nullptr, 0, st),
                   "init launch");
}

// First order: step 0 is the plain step keeping its matrices (then the trees);
// every later proposal, forward and reverse, uses them.
akf_status fixed_step_impl(const Layout& Lo, const KModel& M, const double* y, const double* x_in,
                           double delta, const double* xi, const double* unif, double* x_out,
                           double* log_ratio, int32_t* accepted, double* logZ_fwd,
                           double* logZ_rev, int32_t* status_out, void* ws, hipStream_t st,
                           int step) {
  const size_t vn = (size_t)M.N * M.d;
  const StepArgs A = make_step_args(Lo, ws, y, x_in, delta, 1, xi, step);
  int* setup_status = at<int>(ws, Lo.status) + 2;
  akf_status s;
  if (step == 0 && (s = init_kept_status(Lo, ws, st)) != AKF_OK) return s;
  int n_part_fwd = 0, n_part_rev = 0;
  if ((s = hip_check(launch_lin(M, A, 0, &n_part_fwd, st), "linearise launch")) != AKF_OK) return s;
  const Kept K = kept_state(Lo, ws, A, xi + vn, setup_status);
  if (step == 0) {
    if ((s = forward_keep(Lo, M, ws, A, K, setup_status, st)) != AKF_OK) return s;
    if ((s = form_trees(Lo, M, K, A.Om, st)) != AKF_OK) return s;
  } else if ((s = kept_proposal(Lo, M, K, A.om, A.Om, A.ell, true, st)) != AKF_OK) {
    return s;
  }
  if ((s = hip_check(launch_lin(M, A, 1, &n_part_rev, st), "linearise launch")) != AKF_OK) return s;
  if ((s = kept_proposal(Lo, M, K, A.om2, A.Om2, A.ell2, false, st)) != AKF_OK) return s;
  return kept_finalize(Lo, M, ws, A, step, nullptr, n_part_fwd, n_part_rev, x_in, x_out, unif,
                       log_ratio, accepted, logZ_fwd, logZ_rev, status_out, st);
}

// Second order: Omega_t depends on x only, so after a rejected step the next
// forward proposal (same x, new u) has the covariances of the one before.
// `fresh`: x changed since the kept matrices were formed (step 0, or the step
// before accepted or failed); `trees`: the kept scans' products are current.
// The reverse proposal is at a new x* every step and runs in full.
// Order 2 with matrix reuse: the forward proposal keeps the plain pass's
// matrices, and after a rejection (x unchanged) the next forward proposal is
// formed from them.  The branch is decided on the device: every launch of the
// three branches is issued each step and gated on the reuse word, so a run
// needs no host synchronisation and can be captured in a graph.
akf_status reuse_step_impl(const Layout& Lo, const KModel& M, const double* y, const double* x_in,
                           double delta, const double* xi, const double* unif, double* x_out,
                           double* log_ratio, int32_t* accepted, double* logZ_fwd,
                           double* logZ_rev, int32_t* status_out, void* ws, hipStream_t st,
                           int step) {
  const size_t vn = (size_t)M.N * M.d;
  const StepArgs A = make_step_args(Lo, ws, y, x_in, delta, 2, xi, step);
  akf_status s;
  if (step == 0 && (s = init_kept_status(Lo, ws, st)) != AKF_OK) return s;
  int n_part_fwd = 0, n_part_rev = 0;
  if ((s = hip_check(launch_lin(M, A, 0, &n_part_fwd, st), "linearise launch")) != AKF_OK) return s;
  // set-up failures of a kept forward pass are this step's own failures
  const Kept K = kept_state(Lo, ws, A, xi + vn, A.status);
  int* gate = reuse_gate_word(Lo, ws);
  KModel Mfresh = M, Mtrees = M, Mkept = M;
  Mfresh.gate = Gate{gate, 0, 0};
  Mtrees.gate = Gate{gate, 1, 1};
  Mkept.gate = Gate{gate, 1, 2};
  if ((s = forward_keep(Lo, Mfresh, ws, A, K, A.status, st)) != AKF_OK) return s;
  if ((s = form_trees(Lo, Mtrees, K, A.Om, st)) != AKF_OK) return s;
  if ((s = kept_proposal(Lo, Mkept, K, A.om, A.Om, A.ell, true, st)) != AKF_OK) return s;
  if ((s = hip_check(launch_lin(M, A, 1, &n_part_rev, st), "linearise launch")) != AKF_OK) return s;
  const double* lz_rev = nullptr;
  if ((s = run_filter_logz(Lo, M, ws, A.om2, A.Om2, nullptr, A.status, ST_REV_NOT_PD, st, nullptr,
                           nullptr, &lz_rev)) != AKF_OK)
    return s;
  if ((s = kept_finalize(Lo, M, ws, A, step, lz_rev, n_part_fwd, n_part_rev, x_in, x_out, unif,
                         log_ratio, accepted, logZ_fwd, logZ_rev, status_out, st)) != AKF_OK)
    return s;
  // the next forward proposal reuses this one's matrices iff x is unchanged
  return hip_check(launch_reuse_gate(A.accept_flag, A.status, gate, st), "reuse gate launch");
}

akf_status check_fact_model(const akf_model* model, int order) {
  akf_status s;
  if ((s = check_model(model, true)) != AKF_OK) return s;
  if ((s = check_linear(model, "the factorised step")) != AKF_OK) return s;
  if ((s = check_order(model, order)) != AKF_OK) return s;
  if (order == 3)
    return fail(AKF_ERR_UNSUPPORTED, "the factorised step takes orders 1 and 2");
  if (model->emit == AKF_EMIT_GAUSSIAN)
    return fail(AKF_ERR_UNSUPPORTED, "the factorised step needs a site-based emission family "
                                     "(its Gaussian emission has a dense H)");
  return AKF_OK;
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
  // launches recorded into a graph are not timed (the events would become
  // graph nodes)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
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

size_t akf_smoother_workspace_bytes(const akf_model* model, int32_t block) {
  if (check_model(model, false) != AKF_OK || check_linear(model, "akf_smoother") != AKF_OK)
    return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, block, LAYOUT_SMOOTH);
  return Lo.total;
}

akf_status akf_smoother(const akf_model* model, const double* mf, const double* Pf, double* ms,
                        double* Ps, int32_t* status, void* ws, size_t ws_bytes, int32_t block,
                        void* stream) {
  akf_status s;
  if ((s = check_model(model, false)) != AKF_OK) return s;
  if ((s = check_linear(model, "akf_smoother")) != AKF_OK) return s;
  if (!mf || !Pf || !ms || !Ps) return fail(AKF_ERR_INVALID, "mf, Pf, ms and Ps must be non-NULL");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, block, LAYOUT_SMOOTH);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  int* dstat = at<int>(ws, Lo.status);
  if ((s = hip_check(launch_step_init(dstat, nullptr, nullptr, 0, st), "init launch")) != AKF_OK)
    return s;
  SmoothArgs S{};
  S.mf = mf;
  S.Pf = Pf;
  S.ldm = model->dx;
  S.E = at<double>(ws, Lo.E);
  S.g = at<double>(ws, Lo.g);
  S.L = at<double>(ws, Lo.Lm);
  S.status = dstat;
  if ((s = hip_check(launch_smooth_build_any(Lo.D, to_kmodel(model), S, st), "smoother build")) !=
      AKF_OK)
    return s;
  if ((s = run_egl(Lo, ws, S.g, Ps, ms, model->dx, model->dx, st)) != AKF_OK) return s;
  if (status)
    return hip_check(hipMemcpyAsync(status, dstat, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy");
  return AKF_OK;
}

namespace {
akf_status check_lgssm(const akf_lgssm* m) {
  if (!m) return fail(AKF_ERR_INVALID, "lgssm is NULL");
  if (m->N < 1) return fail(AKF_ERR_SHAPE, "N must be >= 1 (got %d)", m->N);
  if (m->dx < 1 || m->dx > 32)
    return fail(AKF_ERR_SHAPE, "dx must be in [1, 32] for the LGSSM likelihood (got %d)", m->dx);
  if (m->dy < 1 || m->dy > 32)
    return fail(AKF_ERR_SHAPE, "dy must be in [1, 32] for the LGSSM likelihood (got %d)", m->dy);
  if (!m->m0 || !m->P0 || !m->F || !m->logq || !m->H || !m->logr || !m->y)
    return fail(AKF_ERR_INVALID, "every LGSSM array must be non-NULL");
  return AKF_OK;
}

int lgssm_D(const akf_lgssm* m) {
  const int d = m->dx > m->dy ? m->dx : m->dy;
  return d <= 16 ? 16 : 32;
}

KModel lgssm_kmodel(const akf_lgssm* m, void* ws, const Layout& Lo) {
  KModel M{};
  M.N = m->N;
  M.d = m->dx;
  M.dy = m->dy;
  M.emit = EMIT_GAUSSIAN;
  M.m0 = m->m0;
  M.P0 = m->P0;
  M.F = m->F;
  M.b = nullptr;
  M.Q = at<double>(ws, Lo.Qd);
  M.H = m->H;
  M.R = at<double>(ws, Lo.Rd);
  return M;
}

LgArgs lgssm_args(const akf_lgssm* m, void* ws, const Layout& Lo) {
  LgArgs G{};
  G.dx = m->dx;
  G.dy = m->dy;
  G.B = Lo.B;
  G.logq = m->logq;
  G.logr = m->logr;
  G.H = m->H;
  G.y = m->y;
  G.Q = at<double>(ws, Lo.Qd);
  G.R = at<double>(ws, Lo.Rd);
  G.mf = at<double>(ws, Lo.mf);
  G.Pf = at<double>(ws, Lo.Pf);
  G.E = at<double>(ws, Lo.E);
  G.U = at<double>(ws, Lo.U);
  G.Cm = at<double>(ws, Lo.Lm);
  G.mbar = at<double>(ws, Lo.mbar);
  G.Pbar = at<double>(ws, Lo.Pbar);
  G.part = at<double>(ws, Lo.part);
  G.status = at<int>(ws, Lo.status);
  return G;
}
}  // namespace

size_t akf_lgssm_workspace_bytes(const akf_lgssm* m, int32_t block) {
  if (check_lgssm(m) != AKF_OK || block < 0) return 0;
  Layout Lo;
  lgssm_layout(Lo, m, block);
  return Lo.total;
}

akf_status akf_lgssm_loglik(const akf_lgssm* m, double* ll, double* ell, int32_t* status, void* ws,
                            size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_lgssm(m)) != AKF_OK) return s;
  if (!ll) return fail(AKF_ERR_INVALID, "ll must be non-NULL");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  lgssm_layout(Lo, m, block);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  int* dstat = at<int>(ws, Lo.status);
  if ((s = hip_check(launch_step_init(dstat, root_flag(Lo, ws), nullptr, 0, st), "init launch")) !=
      AKF_OK)
    return s;
  LgArgs G = lgssm_args(m, ws, Lo);
  if ((s = hip_check(launch_lgssm_prep(G, st), "parameter launch")) != AKF_OK) return s;
  const KModel M = lgssm_kmodel(m, ws, Lo);
  double* ellw = ell ? ell : at<double>(ws, Lo.ell);
  if ((s = run_filter(Lo, M, ws, nullptr, nullptr, nullptr, at<double>(ws, Lo.mf),
                      at<double>(ws, Lo.Pf), Lo.D, ellw, dstat, ST_FWD_NOT_PD, st, m->y, m->H,
                      G.R, m->dy)) != AKF_OK)
    return s;
  if ((s = hip_check(launch_sum(ellw, m->N, ll, dstat, st), "sum launch")) != AKF_OK) return s;
  if (status)
    return hip_check(hipMemcpyAsync(status, dstat, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy");
  return AKF_OK;
}

akf_status akf_lgssm_loglik_grad(const akf_lgssm* m, const double* ll_bar, double* dF,
                                 double* dlogq, double* dH, double* dlogr, int32_t* status,
                                 void* ws, size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_lgssm(m)) != AKF_OK) return s;
  if (!dF || !dlogq || !dH || !dlogr)
    return fail(AKF_ERR_INVALID, "dF, dlogq, dH and dlogr must be non-NULL");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  lgssm_layout(Lo, m, block);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  const int D = Lo.D;
  LgArgs G = lgssm_args(m, ws, Lo);
  G.dF = dF;
  G.dlogq = dlogq;
  G.dH = dH;
  G.dlogr = dlogr;
  KModel M = lgssm_kmodel(m, ws, Lo);
  // adjoint elements: E = Phi', U = H'w, Cm = -1/2 H' Sig H.  The status word
  // keeps the forward pass's bits (the adjoint adds its own), so a failed
  // forward pass also leaves NaN gradients.
  if ((s = hip_check(launch_step_init(nullptr, nullptr, at<double>(ws, Lo.xin[Lo.L]), D, st),
                     "init launch")) != AKF_OK)
    return s;
  if ((s = hip_check(launch_adj_build_any(D, M, G, st), "adjoint build")) != AKF_OK) return s;
  // mbar: path scan with (E, U) (output stride D)
  SampArgs S{};
  S.B = Lo.B;
  S.E = G.E;
  S.U = G.U;
  S.agg = at<double>(ws, Lo.sagg[0]);
  S.xin = at<double>(ws, Lo.xin[0]);
  S.xs = G.mbar;
  S.status = G.status;
  TreeArgs up[kMaxLevels], down[kMaxLevels];
  fill_tree(Lo, ws, 0, Lo.sagg, Lo.xin, G.status, ST_FWD_NOT_PD, up, down);
  KModel Mv = M;
  Mv.d = D;
  if ((s = hip_check(launch_samp_scan_any(D, Mv, S, up, down, Lo.L, st), "mbar scan")) != AKF_OK)
    return s;
  // G_t in place of Cm, then Pbar: (E, L) scan
  if ((s = hip_check(launch_adj_G_any(D, G, m->N, st), "adjoint G")) != AKF_OK) return s;
  if ((s = run_egl(Lo, ws, nullptr, G.Pbar, nullptr, D, D, st)) != AKF_OK) return s;
  // Gradient blocks: at width 32 a one-wave team of k_adj_grad fits three to a
  // CU, so blocks of at least Lo.B steps are made long enough that all of them
  // run at once (there are then no more of them than the layout's partial
  // sums hold)
  int nblk = Lo.nb;
  if (D == 32) {
    int dev = 0, ncu = 0;
    if ((s = hip_check(hipGetDevice(&dev), "device query")) != AKF_OK) return s;
    if ((s = hip_check(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev),
                       "CU count query")) != AKF_OK)
      return s;
    const int slots = 3 * (ncu > 0 ? ncu : 1);
    const int Bg = std::max(Lo.B, (m->N + slots - 1) / slots);
    G.B = Bg;
    nblk = (m->N + Bg - 1) / Bg;
  }
  if ((s = hip_check(launch_adj_finish_any(D, M, G, nblk, ll_bar, st), "adjoint gradient")) !=
      AKF_OK)
    return s;
  if (status)
    return hip_check(hipMemcpyAsync(status, G.status, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy");
  return AKF_OK;
}

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

const char* akf_last_error(void) { return akf::last_error(); }

size_t akf_mh_workspace_bytes(const akf_model* model, int32_t order, int32_t block) {
  if (check_model(model, true) != AKF_OK || check_order(model, order) != AKF_OK) return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP, model->dyn != 0);
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
  if ((s = check_order(model, order)) != AKF_OK) return s;
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP, model->dyn != 0);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  const KModel M = to_kmodel(model);
  if (M.dyn != DYN_LINEAR &&
      (s = hip_check(launch_qinv(M, at<double>(ws, Lo.Qinv), (hipStream_t)stream), "Q^-1 launch")) !=
          AKF_OK)
    return s;
  return mh_step_impl(Lo, M, y, x_in, delta, order, xi, unif, x_out, log_ratio, accepted, logZ_fwd,
                      logZ_rev, status, ws, (hipStream_t)stream, 0);
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
  if ((s = check_order(model, order)) != AKF_OK) return s;
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP, model->dyn != 0);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  const KModel M = to_kmodel(model);
  const size_t vn = (size_t)M.N * M.d;
  if (M.dyn != DYN_LINEAR && n_steps > 0 &&
      (s = hip_check(launch_qinv(M, at<double>(ws, Lo.Qinv), (hipStream_t)stream), "Q^-1 launch")) !=
          AKF_OK)
    return s;
  for (int k = 0; k < n_steps; ++k) {
    s = mh_step_impl(Lo, M, y, x, delta, order, xi + (size_t)k * 2 * vn, unif + k, x,
                     log_ratio ? log_ratio + k : nullptr, accepted ? accepted + k : nullptr,
                     logZ_fwd ? logZ_fwd + k : nullptr, logZ_rev ? logZ_rev + k : nullptr,
                     status ? status + k : nullptr, ws, (hipStream_t)stream, k);
    if (s != AKF_OK) return s;
  }
  return AKF_OK;
}

size_t akf_mh_factorised_workspace_bytes(const akf_model* model, int32_t order) {
  if (check_fact_model(model, order) != AKF_OK) return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, 0, LAYOUT_FACT);
  return Lo.total;
}

akf_status akf_mh_step_factorised(const akf_model* model, const double* y, const double* x_in,
                                  double delta, int32_t order, const double* xi,
                                  const double* unif, double* x_out, double* log_ratio,
                                  int32_t* accepted, double* logZ_fwd, double* logZ_rev,
                                  int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  akf_status s;
  if ((s = check_fact_model(model, order)) != AKF_OK) return s;
  if (!y || !x_in || !xi || !unif || !x_out)
    return fail(AKF_ERR_INVALID, "y, x_in, xi, unif and x_out must be non-NULL");
  if (!(delta > 0.0)) return fail(AKF_ERR_INVALID, "delta must be > 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, 0, LAYOUT_FACT);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  return fact_step_impl(Lo, to_kmodel(model), y, x_in, delta, order, xi, unif, x_out, log_ratio,
                        accepted, logZ_fwd, logZ_rev, status, ws, (hipStream_t)stream, 0);
}

akf_status akf_mh_run_factorised(const akf_model* model, const double* y, double* x, double delta,
                                 int32_t order, int32_t n_steps, const double* xi,
                                 const double* unif, double* log_ratio, int32_t* accepted,
                                 double* logZ_fwd, double* logZ_rev, int32_t* status, void* ws,
                                 size_t ws_bytes, void* stream) {
  akf_status s;
  if ((s = check_fact_model(model, order)) != AKF_OK) return s;
  if (!y || !x || !xi || !unif) return fail(AKF_ERR_INVALID, "y, x, xi and unif must be non-NULL");
  if (n_steps < 0) return fail(AKF_ERR_INVALID, "n_steps must be >= 0");
  if (!(delta > 0.0)) return fail(AKF_ERR_INVALID, "delta must be > 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, 0, LAYOUT_FACT);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  const KModel M = to_kmodel(model);
  const size_t vn = (size_t)M.N * M.d;
  for (int k = 0; k < n_steps; ++k) {
    s = fact_step_impl(Lo, M, y, x, delta, order, xi + (size_t)k * 2 * vn, unif + k, x,
                       log_ratio ? log_ratio + k : nullptr, accepted ? accepted + k : nullptr,
                       logZ_fwd ? logZ_fwd + k : nullptr, logZ_rev ? logZ_rev + k : nullptr,
                       status ? status + k : nullptr, ws, (hipStream_t)stream, k);
    if (s != AKF_OK) return s;
  }
  return AKF_OK;
}

size_t akf_mh_first_order_workspace_bytes(const akf_model* model, int32_t block) {
  if (check_model(model, true) != AKF_OK || check_order(model, 1) != AKF_OK ||
      check_linear(model, "akf_mh_run_first_order") != AKF_OK || block < 0)
    return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP, false, true);
  return Lo.total;
}

akf_status akf_mh_run_first_order(const akf_model* model, const double* y, double* x,
                                  double delta, int32_t n_steps, const double* xi,
                                  const double* unif, double* log_ratio, int32_t* accepted,
                                  double* logZ_fwd, double* logZ_rev, int32_t* status, void* ws,
                                  size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_model(model, true)) != AKF_OK) return s;
  if ((s = check_linear(model, "akf_mh_run_first_order")) != AKF_OK) return s;
  if ((s = check_order(model, 1)) != AKF_OK) return s;
  if (!y || !x || !xi || !unif) return fail(AKF_ERR_INVALID, "y, x, xi and unif must be non-NULL");
  if (n_steps < 0) return fail(AKF_ERR_INVALID, "n_steps must be >= 0");
  if (!(delta > 0.0)) return fail(AKF_ERR_INVALID, "delta must be > 0");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP, false, true);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  const KModel M = to_kmodel(model);
  const size_t vn = (size_t)M.N * M.d;
  for (int k = 0; k < n_steps; ++k) {
    s = fixed_step_impl(Lo, M, y, x, delta, xi + (size_t)k * 2 * vn, unif + k, x,
                        log_ratio ? log_ratio + k : nullptr, accepted ? accepted + k : nullptr,
                        logZ_fwd ? logZ_fwd + k : nullptr, logZ_rev ? logZ_rev + k : nullptr,
                        status ? status + k : nullptr, ws, (hipStream_t)stream, k);
    if (s != AKF_OK) return s;
  }
  return AKF_OK;
}

akf_status check_reuse_model(const akf_model* model, int order) {
  akf_status s;
  if ((s = check_model(model, true)) != AKF_OK) return s;
  if ((s = check_linear(model, "akf_mh_run_reuse")) != AKF_OK) return s;
  if ((s = check_order(model, order)) != AKF_OK) return s;
  if (order == 3) return fail(AKF_ERR_UNSUPPORTED, "akf_mh_run_reuse takes orders 1 and 2");
  if (order == 2 && model->emit == AKF_EMIT_GAUSSIAN)
    return fail(AKF_ERR_UNSUPPORTED, "akf_mh_run_reuse keeps diagonal-Omega matrices; the "
                                     "GAUSSIAN emission has a dense Omega under order 2");
  return AKF_OK;
}

size_t akf_mh_reuse_workspace_bytes(const akf_model* model, int32_t order, int32_t block) {
  if (check_reuse_model(model, order) != AKF_OK || block < 0) return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP, false, true);
  return Lo.total;
}

akf_status akf_mh_run_reuse(const akf_model* model, const double* y, double* x, double delta,
                            int32_t order, int32_t n_steps, const double* xi, const double* unif,
                            double* log_ratio, int32_t* accepted, double* logZ_fwd,
                            double* logZ_rev, int32_t* status, void* ws, size_t ws_bytes,
                            int32_t block, void* stream) {
  akf_status s;
  if ((s = check_reuse_model(model, order)) != AKF_OK) return s;
  if (!y || !x || !xi || !unif) return fail(AKF_ERR_INVALID, "y, x, xi and unif must be non-NULL");
  if (n_steps < 0) return fail(AKF_ERR_INVALID, "n_steps must be >= 0");
  if (!(delta > 0.0)) return fail(AKF_ERR_INVALID, "delta must be > 0");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, model->dy, block, LAYOUT_STEP, false, true);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  if ((s = prepare_device()) != AKF_OK) return s;
  const KModel M = to_kmodel(model);
  const size_t vn = (size_t)M.N * M.d;
  hipStream_t st = (hipStream_t)stream;
  for (int k = 0; k < n_steps; ++k) {
    double* lr = log_ratio ? log_ratio + k : nullptr;
    int32_t* acc = accepted ? accepted + k : nullptr;
    double* zf = logZ_fwd ? logZ_fwd + k : nullptr;
    double* zr = logZ_rev ? logZ_rev + k : nullptr;
    int32_t* so = status ? status + k : nullptr;
    const double* xik = xi + (size_t)k * 2 * vn;
    if (order == 1)
      s = fixed_step_impl(Lo, M, y, x, delta, xik, unif + k, x, lr, acc, zf, zr, so, ws, st, k);
    else
      s = reuse_step_impl(Lo, M, y, x, delta, xik, unif + k, x, lr, acc, zf, zr, so, ws, st, k);
    if (s != AKF_OK) return s;
  }
  return AKF_OK;
}

size_t akf_dnc_workspace_bytes(const akf_model* model) {
  if (check_model(model, false) != AKF_OK || check_linear(model, "akf_dnc_sample") != AKF_OK)
    return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, 0, LAYOUT_DNC);
  return Lo.total;
}

akf_status akf_dnc_sample(const akf_model* model, const double* mf, const double* Pf,
                          const double* xi, double* x, int32_t* status, void* ws,
                          size_t ws_bytes, void* stream) {
  akf_status s;
  if ((s = check_model(model, false)) != AKF_OK) return s;
  if ((s = check_linear(model, "akf_dnc_sample")) != AKF_OK) return s;
  if (!mf || !Pf || !xi || !x) return fail(AKF_ERR_INVALID, "mf, Pf, xi and x must be non-NULL");
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, 0, LAYOUT_DNC);
  if ((s = check_ws(Lo, ws, ws_bytes)) != AKF_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  int* dstat = at<int>(ws, Lo.status);
  if ((s = hip_check(launch_step_init(dstat, nullptr, nullptr, 0, st), "init launch")) != AKF_OK)
    return s;
  DncArgs A{};
  A.T = model->N - 1;
  A.mf = mf;
  A.Pf = Pf;
  A.ldm = model->dx;
  A.xi = xi;
  A.x = x;
  A.Elf = at<double>(ws, Lo.Elf);
  A.glf = at<double>(ws, Lo.glf);
  A.Llf = at<double>(ws, Lo.Llf);
  A.Eno = at<double>(ws, Lo.Eno);
  A.gno = at<double>(ws, Lo.gno);
  A.Lno = at<double>(ws, Lo.Lno);
  A.Gb = at<double>(ws, Lo.Gb);
  A.Gam = at<double>(ws, Lo.Gam);
  A.wb = at<double>(ws, Lo.wb);
  A.Vc = at<double>(ws, Lo.Vc);
  A.status = dstat;
  if ((s = hip_check(launch_dnc_any(Lo.D, to_kmodel(model), A, st), "divide-and-conquer launch")) !=
      AKF_OK)
    return s;
  if (status)
    return hip_check(hipMemcpyAsync(status, dstat, sizeof(int), hipMemcpyDeviceToDevice, st),
                     "status copy");
  return AKF_OK;
}

size_t akf_filter_workspace_bytes(const akf_model* model, int32_t block) {
  if (check_model(model, false) != AKF_OK || check_linear(model, "akf_aux_filter") != AKF_OK)
    return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, block, LAYOUT_FILTER);
  return Lo.total;
}

akf_status akf_aux_filter(const akf_model* model, const double* omega, const double* Omega,
                          double* mf, double* Pf, double* ell, int32_t* status, void* ws,
                          size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_model(model, false)) != AKF_OK) return s;
  if ((s = check_linear(model, "akf_aux_filter")) != AKF_OK) return s;
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
  if (check_model(model, false) != AKF_OK || check_linear(model, "akf_rts_sample") != AKF_OK)
    return 0;
  Layout Lo;
  make_layout(Lo, model->N, model->dx, 0, block, LAYOUT_SAMPLER);
  return Lo.total;
}

akf_status akf_rts_sample(const akf_model* model, const double* mf, const double* Pf,
                          const double* xi, double* x, int32_t* status, void* ws,
                          size_t ws_bytes, int32_t block, void* stream) {
  akf_status s;
  if ((s = check_model(model, false)) != AKF_OK) return s;
  if ((s = check_linear(model, "akf_rts_sample")) != AKF_OK) return s;
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
