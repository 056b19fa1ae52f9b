// akf_layout.cpp -- host-side helpers shared by the C ABI translation units
// (see akf_layout.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "akf_layout.h"

namespace akf {


thread_local char g_err[512] = "";

akf_status fail(akf_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int pick_D(int d) { return d <= 16 ? 16 : (d <= 32 ? 32 : (d <= 64 ? 64 : 0)); }

// Default scan block: enough blocks to give every CU (256) its resident teams
// and no more, so that the fold runs in one round (LDS-limited: 1 team of 4
// waves at D = 64; at D = 32 four single-wave teams, three with a general
// observation matrix, whose fold holds a fifth matrix; eight at D = 16), and at
// least 4 steps per block so that small problems do not pay for a deep tree of
// tiny launches.
int auto_block(int N, int D, bool general_obs) {
  const int teams_per_cu = D == 64 ? 1 : (D == 32 ? (general_obs ? 3 : 4) : 8);
  const int target = 256 * teams_per_cu;
  int B = (N + target - 1) / target;
  if (B < 4) B = 4;
  if (B > N) B = N;
  return B;
}

void make_layout(Layout& Lo, int N, int d, int dy, int block, int kind, bool dyn, bool fixed) {
  Lo.N = N;
  Lo.d = d;
  Lo.dy = dy;
  Lo.D = pick_D(d);
  const int D = Lo.D;
  Lo.B = block > 0 ? (block > N ? N : block) : auto_block(N, D, kind == LAYOUT_LGSSM);
  Lo.nb = (N + Lo.B - 1) / Lo.B;
  Lo.n_lvl[0] = Lo.nb;
  Lo.L_hs = 0;
  while ((1 << Lo.L_hs) < Lo.nb) ++Lo.L_hs;
  Lo.L = 0;
  while (Lo.n_lvl[Lo.L] > 1 && Lo.L < kMaxLevels) {
    Lo.n_lvl[Lo.L + 1] = (Lo.n_lvl[Lo.L] + 1) / 2;
    ++Lo.L;
  }
  const size_t dbl = sizeof(double);
  const size_t vn = (size_t)N * d * dbl;
  const size_t ES = (size_t)(3 * D * D + 2 * D + 2) * dbl;  // ElemLayout<D>::SIZE
  const size_t PS = (size_t)(D * D + D + 2) * dbl;
  const size_t SS = (size_t)(D * D + D) * dbl;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes == 0 ? 1 : bytes);
    return o;
  };
  const int nparts_diag = (int)(((int64_t)N * d + 255) / 256);
  const int nparts_gauss = (N + kGaussStepsPerBlock - 1) / kGaussStepsPerBlock;
  const int nparts_mvt = (N + kMvtWaves - 1) / kMvtWaves;
  Lo.n_part = nparts_diag > nparts_gauss ? nparts_diag : nparts_gauss;
  if (nparts_mvt > Lo.n_part) Lo.n_part = nparts_mvt;
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
    Lo.gHt = take((size_t)d * (dy > 0 ? dy : 1) * dbl);
    Lo.gRinv = take((size_t)(dy > 0 ? dy * dy : 1) * dbl);
    Lo.gOmd = take((size_t)d * d * dbl);
    Lo.gOmdinv = take((size_t)d * d * dbl);
    Lo.gscal = take(8 * dbl);
    Lo.accept = take(sizeof(int));
    if (dyn) {
      Lo.Ft = take((size_t)N * d * d * dbl);
      Lo.bt = take(vn);
      Lo.Qinv = take((size_t)d * d * dbl);
      Lo.n_part_dyn = (N + 3) / 4;
      Lo.pdyn = take((size_t)Lo.n_part_dyn * dbl);
    }
    if (fixed) {
      const size_t mat = (size_t)D * D * dbl;
      Lo.Sinv = take((size_t)N * mat);
      Lo.ldS = take((size_t)N * dbl);
      Lo.Phi = take((size_t)N * mat);
      Lo.Lc = take((size_t)N * mat);
      Lo.Et = take((size_t)N * mat);
      Lo.Fp = take(mat);
      Lo.Gs = take((size_t)N * D * dbl);
      for (int l = 0; l <= Lo.L; ++l) {
        Lo.tphi[l] = take((size_t)Lo.n_lvl[l] * mat);
        Lo.te[l] = take((size_t)Lo.n_lvl[l] * mat);
        Lo.vagg[l] = take((size_t)Lo.n_lvl[l] * D * dbl);
      }
    }
  }
  if (kind == LAYOUT_FACT) {
    // the scan keeps no elements: only vectors [N*d] and per-coordinate sums
    Lo.u = take(vn);
    Lo.om = take(vn);
    Lo.Om = take(vn);
    Lo.om2 = take(vn);
    Lo.Om2 = take(vn);
    Lo.xs = take(vn);
    Lo.mf = take(vn);
    Lo.Pf = take(vn);
    Lo.ell = take((size_t)d * dbl);
    Lo.ell2 = take((size_t)d * dbl);
    Lo.plhx = take((size_t)Lo.n_part * dbl);
    Lo.plhxs = take((size_t)Lo.n_part * dbl);
    Lo.pterms = take((size_t)Lo.n_part * dbl);
    Lo.accept = take(sizeof(int));
    Lo.status = take(2 * sizeof(int));  // two words: consecutive steps alternate
    Lo.total = off;
    return;
  }
  if (kind == LAYOUT_DNC) {
    const size_t mat = (size_t)N * D * D * dbl, vec = (size_t)N * D * dbl;
    Lo.Elf = take(mat);
    Lo.glf = take(vec);
    Lo.Llf = take(mat);
    Lo.Eno = take(mat);
    Lo.gno = take(vec);
    Lo.Lno = take(mat);
    Lo.Gb = take(mat);
    Lo.Gam = take(mat);
    Lo.wb = take(vec);
    Lo.Vc = take(mat);
    Lo.status = take(2 * sizeof(int));  // two words: consecutive steps alternate
    Lo.total = off;
    return;
  }
  if (kind == LAYOUT_LGSSM) {
    Lo.Qd = take((size_t)d * d * dbl);
    Lo.Rd = take((size_t)dy * dy * dbl);
    Lo.llv = take(8 * dbl);
  }
  if (kind == LAYOUT_STEP || kind == LAYOUT_FILTER || kind == LAYOUT_LGSSM) {
    Lo.ell = take((size_t)N * dbl);
    for (int l = 0; l <= Lo.L; ++l) Lo.elem[l] = take((size_t)Lo.n_lvl[l] * ES);
    Lo.hs = take((size_t)Lo.nb * ES);
    for (int l = 0; l <= Lo.L; ++l) Lo.pre[l] = take((size_t)Lo.n_lvl[l] * PS);
  }
  if (kind == LAYOUT_STEP || kind == LAYOUT_LGSSM) {
    Lo.mf = take((size_t)N * D * dbl);
    Lo.Pf = take((size_t)N * D * D * dbl);
  }
  if (kind == LAYOUT_STEP || kind == LAYOUT_SAMPLER || kind == LAYOUT_LGSSM ||
      kind == LAYOUT_SMOOTH) {
    Lo.E = take((size_t)N * D * D * dbl);
  }
  if (kind == LAYOUT_STEP || kind == LAYOUT_SAMPLER || kind == LAYOUT_LGSSM) {
    Lo.U = take((size_t)N * D * dbl);
    for (int l = 0; l <= Lo.L; ++l) Lo.sagg[l] = take((size_t)Lo.n_lvl[l] * SS);
    for (int l = 0; l <= Lo.L; ++l) Lo.xin[l] = take((size_t)Lo.n_lvl[l] * D * dbl);
  }
  if (kind == LAYOUT_SMOOTH || kind == LAYOUT_LGSSM) {
    const size_t EG = (size_t)(2 * D * D + D) * dbl;
    const size_t ESt = (size_t)(D * D + D) * dbl;
    Lo.Lm = take((size_t)N * D * D * dbl);
    for (int l = 0; l <= Lo.L; ++l) Lo.eagg[l] = take((size_t)Lo.n_lvl[l] * EG);
    for (int l = 0; l <= Lo.L; ++l) Lo.estate[l] = take((size_t)Lo.n_lvl[l] * ESt);
  }
  if (kind == LAYOUT_SMOOTH) Lo.g = take((size_t)N * D * dbl);
  if (kind == LAYOUT_LGSSM) {
    Lo.mbar = take((size_t)N * D * dbl);
    Lo.Pbar = take((size_t)N * D * D * dbl);
    Lo.part = take((size_t)Lo.nb * (2 * D * D + 2 * D) * dbl);
  }
  // two words: consecutive steps alternate; runs that keep matrices add two
  // for the set-up of the shared matrices and two for the reuse gate (the
  // branch of the next step, decided on the device)
  Lo.status = take((fixed ? 6 : 2) * sizeof(int));
  Lo.total = off;
}


akf_status check_model(const akf_model* m, bool need_emission, bool allow_f32) {
  if (!m) return fail(AKF_ERR_INVALID, "model is NULL");
  if (m->N < 1) return fail(AKF_ERR_SHAPE, "N must be >= 1 (got %d)", m->N);
  if (m->dx < 1 || m->dx > 64) return fail(AKF_ERR_SHAPE, "dx must be in [1, 64] (got %d)", m->dx);
  if (m->dtype == AKF_F32 && !allow_f32)
    return fail(AKF_ERR_UNSUPPORTED, "dtype AKF_F32 is built for the square-root filter and "
                                     "sampler only (akf_sqrt_filter_sample); this entry point "
                                     "computes in FP64");
  if (m->dtype != AKF_F64 && m->dtype != AKF_F32)
    return fail(AKF_ERR_INVALID, "unknown dtype %d", m->dtype);
  switch (m->dyn) {
    case AKF_DYN_LINEAR:
      if (!m->F) return fail(AKF_ERR_INVALID, "linear dynamics need F");
      break;
    case AKF_DYN_LORENZ63:
      if (m->dx != 3) return fail(AKF_ERR_SHAPE, "Lorenz-63 dynamics need dx = 3 (got %d)", m->dx);
      if (!(m->dyn_par[3] > 0.0)) return fail(AKF_ERR_INVALID, "Lorenz-63 needs dt = dyn_par[3] > 0");
      break;
    case AKF_DYN_LORENZ96:
      if (m->dx < 4) return fail(AKF_ERR_SHAPE, "Lorenz-96 dynamics need dx >= 4 (got %d)", m->dx);
      if (!(m->dyn_par[1] > 0.0)) return fail(AKF_ERR_INVALID, "Lorenz-96 needs dt = dyn_par[1] > 0");
      break;
    default:
      return fail(AKF_ERR_INVALID, "unknown dynamics family %d", m->dyn);
  }
  if (!m->m0 || !m->P0 || !m->Q) return fail(AKF_ERR_INVALID, "m0, P0 and Q must be non-NULL");
  if (!need_emission) return AKF_OK;
  if (m->dy < 1 || m->dy > 64) return fail(AKF_ERR_SHAPE, "dy must be in [1, 64] (got %d)", m->dy);
  switch (m->emit) {
    case AKF_EMIT_GAUSSIAN:
      if (!m->H || !m->R) return fail(AKF_ERR_INVALID, "Gaussian emission needs H and R");
      break;
    case AKF_EMIT_POISSON_LOG:
      if (!m->site) return fail(AKF_ERR_INVALID, "Poisson emission needs site");
      break;
    case AKF_EMIT_STOCH_VOL:
      if (!m->site) return fail(AKF_ERR_INVALID, "stochastic-volatility emission needs site");
      break;
    case AKF_EMIT_STUDENT_T:
      if (!m->site) return fail(AKF_ERR_INVALID, "Student-t emission needs site");
      if (!(m->nu > 0.0) || !(m->scale > 0.0))
        return fail(AKF_ERR_INVALID, "Student-t emission needs nu > 0 and scale > 0");
      break;
    case AKF_EMIT_GAUSS_SITE:
      if (!m->site) return fail(AKF_ERR_INVALID, "Gaussian-at-sites emission needs site");
      if (!(m->scale > 0.0)) return fail(AKF_ERR_INVALID, "Gaussian-at-sites emission needs scale > 0");
      break;
    case AKF_EMIT_GAUSS_QUAD:
      if (!m->site) return fail(AKF_ERR_INVALID, "quadratic-mean Gaussian emission needs site");
      if (!(m->scale > 0.0) || !isfinite(m->obs_beta))
        return fail(AKF_ERR_INVALID,
                    "quadratic-mean Gaussian emission needs scale > 0 and a finite obs_beta");
      break;
    case AKF_EMIT_MVT:
      if (!m->site || !m->R) return fail(AKF_ERR_INVALID, "multivariate-t emission needs site and R");
      if (!(m->nu > 0.0)) return fail(AKF_ERR_INVALID, "multivariate-t emission needs nu > 0");
      break;
    default:
      return fail(AKF_ERR_INVALID, "unknown emission family %d", m->emit);
  }
  return AKF_OK;
}

akf_status check_order(const akf_model* m, int order) {
  if (order < 1 || order > 3) return fail(AKF_ERR_INVALID, "order must be 1, 2 or 3");
  if (order == 3) {
    if (m->emit != AKF_EMIT_GAUSS_SITE && m->emit != AKF_EMIT_GAUSS_QUAD)
      return fail(AKF_ERR_UNSUPPORTED, "order 3 (the observation model's linearisation) needs a "
                                       "Gaussian-around-a-mean family: GAUSS_SITE or GAUSS_QUAD");
    if (!(m->slr_var >= 0.0) || !isfinite(m->slr_var))
      return fail(AKF_ERR_INVALID, "order 3 needs a finite reference variance slr_var >= 0");
  }
  if (order == 2 && m->emit == AKF_EMIT_MVT)
    return fail(AKF_ERR_UNSUPPORTED,
                "the multivariate-t emission supports first-order proposals only (its Hessian "
                "would make Omega_t dense and time-varying)");
  return AKF_OK;
}

akf_status check_linear(const akf_model* m, const char* what) {
  if (m->dyn != AKF_DYN_LINEAR)
    return fail(AKF_ERR_UNSUPPORTED, "%s needs linear dynamics (nonlinear dynamics are "
                                     "accepted by akf_mh_step and akf_mh_run only)", what);
  return AKF_OK;
}

KModel to_kmodel(const akf_model* m) {
  KModel M{};
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
  M.dyn = m->dyn;
  for (int i = 0; i < 4; ++i) M.dyn_par[i] = m->dyn_par[i];
  M.obs_beta = m->obs_beta;
  M.slr_var = m->slr_var;
  return M;
}

void lgssm_layout(Layout& Lo, const akf_lgssm* m, int block) {
  // team size follows max(dx, dy): the observation block is padded to the same D
  make_layout(Lo, m->N, m->dx > m->dy ? m->dx : m->dy, m->dy, block, LAYOUT_LGSSM);
  Lo.d = m->dx;
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
                      double* ell, int* status, int fail_bit, hipStream_t st,
                      const double* yo, const double* Ho, const double* Ro, int dyo,
                      const double* Ft, const double* bt, double* Sinv, double* ldS) {
  FilterArgs P{};
  P.Ft = Ft;
  P.bt = bt;
  P.Sinv = Sinv;
  P.ldS = ldS;
  P.yo = yo;
  P.Ho = Ho;
  P.Ro = Ro;
  P.dyo = dyo;
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
  // one chain: Hillis-Steele scan over the block elements (every level keeps
  // up to nb teams busy, and no down-sweep is needed)
  HsArgs lv[32];
  double* buf[2] = {at<double>(ws, Lo.elem[0]), at<double>(ws, Lo.hs)};
  for (int l = 0; l < Lo.L_hs; ++l) {
    lv[l].src = buf[l & 1];
    lv[l].dst = buf[(l + 1) & 1];
    lv[l].n = Lo.nb;
    lv[l].s = 1 << l;
    lv[l].status = status;
    lv[l].fail_bit = fail_bit;
  }
  P.pre_elem = buf[Lo.L_hs & 1];
  return hip_check(launch_filter_scan_any(Lo.D, M, P, lv, Lo.L_hs, st), "filter launch");
}

// log Z of the auxiliary model only: block fold, then the up-sweep reduction
// of the block elements; *lz points at the root element's normaliser.
akf_status run_filter_logz(const Layout& Lo, const KModel& M, void* ws, const double* om,
                           const double* Om, const double* Omd, int* status, int fail_bit,
                           hipStream_t st, const double* Ft, const double* bt,
                           const double** lz) {
  FilterArgs P{};
  P.B = Lo.B;
  P.om = om;
  P.Om = Om;
  P.Omd = Omd;
  P.elem = at<double>(ws, Lo.elem[0]);
  P.ldm = Lo.D;
  P.status = status;
  P.fail_bit = fail_bit;
  P.Ft = Ft;
  P.bt = bt;
  TreeArgs up[kMaxLevels], down[kMaxLevels];
  fill_tree(Lo, ws, 0, Lo.elem, Lo.pre, status, fail_bit, up, down);
  const int D = Lo.D;
  *lz = at<double>(ws, Lo.elem[Lo.L]) + (3 * D * D + 2 * D);  // ElemLayout<D>::lc
  return hip_check(launch_filter_logz_any(D, M, P, up, Lo.L, st), "log-likelihood launch");
}

akf_status run_sampler(const Layout& Lo, const KModel& M, void* ws, const double* mf,
                       const double* Pf, int ldm, const double* xi_x, double* xs, int* status,
                       hipStream_t st, const double* Ft, const double* bt, double* Lc,
                       double* Et) {
  SampArgs S{};
  S.Ft = Ft;
  S.bt = bt;
  S.Lc = Lc;
  S.Et = Et;
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

void fill_egl_tree(const Layout& Lo, void* ws, EglTree* up, EglTree* down) {
  for (int l = 1; l <= Lo.L; ++l) {
    EglTree u{};
    u.src = at<double>(ws, Lo.eagg[l - 1]);
    u.dst = at<double>(ws, Lo.eagg[l]);
    u.n_src = Lo.n_lvl[l - 1];
    u.n_dst = Lo.n_lvl[l];
    up[l - 1] = u;
    EglTree d{};
    d.src = at<double>(ws, Lo.eagg[l - 1]);
    d.pre_src = at<double>(ws, Lo.estate[l]);
    d.pre_dst = at<double>(ws, Lo.estate[l - 1]);
    d.n_src = Lo.n_lvl[l];
    d.n_dst = Lo.n_lvl[l - 1];
    down[l - 1] = d;
  }
}

// Suffix (E, g, L) scan over E = ws.E, L = ws.Lm, g (nullable); writes outL/outg.
akf_status run_egl(const Layout& Lo, void* ws, const double* g, double* outL, double* outg,
                   int ldo, int dout, hipStream_t st) {
  const int D = Lo.D;
  akf_status s;
  // the suffix state entering the last block is zero (it meets E = 0)
  if ((s = hip_check(launch_zero(at<double>(ws, Lo.estate[Lo.L]), (int64_t)D * D + D, st),
                     "zero launch")) != AKF_OK)
    return s;
  EglArgs A{};
  A.N = Lo.N;
  A.B = Lo.B;
  A.E = at<double>(ws, Lo.E);
  A.g = g;
  A.L = at<double>(ws, Lo.Lm);
  A.agg = at<double>(ws, Lo.eagg[0]);
  A.state = at<double>(ws, Lo.estate[0]);
  A.outL = outL;
  A.outg = outg;
  A.ldo = ldo;
  A.dout = dout;
  EglTree up[kMaxLevels], down[kMaxLevels];
  fill_egl_tree(Lo, ws, up, down);
  return hip_check(launch_egl_scan_any(D, A, up, down, Lo.L, st), "(E,g,L) scan launch");
}


const char* last_error() { return g_err; }

}  // namespace akf
