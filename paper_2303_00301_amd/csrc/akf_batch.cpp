// akf_batch.cpp -- batched chains: plan creation (per-chain workspaces,
// device descriptors, work tables), the scan-block autotuner, and the
// graph-captured multi-step run (include/akf.h, akf_batch_*).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/akf.h"
#include "akf_internal.h"
#include "akf_layout.h"

using namespace akf;

struct ClassPlan {
  int D = 0, B = 0, Lmax = 0;
  int sb_teams = 2;  // sampler-build teams per SIMD (1 or 2; D = 64 teams take a CU)
  std::vector<int> chains;
  struct Tab {
    size_t off = 0;  // index into the item table
    int n = 0, grid = 0;
  };
  // fold_team / fold_lane and sbuild / sbuild_lane: the per-block and
  // per-step items of the chains on teams and of those on one lane per item
  // (d <= 4 in the 16-wide class)
  Tab init, lin, fold_team, fold_lane, sbuild, sbuild_lane, fin, up[kMaxLv + 1],
      down[kMaxLv + 1];
};

struct akf_batch_plan {
  int n_chains = 0, n_steps = 0;
  std::vector<akf_chain> chains;
  std::vector<ClassPlan> classes;
  char* dmem = nullptr;
  size_t dbytes = 0;
  ChainDev* d_desc = nullptr;
  Item* d_items = nullptr;
  int* d_step = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int grid_for(int n, int cap) { return std::max(1, std::min(n, cap)); }

akf_status check_chain(const akf_chain& c, int k) {
  akf_status s = check_model(&c.model, true);
  if (s != AKF_OK) return s;
  if ((s = check_linear(&c.model, "batched chains")) != AKF_OK) return s;
  if (c.model.emit == AKF_EMIT_GAUSSIAN || c.model.emit == AKF_EMIT_MVT)
    return fail(AKF_ERR_UNSUPPORTED, "chain %d: batched chains support the Poisson, "
                    "Student-t and stochastic-volatility emission families", k);
  if (!c.y || !c.x || !c.xi || !c.unif)
    return fail(AKF_ERR_INVALID, "chain %d: y, x, xi and unif must be non-NULL", k);
  if (!(c.delta > 0.0)) return fail(AKF_ERR_INVALID, "chain %d: delta must be > 0", k);
  if (c.order != 1 && c.order != 2) return fail(AKF_ERR_INVALID, "chain %d: order must be 1 or 2", k);
  return AKF_OK;
}

// Host-side description of one class layout (without device memory).
struct Built {
  std::vector<ChainDev> desc;   // indexed by global chain id (only class members filled)
  std::vector<Item> items;
  std::vector<size_t> ws_off;   // per global chain
  size_t ws_total = 0;
};

// Scratch outputs of an autotuning candidate's first step: paths in place of
// the chains' x, and per-chain log ratio, decision and status.
// steps per trial (the device step counter is reset before the checked step
// and before the timed ones)
constexpr int kTrialSteps = 2;
struct TrialOut {
  std::vector<double*> x;
  double* lr = nullptr;
  int* acc = nullptr;
  int* st = nullptr;
};

void build_class(ClassPlan& cp, const std::vector<akf_chain>& chains, Built& b, char* ws_base,
                 const TrialOut* trial) {
  cp.Lmax = 0;
  std::vector<Layout> lay(chains.size());
  for (int c : cp.chains) {
    make_layout(lay[c], chains[c].model.N, chains[c].model.dx, chains[c].model.dy, cp.B,
                LAYOUT_STEP);
    cp.Lmax = std::max(cp.Lmax, lay[c].L);
  }
  auto tab = [&](ClassPlan::Tab& t, auto gen, int cap) {
    t.off = b.items.size();
    gen();
    t.n = (int)(b.items.size() - t.off);
    t.grid = grid_for(t.n, cap);
  };
  // team phases: one workgroup per item here; each launch then caps its grid
  // at what its kernel keeps resident on the chip (launch_batch_phase)
  const int team_cap = INT_MAX;
  tab(cp.init, [&] { for (int c : cp.chains) b.items.push_back({c, 0}); }, 1024);
  tab(cp.lin, [&] {
    for (int c : cp.chains) {
      const int nchunk = (int)(((int64_t)chains[c].model.N * chains[c].model.dx + 255) / 256);
      for (int k = 0; k < nchunk; ++k) b.items.push_back({c, k});
    }
  }, 8192);
  auto on_lane = [&](int c) { return cp.D == 16 && chains[c].model.dx <= kLaneMaxD; };
  tab(cp.fold_team, [&] {
    for (int c : cp.chains)
      if (!on_lane(c))
        for (int k = 0; k < lay[c].nb; ++k) b.items.push_back({c, k});
  }, team_cap);
  tab(cp.fold_lane, [&] {
    for (int c : cp.chains)
      if (on_lane(c))
        for (int k = 0; k < lay[c].nb; ++k) b.items.push_back({c, k});
  }, team_cap);
  tab(cp.sbuild, [&] {
    for (int c : cp.chains)
      if (!on_lane(c))
        for (int t = 0; t < chains[c].model.N; ++t) b.items.push_back({c, t});
  }, team_cap);
  tab(cp.sbuild_lane, [&] {
    for (int c : cp.chains)
      if (on_lane(c))
        for (int t = 0; t < chains[c].model.N; ++t) b.items.push_back({c, t});
  }, team_cap);
  tab(cp.fin, [&] { for (int c : cp.chains) b.items.push_back({c, 0}); }, 1024);
  for (int l = 1; l <= cp.Lmax; ++l) {
    tab(cp.up[l], [&] {
      for (int c : cp.chains)
        if (lay[c].L >= l)
          for (int k = 0; k < lay[c].n_lvl[l]; ++k) b.items.push_back({c, k});
    }, team_cap);
    tab(cp.down[l], [&] {
      for (int c : cp.chains)
        if (lay[c].L >= l)
          for (int k = 0; k < lay[c].n_lvl[l]; ++k) b.items.push_back({c, k});
    }, team_cap);
  }
  // workspaces and descriptors
  for (int c : cp.chains) {
    const Layout& Lo = lay[c];
    b.ws_off[c] = b.ws_total;
    b.ws_total += (Lo.total + 255) / 256 * 256;
  }
  if (!ws_base) return;
  for (int c : cp.chains) {
    const Layout& Lo = lay[c];
    const akf_chain& ch = chains[c];
    void* ws = ws_base + b.ws_off[c];
    ChainDev& d = b.desc[c];
    memset(&d, 0, sizeof d);
    d.M = to_kmodel(&ch.model);
    double* x = trial ? trial->x[c] : ch.x;
    StepArgs& A = d.A;
    A.y = ch.y;
    A.x = x;
    A.delta = ch.delta;
    A.order = ch.order;
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
    A.status = at<int>(ws, Lo.status);
    A.accept_flag = at<int>(ws, Lo.accept);
    FilterArgs F{};
    F.B = Lo.B;
    F.elem = at<double>(ws, Lo.elem[0]);
    F.pre = at<double>(ws, Lo.pre[0]);
    F.status = A.status;
    d.Ff = F;
    d.Ff.om = A.om;
    d.Ff.Om = A.Om;
    d.Ff.mf = at<double>(ws, Lo.mf);
    d.Ff.Pf = at<double>(ws, Lo.Pf);
    d.Ff.ldm = Lo.D;
    d.Ff.ell = A.ell;
    d.Ff.fail_bit = ST_FWD_NOT_PD;
    d.Fr = F;
    d.Fr.om = A.om2;
    d.Fr.Om = A.Om2;
    d.Fr.ldm = Lo.D;
    d.Fr.ell = A.ell2;
    d.Fr.fail_bit = ST_REV_NOT_PD;
    SampArgs& S = d.S;
    S.B = Lo.B;
    S.mf = d.Ff.mf;
    S.Pf = d.Ff.Pf;
    S.ldm = Lo.D;
    S.E = at<double>(ws, Lo.E);
    S.U = at<double>(ws, Lo.U);
    S.agg = at<double>(ws, Lo.sagg[0]);
    S.xin = at<double>(ws, Lo.xin[0]);
    S.xs = A.xs;
    S.status = A.status;
    const int nchunk = (int)(((int64_t)ch.model.N * ch.model.dx + 255) / 256);
    d.Fin.n_part_fwd = nchunk;
    d.Fin.n_part_rev = nchunk;
    d.L = Lo.L;
    d.n_part = nchunk;
    TreeArgs up[kMaxLevels], down[kMaxLevels];
    fill_tree(Lo, ws, 0, Lo.elem, Lo.pre, A.status, ST_FWD_NOT_PD, up, down);
    for (int l = 0; l < Lo.L; ++l) {
      d.fup[l] = up[l];
      d.fdown[l] = down[l];
    }
    fill_tree(Lo, ws, 0, Lo.sagg, Lo.xin, A.status, ST_FWD_NOT_PD, up, down);
    for (int l = 0; l < Lo.L; ++l) {
      d.sup[l] = up[l];
      d.sdown[l] = down[l];
    }
    d.root_flag = root_flag(Lo, ws);
    d.root_xin = at<double>(ws, Lo.xin[Lo.L]);
    d.xi_base = ch.xi;
    d.xi_stride = 2 * (int64_t)ch.model.N * ch.model.dx;
    d.unif_base = ch.unif;
    if (!trial) {
      d.lr_base = ch.log_ratio;
      d.acc_base = ch.accepted;
      d.lzf_base = ch.logZ_fwd;
      d.lzr_base = ch.logZ_rev;
      d.st_base = ch.status;
    } else {
      // kTrialSteps slots per chain; only the first step of a trial is read back
      d.lr_base = trial->lr + (size_t)kTrialSteps * c;
      d.acc_base = trial->acc + (size_t)kTrialSteps * c;
      d.st_base = trial->st + (size_t)kTrialSteps * c;
    }
    d.x = x;
  }
}

hipError_t enqueue_class_step_part(const ClassPlan& cp, const ChainDev* d_desc, const Item* d_items,
                                   const int* d_step, int part, hipStream_t st) {
  auto L = [&](const ClassPlan::Tab& t) {
    BatchLaunch b;
    b.cd = d_desc;
    b.items = d_items + t.off;
    b.n_items = t.n;
    b.grid = t.grid;
    return b;
  };
  hipError_t e = hipSuccess;
  auto run = [&](int phase, const ClassPlan::Tab& t, int level, int rev) {
    if (e == hipSuccess) e = launch_batch_phase(cp.D, phase, L(t), level, rev, d_step, st);
  };
  // the timing hook brackets a phase's team and lane launches together
  const int fam_off = cp.D == 16 ? 0 : cp.D == 32 ? 1 : 2;
  auto filter = [&](int rev) {
    timing_mark(FAM_BATCH_FOLD16 + fam_off, 1, st);
    run(BP_FOLD_LANE, cp.fold_lane, 0, rev);
    run(BP_FOLD, cp.fold_team, 0, rev);
    timing_mark(FAM_BATCH_FOLD16 + fam_off, 0, st);
    for (int l = 1; l <= cp.Lmax; ++l) run(BP_UP, cp.up[l], l, rev);
    for (int l = cp.Lmax; l >= 1; --l) run(BP_DOWN, cp.down[l], l, rev);
    run(BP_FINAL_LANE, cp.fold_lane, 0, rev);
    run(BP_FINAL, cp.fold_team, 0, rev);
  };
  switch (part) {
    case 0:
      run(BP_INIT, cp.init, 0, 0);
      run(BP_LIN_FWD, cp.lin, 0, 0);
      filter(0);
      break;
    case 1:
      timing_mark(FAM_BATCH_SBUILD16 + fam_off, 1, st);
      run(BP_SBUILD_LANE, cp.sbuild_lane, 0, 0);
      run(cp.sb_teams == 2 ? BP_SBUILD : BP_SBUILD1, cp.sbuild, 0, 0);
      timing_mark(FAM_BATCH_SBUILD16 + fam_off, 0, st);
      run(BP_SFOLD_LANE, cp.fold_lane, 0, 0);
      run(BP_SFOLD, cp.fold_team, 0, 0);
      for (int l = 1; l <= cp.Lmax; ++l) run(BP_SUP, cp.up[l], l, 0);
      for (int l = cp.Lmax; l >= 1; --l) run(BP_SDOWN, cp.down[l], l, 0);
      run(BP_SFINAL_LANE, cp.fold_lane, 0, 0);
      run(BP_SFINAL, cp.fold_team, 0, 0);
      break;
    case 2:
      run(BP_LIN_REV, cp.lin, 0, 1);
      filter(1);
      run(BP_FINALIZE, cp.fin, 0, 0);
      run(BP_SELECT, cp.lin, 0, 0);
      break;
  }
  return e;
}

hipError_t enqueue_step(const std::vector<ClassPlan>& classes, const ChainDev* d_desc,
                        const Item* d_items, int* d_step, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int part = 0; part < 3 && e == hipSuccess; ++part)
    for (const ClassPlan& cp : classes) {
      e = enqueue_class_step_part(cp, d_desc, d_items, d_step, part, st);
      if (e != hipSuccess) break;
    }
  if (e == hipSuccess) e = launch_step_advance(d_step, 0, st);
  return e;
}

// Plain per-chain reference for the autotuner: one akf_mh_step of every chain
// of the class from its current path with the run's first normals and uniform.
struct PlainRef {
  std::vector<std::vector<double>> x;  // by global chain id (class members only)
  std::vector<double> lr;
  std::vector<int> acc, st;
};

akf_status plain_reference(const std::vector<akf_chain>& chains, const ClassPlan& cp,
                           hipStream_t st, PlainRef& ref) {
  size_t ws_need = 0, x_need = 0;
  for (int c : cp.chains) {
    const akf_chain& ch = chains[c];
    ws_need = std::max(ws_need, akf_mh_workspace_bytes(&ch.model, ch.order, 0));
    x_need = std::max(x_need, (size_t)ch.model.N * ch.model.dx);
  }
  if (ws_need == 0) return fail(AKF_ERR_INVALID, "autotuning: a chain's workspace query failed");
  const size_t xb = (x_need * 8 + 255) / 256 * 256;
  char* mem = nullptr;
  if (hipMalloc(&mem, xb + 256 + ws_need) != hipSuccess)
    return fail(AKF_ERR_HIP, "autotuning: hipMalloc of the plain reference's workspace failed");
  double* xo = reinterpret_cast<double*>(mem);
  double* lr = reinterpret_cast<double*>(mem + xb);
  int* ai = reinterpret_cast<int*>(mem + xb + 8);
  int* si = reinterpret_cast<int*>(mem + xb + 16);
  void* ws = mem + xb + 256;
  ref.x.assign(chains.size(), {});
  ref.lr.assign(chains.size(), 0.0);
  ref.acc.assign(chains.size(), 0);
  ref.st.assign(chains.size(), 0);
  akf_status s = AKF_OK;
  for (int c : cp.chains) {
    const akf_chain& ch = chains[c];
    s = akf_mh_step(&ch.model, ch.y, ch.x, ch.delta, ch.order, ch.xi, ch.unif, xo, lr, ai,
                    nullptr, nullptr, si, ws, ws_need, 0, st);
    if (s != AKF_OK) break;
    ref.x[c].resize((size_t)ch.model.N * ch.model.dx);
    hipError_t e = hipMemcpyAsync(ref.x[c].data(), xo, ref.x[c].size() * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&ref.lr[c], lr, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&ref.acc[c], ai, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&ref.st[c], si, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      s = fail(AKF_ERR_HIP, "autotuning: plain reference step: %s", hipGetErrorString(e));
      break;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(mem);
  return s;
}

// The candidate's first step agrees with the plain step of every chain: the
// same status; with the same decision, the same log ratio and path up to the
// rounding of a different association of the scans; a different decision
// only at a tie of the log ratio with log U.
bool candidate_agrees(const std::vector<akf_chain>& chains, const ClassPlan& cp,
                      const PlainRef& ref, const std::vector<std::vector<double>>& x,
                      const std::vector<double>& lr, const std::vector<int>& acc,
                      const std::vector<int>& stv) {
  for (int c : cp.chains) {
    const akf_chain& ch = chains[c];
    const double nd = (double)ch.model.N * ch.model.dx;
    const double tol_lr = 1e-9 * nd + 1e-9 * std::max(1.0, std::fabs(ref.lr[c]));
    if (stv[c] != ref.st[c]) return false;
    if (ref.st[c] != 0) continue;  // both rejected by a status bit: x unchanged
    if (!(std::fabs(lr[c] - ref.lr[c]) <= tol_lr)) return false;
    if (acc[c] != ref.acc[c]) continue;  // a tie: the log ratios agree
    double num = 0.0, den = 0.0;
    for (size_t i = 0; i < x[c].size(); ++i) {
      const double e = x[c][i] - ref.x[c][i];
      num += e * e;
      den += ref.x[c][i] * ref.x[c][i];
    }
    if (!(std::sqrt(num) <= 1e-7 * std::max(1.0, std::sqrt(den)))) return false;
  }
  return true;
}

// Time one eager step of class `cp` with block B on scratch state (after an
// untimed first step whose outputs are checked against `ref`).  Returns ms,
// -1 on a failure, -2 when the first step disagrees with the plain path.
double time_candidate(const std::vector<akf_chain>& chains, ClassPlan cp, const PlainRef& ref,
                      hipStream_t st) {
  Built b;
  b.desc.resize(chains.size());
  b.ws_off.assign(chains.size(), 0);
  build_class(cp, chains, b, nullptr, nullptr);
  // scratch x copies and per-chain outputs
  size_t xbytes = 0;
  for (int c : cp.chains) xbytes += ((size_t)chains[c].model.N * chains[c].model.dx * 8 + 255) / 256 * 256;
  const size_t nc = chains.size();
  const size_t out_bytes = (nc * 16 * kTrialSteps + 255) / 256 * 256;
  const size_t desc_bytes = (nc * sizeof(ChainDev) + 255) / 256 * 256;
  const size_t item_bytes = (b.items.size() * sizeof(Item) + 255) / 256 * 256;
  const size_t head = desc_bytes + item_bytes + 256 + out_bytes;
  const size_t total = head + xbytes + b.ws_total;
  char* mem = nullptr;
  if (hipMalloc(&mem, total) != hipSuccess) return -1.0;
  char* ws = mem + head + xbytes;
  TrialOut tr;
  tr.x.assign(nc, nullptr);
  tr.lr = reinterpret_cast<double*>(mem + desc_bytes + item_bytes + 256);
  tr.acc = reinterpret_cast<int*>(tr.lr + kTrialSteps * nc);
  tr.st = tr.acc + kTrialSteps * nc;
  size_t xo = 0;
  for (int c : cp.chains) {
    tr.x[c] = reinterpret_cast<double*>(mem + head + xo);
    const size_t nb = (size_t)chains[c].model.N * chains[c].model.dx * 8;
    (void)hipMemcpyAsync(tr.x[c], chains[c].x, nb, hipMemcpyDeviceToDevice, st);
    xo += (nb + 255) / 256 * 256;
  }
  b.items.clear();
  b.ws_total = 0;
  build_class(cp, chains, b, ws, &tr);
  (void)launch_zero(reinterpret_cast<double*>(ws), (int64_t)(b.ws_total / 8), st);  // as the plan's
  ChainDev* d_desc = reinterpret_cast<ChainDev*>(mem);
  Item* d_items = reinterpret_cast<Item*>(mem + desc_bytes);
  int* d_step = reinterpret_cast<int*>(mem + desc_bytes + item_bytes);
  (void)hipMemcpyAsync(d_desc, b.desc.data(), nc * sizeof(ChainDev), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(d_items, b.items.data(), b.items.size() * sizeof(Item), hipMemcpyHostToDevice, st);
  std::vector<ClassPlan> one{cp};
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double ms = -1.0;
  hipError_t err = launch_step_advance(d_step, 1, st);
  if (err == hipSuccess) err = enqueue_step(one, d_desc, d_items, d_step, st);  // checked step
  // read the checked step back before the timed steps overwrite x
  std::vector<std::vector<double>> xh(nc);
  std::vector<double> lr(kTrialSteps * nc, 0.0), lr0(nc, 0.0);
  std::vector<int> acc(kTrialSteps * nc, 0), stv(kTrialSteps * nc, 0), acc0(nc, 0), st0(nc, 0);
  for (int c : cp.chains) {
    if (err != hipSuccess) break;
    xh[c].resize((size_t)chains[c].model.N * chains[c].model.dx);
    err = hipMemcpyAsync(xh[c].data(), tr.x[c], xh[c].size() * 8, hipMemcpyDeviceToHost, st);
  }
  if (err == hipSuccess)
    err = hipMemcpyAsync(lr.data(), tr.lr, lr.size() * 8, hipMemcpyDeviceToHost, st);
  if (err == hipSuccess)
    err = hipMemcpyAsync(acc.data(), tr.acc, acc.size() * 4, hipMemcpyDeviceToHost, st);
  if (err == hipSuccess)
    err = hipMemcpyAsync(stv.data(), tr.st, stv.size() * 4, hipMemcpyDeviceToHost, st);
  if (err == hipSuccess) err = hipStreamSynchronize(st);
  for (int c : cp.chains) {
    lr0[c] = lr[(size_t)kTrialSteps * c];
    acc0[c] = acc[(size_t)kTrialSteps * c];
    st0[c] = stv[(size_t)kTrialSteps * c];
  }
  const bool agrees = err == hipSuccess && candidate_agrees(chains, cp, ref, xh, lr0, acc0, st0);
  if (err == hipSuccess && agrees) {
    err = launch_step_advance(d_step, 1, st);
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 2 && err == hipSuccess; ++r) {
      err = enqueue_step(one, d_desc, d_items, d_step, st);
      if (err == hipSuccess) err = launch_step_advance(d_step, 1, st);
    }
    (void)hipEventRecord(e1, st);
    if (err == hipSuccess && hipEventSynchronize(e1) == hipSuccess) {
      float f = 0.f;
      if (hipEventElapsedTime(&f, e0, e1) == hipSuccess) ms = f / 2.0;
    }
  } else if (err == hipSuccess) {
    ms = -2.0;
  }
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(mem);
  return ms;
}

// Cache key of a class: its team size and the shape of its batch (chain
// count, lengths, the histograms of d_x, order and emission family).  Stored
// as the leading fields of a cache line, before "block".
std::string cache_key(const ClassPlan& cp, const std::vector<akf_chain>& chains) {
  long long sumN = 0;
  int maxN = 0;
  int ndx[65] = {0}, nord[3] = {0}, nemit[8] = {0};
  for (int c : cp.chains) {
    const akf_model& m = chains[c].model;
    sumN += m.N;
    maxN = std::max(maxN, (int)m.N);
    ndx[m.dx] += 1;
    nord[chains[c].order] += 1;
    nemit[m.emit & 7] += 1;
  }
  std::string k;
  char buf[96];
  snprintf(buf, sizeof buf, "\"D\": %d, \"chains\": %zu, \"sum_N\": %lld, \"max_N\": %d, \"dx\": \"",
           cp.D, cp.chains.size(), sumN, maxN);
  k += buf;
  bool first = true;
  for (int d = 1; d <= 64; ++d)
    if (ndx[d]) {
      snprintf(buf, sizeof buf, "%s%d:%d", first ? "" : " ", d, ndx[d]);
      k += buf;
      first = false;
    }
  snprintf(buf, sizeof buf, "\", \"order\": \"1:%d 2:%d\", \"emit\": \"", nord[1], nord[2]);
  k += buf;
  first = true;
  for (int e = 0; e < 8; ++e)
    if (nemit[e]) {
      snprintf(buf, sizeof buf, "%s%d:%d", first ? "" : " ", e, nemit[e]);
      k += buf;
      first = false;
    }
  k += "\"";
  return k;
}

// Block and sampler-build layout of the last verified line whose key fields
// equal `key` exactly; B = 0 when there is none.
int cache_lookup(const char* path, const std::string& key, int* sb_teams) {
  if (!path) return 0;
  FILE* f = fopen(path, "r");
  if (!f) return 0;
  std::string line;
  int B = 0;
  char buf[1024];
  while (fgets(buf, sizeof buf, f)) {
    line = buf;
    const size_t kb = line.find(", \"block\": ");
    if (line.size() < 2 || line[0] != '{' || kb == std::string::npos) continue;
    if (line.compare(1, kb - 1, key) != 0 || kb - 1 != key.size()) continue;
    if (line.find("\"verified\": true") == std::string::npos) continue;
    static const char kTeams[] = "\"sbuild_teams_per_simd\": ";
    const size_t ks = line.find(kTeams);
    if (ks == std::string::npos) continue;  // a line of an older layout search
    const int b = atoi(line.c_str() + kb + 11);
    const int t = atoi(line.c_str() + ks + sizeof kTeams - 1);
    if (b > 0 && (t == 1 || t == 2)) {
      B = b;
      *sb_teams = t;
    }
  }
  fclose(f);
  return B;
}

void cache_store(const char* path, const std::string& key, int B, int sb_teams, double ms) {
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f,
          "{%s, \"block\": %d, \"sbuild_teams_per_simd\": %d, \"ms_per_step\": %.4f, "
          "\"verified\": true}\n",
          key.c_str(), B, sb_teams, ms);
  fclose(f);
}

}  // namespace

extern "C" {

akf_status akf_batch_plan_create(akf_batch_plan** out, int32_t n_chains, const akf_chain* chains,
                                 int32_t n_steps, int32_t block, const char* tune_cache,
                                 void* stream) {
  if (!out) return fail(AKF_ERR_INVALID, "plan output pointer is NULL");
  *out = nullptr;
  if (n_chains < 1 || !chains) return fail(AKF_ERR_INVALID, "need at least one chain");
  if (n_steps < 0) return fail(AKF_ERR_INVALID, "n_steps must be >= 0");
  if (block < 0) return fail(AKF_ERR_INVALID, "block must be >= 0");
  for (int k = 0; k < n_chains; ++k) {
    akf_status s = check_chain(chains[k], k);
    if (s != AKF_OK) return s;
    if (block > 0) {
      Layout Lo;
      make_layout(Lo, chains[k].model.N, chains[k].model.dx, chains[k].model.dy, block, LAYOUT_STEP);
      if (Lo.L > kMaxLv) return fail(AKF_ERR_SHAPE, "chain %d: scan tree deeper than %d levels", k, kMaxLv);
    }
  }
  akf_status s = prepare_device();
  if (s != AKF_OK) return s;
  for (int D : {16, 32, 64}) batch_caps(D);
  hipStream_t st = (hipStream_t)stream;
  akf_batch_plan* P = new akf_batch_plan();
  P->n_chains = n_chains;
  P->n_steps = n_steps;
  P->chains.assign(chains, chains + n_chains);
  // group chains by team size D
  for (int D : {16, 32, 64}) {
    ClassPlan cp;
    cp.D = D;
    for (int k = 0; k < n_chains; ++k)
      if (pick_D(chains[k].model.dx) == D) cp.chains.push_back(k);
    if (cp.chains.empty()) continue;
    int B = block;
    int sb_teams = 2;
    if (B == 0) {
      const std::string key = cache_key(cp, P->chains);
      B = cache_lookup(tune_cache, key, &sb_teams);
      if (B == 0) {
        // autotune the scan block on this batch: each candidate's first step is
        // checked against plain per-chain steps, then two eager steps are timed
        PlainRef ref;
        akf_status rs = plain_reference(P->chains, cp, st, ref);
        if (rs != AKF_OK) {
          delete P;
          return rs;
        }
        double best = 1e300;
        int maxN = 0, n_disagree = 0;
        for (int c : cp.chains) maxN = std::max(maxN, (int)chains[c].model.N);
        // the search covers the block and, at D = 32, the sampler build's
        // teams per SIMD
        for (int cand : {4, 8, 16, 32, 64, 128}) {
          if (cand > maxN && cand != 4) break;
          for (int teams : {2, 1}) {
            if (teams == 1 && D != 32) continue;
            ClassPlan trial = cp;
            trial.B = cand;
            trial.sb_teams = teams;
            const double ms = time_candidate(P->chains, trial, ref, st);
            if (ms == -2.0) ++n_disagree;
            if (ms > 0 && ms < best) {
              best = ms;
              B = cand;
              sb_teams = teams;
            }
          }
        }
        if (B == 0) {
          delete P;
          return fail(AKF_ERR_HIP, "autotuning failed for D = %d (%d candidates disagreed with "
                      "the plain per-chain step)", D, n_disagree);
        }
        cache_store(tune_cache, key, B, sb_teams, best);
      }
    }
    cp.B = B;
    cp.sb_teams = sb_teams;
    P->classes.push_back(cp);
  }
  // final layout: descriptors, items, step counter, workspaces in one allocation
  Built b;
  b.desc.resize(n_chains);
  b.ws_off.assign(n_chains, 0);
  for (ClassPlan& cp : P->classes) build_class(cp, P->chains, b, nullptr, nullptr);
  const size_t desc_bytes = ((size_t)n_chains * sizeof(ChainDev) + 255) / 256 * 256;
  const size_t item_bytes = (b.items.size() * sizeof(Item) + 255) / 256 * 256;
  P->dbytes = desc_bytes + item_bytes + 256 + b.ws_total;
  if (hipMalloc(&P->dmem, P->dbytes) != hipSuccess) {
    delete P;
    return fail(AKF_ERR_HIP, "hipMalloc of %zu bytes for the batch plan failed", b.ws_total);
  }
  char* ws = P->dmem + desc_bytes + item_bytes + 256;
  b.items.clear();
  b.ws_total = 0;
  for (ClassPlan& cp : P->classes) build_class(cp, P->chains, b, ws, nullptr);
  // zero once: the padding of arrays that only the lane kernels write
  // (akf_lane.hip stores the 4 x 4 corners) stays zero from here on
  if (launch_zero(reinterpret_cast<double*>(ws), (int64_t)(b.ws_total / 8), st) != hipSuccess) {
    akf_batch_plan_destroy(P);
    return fail(AKF_ERR_HIP, "zeroing the batch plan's workspace failed");
  }
  P->d_desc = reinterpret_cast<ChainDev*>(P->dmem);
  P->d_items = reinterpret_cast<Item*>(P->dmem + desc_bytes);
  P->d_step = reinterpret_cast<int*>(P->dmem + desc_bytes + item_bytes);
  hipError_t e = hipMemcpyAsync(P->d_desc, b.desc.data(), (size_t)n_chains * sizeof(ChainDev),
                                hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->d_items, b.items.data(), b.items.size() * sizeof(Item),
                       hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    akf_batch_plan_destroy(P);
    return fail(AKF_ERR_HIP, "uploading the batch plan failed: %s", hipGetErrorString(e));
  }
  *out = P;
  return AKF_OK;
}

akf_status akf_batch_mh_run(akf_batch_plan* P, int32_t use_graph, void* stream) {
  if (!P) return fail(AKF_ERR_INVALID, "plan is NULL");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = launch_step_advance(P->d_step, 1, st);
  if (e != hipSuccess) return fail(AKF_ERR_HIP, "step reset: %s", hipGetErrorString(e));
  if (!use_graph) {
    for (int k = 0; k < P->n_steps; ++k) {
      e = enqueue_step(P->classes, P->d_desc, P->d_items, P->d_step, st);
      if (e != hipSuccess) return fail(AKF_ERR_HIP, "batched step: %s", hipGetErrorString(e));
    }
    return AKF_OK;
  }
  if (!P->exec) {
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess)
      return fail(AKF_ERR_HIP, "stream capture needs a non-default stream: %s",
                      hipGetErrorString(e));
    hipError_t e2 = enqueue_step(P->classes, P->d_desc, P->d_items, P->d_step, st);
    e = hipStreamEndCapture(st, &P->graph);
    if (e2 != hipSuccess || e != hipSuccess)
      return fail(AKF_ERR_HIP, "capturing the batched step failed: %s",
                      hipGetErrorString(e2 != hipSuccess ? e2 : e));
    e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    if (e != hipSuccess)
      return fail(AKF_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  }
  for (int k = 0; k < P->n_steps; ++k) {
    e = hipGraphLaunch(P->exec, st);
    if (e != hipSuccess) return fail(AKF_ERR_HIP, "graph launch: %s", hipGetErrorString(e));
  }
  return AKF_OK;
}

akf_status akf_batch_plan_info(const akf_batch_plan* P, int32_t max_classes, int32_t* n_classes,
                               int32_t* D, int32_t* block, int32_t* n_chains_in_class,
                               int32_t* sbuild_teams_per_simd, size_t* device_bytes) {
  if (!P || !n_classes) return fail(AKF_ERR_INVALID, "plan and n_classes must be non-NULL");
  *n_classes = (int32_t)P->classes.size();
  for (int i = 0; i < (int)P->classes.size() && i < max_classes; ++i) {
    if (D) D[i] = P->classes[i].D;
    if (block) block[i] = P->classes[i].B;
    if (n_chains_in_class) n_chains_in_class[i] = (int32_t)P->classes[i].chains.size();
    if (sbuild_teams_per_simd)
      sbuild_teams_per_simd[i] = P->classes[i].D == 32 ? P->classes[i].sb_teams : 0;
  }
  if (device_bytes) *device_bytes = P->dbytes;
  return AKF_OK;
}

void akf_batch_plan_destroy(akf_batch_plan* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->dmem) (void)hipFree(P->dmem);
  delete P;
}

}  // extern "C"
