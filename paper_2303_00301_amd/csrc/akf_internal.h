// akf_internal.h -- structures shared by the kernels and the host launcher.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace akf {

enum { EMIT_GAUSSIAN = 0, EMIT_POISSON_LOG = 1, EMIT_STUDENT_T = 2, EMIT_STOCH_VOL = 3,
       EMIT_MVT = 4, EMIT_GAUSS_SITE = 5, EMIT_GAUSS_QUAD = 6 };
enum { DYN_LINEAR = 0, DYN_LORENZ63 = 1, DYN_LORENZ96 = 2 };
enum { ST_FWD_NOT_PD = 1, ST_REV_NOT_PD = 2, ST_NONFINITE = 4 };

// time steps (one wave each) per workgroup of the multivariate-t linearisation
constexpr int kMvtWaves = 4;
// time steps per workgroup of the Gaussian-emission linearisation (four waves,
// each taking every fourth of them)
constexpr int kGaussStepsPerBlock = 16;

// Device-side gate of a launch: the kernel runs iff w == nullptr or
// lo <= *w <= hi; every workgroup reads the word at entry and leaves at once
// when the gate is shut, so one launch sequence can serve branches that are
// decided on the device (and be captured in a graph).
struct Gate {
  const int* w;
  int lo, hi;
};

__device__ __forceinline__ bool gate_shut(const Gate& g) {
  if (!g.w) return false;
  const int v = *g.w;
  return v < g.lo || v > g.hi;
}

// Model as the kernels see it (all arrays are device pointers, d-sized).
struct KModel {
  int N, d, dy, emit;
  const double *m0, *P0, *F, *b, *Q;
  const double *H, *R;
  const int* site;
  double nu, scale;
  int dyn;
  double dyn_par[4];
  double obs_beta, slr_var;  // quadratic observation mean; order-3 reference variance
  Gate gate;                 // launches of the reuse path's branches (closed = skip)
};

// Filter element (A, b, C, eta, J), padded to D, and lc = log c, the
// normaliser of p(omega | x_prev) = exp(lc + eta' x - x' J x / 2); the prefix
// from t = 0 carries log p(omega_{0:t}).
template <int D>
struct ElemLayout {
  static constexpr int A = 0, C = D * D, J = 2 * D * D, b = 3 * D * D, eta = 3 * D * D + D;
  static constexpr int lc = 3 * D * D + 2 * D;
  static constexpr int SIZE = 3 * D * D + 2 * D + 2;
};

// Filtering moments entering a tree node; flag != 0 marks the identity prefix.
template <int D>
struct PrefLayout {
  static constexpr int P = 0, m = D * D, flag = D * D + D;
  static constexpr int SIZE = D * D + D + 2;
};

// Sampling path element (E, U).
template <int D>
struct SampLayout {
  static constexpr int E = 0, U = D * D;
  static constexpr int SIZE = D * D + D;
};

struct StepArgs {
  const double* y;
  const double* x;
  const double* xi_u;
  double delta;
  int order;
  double *u, *om, *Om, *om2, *Om2;  // [N*d]
  double* xs;                       // [N*d]
  double *ell, *ell2;               // [N]
  double *part_lh_x, *part_lh_xs, *part_terms;
  double *g_G, *g_Ht, *g_Rinv, *g_Omd, *g_Omd_inv, *g_scal;
  int* status;
  int* accept_flag;
};

// pseudo-observation model of a filter: diagonal Omega_t, dense constant
// Omega, or a general y_t = H x_t + N(0, R)
enum { OBS_DIAG = 0, OBS_DENSE = 1, OBS_GH = 2 };

struct FilterArgs {
  int B;
  const double* om;
  const double* Om;   // diagonal Omega [N*d]
  const double* Omd;  // dense constant Omega [d*d] or nullptr
  double* elem;       // block elements, level 0 of the tree
  const double* pre;  // prefixes entering each block (PrefLayout), or
  const double* pre_elem;  // inclusive scan elements: block k starts from
                           // element k-1 read as a moment pair (b, C)
  double *mf, *Pf;    // [N*ldm], [N*ldm*ldm] or nullptr
  int ldm;            // leading dimension of mf/Pf (D inside the step, d for callers)
  double* ell;        // [N]
  int* status;
  int fail_bit;
  // general observation model y_t = H x_t + N(0, R) (Ho != nullptr; D <= 32)
  const double* yo;   // [N*dyo]
  const double* Ho;   // [dyo*d]
  const double* Ro;   // [dyo*dyo]
  int dyo;
  // per-step dynamics F_t [N*d*d], b_t [N*d] (transition into step t), or
  // nullptr for the model's F, b
  const double *Ft, *bt;
  // re-scan outputs kept for steps that reuse the covariances (diagonal Omega
  // path; nullptr = not kept): S_t^{-1} [N*D*D] transposed, log det S_t [N]
  double *Sinv, *ldS;
};

struct TreeArgs {
  const double* src;
  double* dst;
  int n_src, n_dst;
  const double* pre_src;
  double* pre_dst;
  int* status;
  int fail_bit;
};

// One level of the Hillis-Steele scan over block elements:
// dst[k] = src[k - s] (x) src[k] for k >= s, dst[k] = src[k] otherwise.
struct HsArgs {
  const double* src;
  double* dst;
  int n, s;
  int* status;
  int fail_bit;
};

struct SampArgs {
  int B;
  const double *mf, *Pf, *xi_x;
  int ldm;           // leading dimension of mf/Pf
  double *E, *U;     // [N*D*D], [N*D]
  double* agg;       // block aggregates, level 0
  const double* xin; // x* entering each block from the right, level 0
  double* xs;        // [N*d]
  int* status;
  const double *Ft, *bt;  // per-step dynamics as in FilterArgs, or nullptr
  // kept for reuse (transposed, [N*D*D]), or nullptr: chol(L_t) and E_t
  double *Lc, *Et;
};

// Proposals whose auxiliary model has covariances formed earlier (first
// order: Omega_t = delta/2 I for every path; second order: the same x as the
// proposal that formed them), with the matrices kept.  Every kept matrix is
// stored transposed (At[j*D + i] = A_ij), so that a matrix-vector product
// reads it in coalesced columns.
struct FixedArgs {
  int B;                   // scan block (steps)
  const double* om;        // [N*d] pseudo-observations of this proposal
  const double* Om;        // [N*d] diagonal Omega_t the matrices were formed with
  const double *Sinv, *ldS;  // S_t^{-1} [N*D*D], log det S_t [N]
  const double *Et, *Lc;   // sampler E_t, chol(L_t) [N*D*D]
  double* Phi;             // [N*D*D] Phi_{N-1-s} at s (set-up, for the tree products)
  double* Fp;              // [D*D] F, padded (set-up)
  double* mf;              // [N*D] filtering means (time order)
  double* ell;             // [N] log-likelihood terms
  const double* xi_x;      // [N*d] path normals
  double *W, *G;           // [N*D] sampler scan: w_t = m^f_t + chol(L_t) xi_t, g_t = F m^f_t + b
  double* xs;              // [N*d] sampled path
  const int* setup_status; // failures of the one-off matrices, copied into status
  int* status;
};

// Node products of a kept scan (set-up): elements Mt [N*D*D] in blocks of B
// steps, then per tree level l the products of node pairs, Tm[l]
// [n_lvl[l]*D*D]; a node maps the state after its range to its first state;
// all transposed.
struct VScanArgs {
  int N, B;
  const double* Mt;
  Gate gate;
};

// Up to kVTreeSpan consecutive tree levels lo .. lo + R in one launch; one
// workgroup per node of level lo + R.
constexpr int kVTreeSpan = 3;
struct VTreeSpan {
  const double* Tm[kVTreeSpan];  // node matrices of levels lo .. lo+R-1 (transposed)
  double* U[kVTreeSpan + 1];     // vector parts of levels lo .. lo+R
  double* X[kVTreeSpan + 1];     // states entering the nodes of levels lo .. lo+R
  int n[kVTreeSpan + 1];         // node counts of levels lo .. lo+R
  int R;
  Gate gate;
};

// Extended linearisation of nonlinear dynamics (one wave per time step):
// F_t = J(a_{t-1}), b_t = f(a_{t-1}) - F_t a_{t-1} around the path `a`; with
// `z` (the other path) also the per-step MH terms of the dynamics mismatch.
struct DynArgs {
  const double* a;     // [N*d] linearisation point
  const double* z;     // [N*d] the other path, or nullptr
  double *Ft, *bt;     // [N*d*d], [N*d]
  const double* Qinv;  // [d*d]
  double* part;        // [n_part] partial sums of the mismatch terms
};

// Divide-and-conquer sampler: filtering moments in, path out; tree storage in
// the workspace (D-padded), leaves by t, nodes and bridges by midpoint.
struct DncArgs {
  int T;                       // N - 1
  const double *mf, *Pf;       // [N*ldm], [N*ldm*ldm]
  int ldm;
  const double* xi;            // [N*d]
  double* x;                   // [N*d]
  const double *Ft, *bt;       // per-step dynamics or nullptr
  double *Elf, *glf, *Llf;     // leaves [t, t+1]
  double *Eno, *gno, *Lno;     // node elements [k, m]
  double *Gb, *Gam, *wb, *Vc;  // bridges G, Gamma, w, chol(V)
  int* status;
};

// Auxiliary LGSSM of a factorising prior: dx scalar models, one per
// coordinate.  The model's P0, F and Q hold diagonals [d].
struct FactArgs {
  const double *om, *Om;  // [N*d] pseudo-observations and their variances
  const double* xi_x;     // [N*d] path normals; nullptr = filter only
  double* xs;             // [N*d] sampled path
  double *mf, *Pf;        // [d*N] filtering moments, coordinate-major (needed with xi_x)
  double* lz;             // [d] log marginal likelihood per coordinate
  int* status;
  int fail_bit;
};

struct FinalArgs {
  int n_ell;  // entries of ell/ell2 summed into log Z (0 = N)
  const double* lz_rev;  // log Z of the reverse proposal as one value, or nullptr (sum ell2)
  const double* part_dyn;  // dynamics mismatch partial sums (n_part_dyn), or nullptr
  int n_part_dyn;
  const double* unif;
  double* log_ratio;
  int* accepted;
  double* logZ_fwd;
  double* logZ_rev;
  int* status_out;
  int* status_next;  // the other status word, cleared for the next step (one chain)
  int n_part_fwd, n_part_rev;
};

// (E, g, L) suffix scan (App. A eq. EgL_comb): elements E [N*D*D], g [N*D]
// (nullable), L [N*D*D]; block aggregates `agg` (level 0); suffix states
// entering each block `state` (level 0); outputs L~ (and g~) per step.
struct EglArgs {
  int N, B;
  const double *E, *g, *L;
  double* agg;
  const double* state;
  double* outL;  // [N*ldo*ldo]
  double* outg;  // [N*ldo] or nullptr
  int ldo, dout;
};

struct EglTree {
  const double* src;
  double* dst;
  int n_src, n_dst;
  const double* pre_src;
  double* pre_dst;
};

struct SmoothArgs {
  const double *mf, *Pf;
  int ldm;
  double *E, *g, *L;  // [N*D*D], [N*D], [N*D*D]
  int* status;
};

// Linear-Gaussian model with theta = (F, log diag Q, H, log diag R).
struct LgArgs {
  int dx, dy, B;
  const double *logq, *logr, *H, *y;
  double *Q, *R;          // dense diagonal matrices built from theta (user dims)
  const double *mf, *Pf;  // forward filtering moments (checkpoint, stride D)
  double *E, *U, *Cm, *mbar, *Pbar, *part;
  double *dF, *dlogq, *dH, *dlogr;
  int* status;
};

// ---------------------------------------------------------------------------
// Batched chains: per-chain descriptors resident in device memory and work
// tables of (chain, item) pairs walked by persistent kernels.
// ---------------------------------------------------------------------------
constexpr int kMaxLv = 24;
// batched chains with d <= kLaneMaxD run their filter fold and re-scan and the
// sampler's element build, block fold and final pass one lane per item
// (akf_lane.hip)
constexpr int kLaneMaxD = 4;

struct ChainDev {
  KModel M;
  StepArgs A;          // xi_u is set per step from xi_base
  FilterArgs Ff, Fr;   // forward (at x) and reverse (at x*) filters
  SampArgs S;          // xi_x is set per step
  FinalArgs Fin;       // unif and outputs are set per step
  int L;               // tree levels of this chain
  int n_part;          // partial-sum blocks of the linearisation
  TreeArgs fup[kMaxLv], fdown[kMaxLv], sup[kMaxLv], sdown[kMaxLv];
  double* root_flag;
  double* root_xin;
  const double* xi_base;  // [n_steps, 2, N, d]
  int64_t xi_stride;      // 2 N d
  const double* unif_base;
  double *lr_base, *lzf_base, *lzr_base;
  int *acc_base, *st_base;
  double* x;              // chain state, updated in place
};

struct Item {
  int c, i;
};

struct BatchLaunch {
  const ChainDev* cd;
  const Item* items;
  int n_items;
  int grid;
};

// Kernel families for the timing hook (include/akf.h, akf_timing_enable).
enum {
  FAM_FILTER_FOLD = 0, FAM_FILTER_UP = 1, FAM_FILTER_DOWN = 2, FAM_FILTER_FINAL = 3,
  FAM_SAMP_BUILD = 4, FAM_SAMP_FOLD = 5, FAM_SAMP_UP = 6, FAM_SAMP_DOWN = 7, FAM_SAMP_FINAL = 8,
  FAM_FACT = 9, FAM_LIN = 10, FAM_DNC = 11, FAM_FIXED_MEAN_FOLD = 12, FAM_FIXED_SAMP_FOLD = 13,
  FAM_ADJ_GRAD = 14, FAM_ADJ_BUILD = 15,
  FAM_BATCH_FOLD16 = 16, FAM_BATCH_FOLD32 = 17, FAM_BATCH_FOLD64 = 18,
  FAM_BATCH_SBUILD16 = 19, FAM_BATCH_SBUILD32 = 20, FAM_BATCH_SBUILD64 = 21,
  FAM_MH = 22,
  FAM_COUNT = 23
};
// Called by the launchers before (begin = 1) and after (begin = 0) each launch.
void timing_mark(int family, int begin, hipStream_t st);

hipError_t launch_filter_scan_any(int D, const KModel& M, FilterArgs P, const HsArgs* lv,
                                  int n_levels, hipStream_t st);
hipError_t launch_filter_any(int D, const KModel& M, FilterArgs P, TreeArgs* up, TreeArgs* down,
                             int n_levels, hipStream_t st);
hipError_t launch_filter_logz_any(int D, const KModel& M, FilterArgs P, TreeArgs* up, int n_levels,
                                  hipStream_t st);
hipError_t launch_sampler_any(int D, const KModel& M, SampArgs S, TreeArgs* up, TreeArgs* down,
                              int n_levels, hipStream_t st);
hipError_t launch_lin(const KModel& M, StepArgs A, int rev, int* n_part, hipStream_t st);
hipError_t launch_reuse_gate(const int* accept, const int* status, int* gate, hipStream_t st);
hipError_t launch_step_init(int* status, double* root_flag, double* root_xin, int D,
                            hipStream_t st);
hipError_t launch_finalize(const KModel& M, StepArgs A, FinalArgs F, const double* x,
                           double* x_out, hipStream_t st);
hipError_t set_lds_limits_all();
hipError_t launch_samp_scan_any(int D, const KModel& M, SampArgs S, TreeArgs* up, TreeArgs* down,
                                int n_levels, hipStream_t st);
hipError_t launch_egl_scan_any(int D, EglArgs A, EglTree* up, EglTree* down, int n_levels,
                               hipStream_t st);
hipError_t launch_smooth_build_any(int D, const KModel& M, SmoothArgs S, hipStream_t st);
hipError_t launch_lgssm_prep(LgArgs G, hipStream_t st);
hipError_t launch_sum(const double* a, int n, double* out, const int* status, hipStream_t st);
hipError_t launch_adj_build_any(int D, const KModel& M, LgArgs G, hipStream_t st);
hipError_t launch_adj_G_any(int D, LgArgs G, int N, hipStream_t st);
hipError_t launch_adj_finish_any(int D, const KModel& M, LgArgs G, int nblk, const double* ll_bar,
                                 hipStream_t st);
hipError_t launch_zero(double* p, int64_t n, hipStream_t st);
hipError_t launch_fact_scan(const KModel& M, FactArgs P, hipStream_t st);
hipError_t launch_fixed_phi_any(int D, const KModel& M, FixedArgs A, hipStream_t st);
// matrix parts of a kept scan (set-up): level 0 from the elements, then L levels
hipError_t launch_vtree_mats_any(int D, const VScanArgs& V, double* const* Tm, const int* n_lvl,
                                 int L, hipStream_t st);
// One proposal's filtering means and log-likelihood terms (which = 0), or its
// sampled path from the kept sampler matrices (which = 1): block fold, the
// kept tree's vector parts, block final.  Tm: that scan's node products.
hipError_t launch_fixed_scan_any(int D, int which, const KModel& M, FixedArgs A,
                                 double* const* Tm, double* const* Uagg, double* const* xin,
                                 const int* n_lvl, int L, hipStream_t st);
hipError_t launch_qinv(const KModel& M, double* Qinv, hipStream_t st);
hipError_t launch_dnc_any(int D, const KModel& M, DncArgs A, hipStream_t st);
int dnc_depth(int T);
hipError_t launch_dyn_lin(const KModel& M, DynArgs A, int* n_part, hipStream_t st);

// Batched launches for one D class.  `step` is the device step counter.
enum BatchPhase {
  BP_INIT = 0, BP_LIN_FWD, BP_LIN_REV, BP_FOLD, BP_UP, BP_DOWN, BP_FINAL, BP_SBUILD, BP_SFOLD,
  BP_SUP, BP_SDOWN, BP_SFINAL, BP_FINALIZE, BP_SELECT,
  BP_SBUILD1,  // the sampler build with one team per SIMD (a layout the autotuner may pick)
  // one lane per item for chains with d <= 4 in the 16-wide class (akf_lane.hip)
  BP_FOLD_LANE, BP_FINAL_LANE, BP_SBUILD_LANE, BP_SFOLD_LANE, BP_SFINAL_LANE
};
hipError_t launch_batch_phase(int D, int phase, BatchLaunch L, int level, int rev,
                              const int* step, hipStream_t st);
hipError_t launch_step_advance(int* step, int reset, hipStream_t st);
size_t batch_lds_bytes(int D, int phase);
// Queries the resident-grid cap of every team phase at width D (kept per kernel).
void batch_caps(int D);
hipError_t launch_lane_phase(int phase, BatchLaunch L, int rev, const int* step, hipStream_t st);

}  // namespace akf
