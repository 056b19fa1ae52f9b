// akf_layout.h -- host-side helpers shared by the C ABI translation units:
// workspace layout, argument validation, error reporting and the launch
// sequences of the filter, sampler and (E, g, L) scans.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/akf.h"
#include "akf_internal.h"

namespace akf {

constexpr size_t kAlign = 256;  // workspace alignment (bytes)
constexpr int kMaxLevels = 32;

struct Layout {
  int N = 0, d = 0, dy = 0, D = 0, B = 0, nb = 0, L = 0;
  int n_lvl[kMaxLevels + 1] = {0};
  int n_part = 0;
  // byte offsets
  size_t u = 0, om = 0, Om = 0, om2 = 0, Om2 = 0, xs = 0, ell = 0, ell2 = 0;
  size_t plhx = 0, plhxs = 0, pterms = 0;
  size_t gG = 0, gHt = 0, gRinv = 0, gOmd = 0, gOmdinv = 0, gscal = 0;
  size_t elem[kMaxLevels + 1] = {0};
  size_t hs = 0;  // second buffer of the scan over block elements
  int L_hs = 0;   // levels of that scan: smallest L with 2^L >= nb
  size_t pre[kMaxLevels + 1] = {0};
  size_t mf = 0, Pf = 0, E = 0, U = 0;
  size_t sagg[kMaxLevels + 1] = {0};
  size_t xin[kMaxLevels + 1] = {0};
  size_t status = 0, accept = 0;
  // nonlinear dynamics: per-step F_t, b_t, Q^{-1}, mismatch partial sums
  size_t Ft = 0, bt = 0, Qinv = 0, pdyn = 0;
  int n_part_dyn = 0;
  // first-order runs: matrices formed once per call, transposed (S^{-1}, log
  // det S, the filtering-mean maps Phi in reversed time, chol(L), the
  // sampler's E, F padded), the node products of the two kept scans, and the
  // vector parts of those scans' tree nodes
  size_t Sinv = 0, ldS = 0, Phi = 0, Lc = 0, Et = 0, Fp = 0, Gs = 0;
  size_t tphi[kMaxLevels + 1] = {0};
  size_t te[kMaxLevels + 1] = {0};
  size_t vagg[kMaxLevels + 1] = {0};
  // divide-and-conquer sampler tree
  size_t Elf = 0, glf = 0, Llf = 0, Eno = 0, gno = 0, Lno = 0, Gb = 0, Gam = 0, wb = 0, Vc = 0;
  // (E, g, L) scan, smoother and adjoint
  size_t g = 0, Lm = 0, Pbar = 0, mbar = 0, part = 0, Qd = 0, Rd = 0, llv = 0;
  size_t eagg[kMaxLevels + 1] = {0};
  size_t estate[kMaxLevels + 1] = {0};
  size_t total = 0;
};

enum LayoutKind { LAYOUT_STEP = 0, LAYOUT_FILTER = 1, LAYOUT_SAMPLER = 2, LAYOUT_SMOOTH = 3,
                  LAYOUT_LGSSM = 4, LAYOUT_FACT = 5, LAYOUT_DNC = 6 };


template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

akf_status fail(akf_status s, const char* fmt, ...);
int pick_D(int d);
int auto_block(int N, int D, bool general_obs);
void make_layout(Layout& Lo, int N, int d, int dy, int block, int kind, bool dyn = false,
                 bool fixed = false);
// workspace layout of akf_lgssm_loglik / akf_lgssm_loglik_grad (filtering
// moments at Lo.mf, Lo.Pf with leading dimension Lo.D)
void lgssm_layout(Layout& Lo, const akf_lgssm* m, int block);
// allow_f32: the entry point computes in FP32 when the model asks for it
akf_status check_model(const akf_model* m, bool need_emission, bool allow_f32 = false);
akf_status check_order(const akf_model* m, int order);
akf_status check_linear(const akf_model* m, const char* what);
KModel to_kmodel(const akf_model* m);
akf_status prepare_device();
akf_status hip_check(hipError_t e, const char* what);
void fill_tree(const Layout& Lo, void* ws, size_t elem_size, const size_t* lvl_elem,
               const size_t* lvl_pre, int* status, int fail_bit, TreeArgs* up, TreeArgs* down);
double* root_flag(const Layout& Lo, void* ws);
akf_status run_filter(const Layout& Lo, const KModel& M, void* ws, const double* om,
                      const double* Om, const double* Omd, double* mf, double* Pf, int ldm,
                      double* ell, int* status, int fail_bit, hipStream_t st,
                      const double* yo = nullptr, const double* Ho = nullptr,
                      const double* Ro = nullptr, int dyo = 0, const double* Ft = nullptr,
                      const double* bt = nullptr, double* Sinv = nullptr,
                      double* ldS = nullptr);
akf_status run_filter_logz(const Layout& Lo, const KModel& M, void* ws, const double* om,
                           const double* Om, const double* Omd, int* status, int fail_bit,
                           hipStream_t st, const double* Ft, const double* bt,
                           const double** lz);
akf_status run_sampler(const Layout& Lo, const KModel& M, void* ws, const double* mf,
                       const double* Pf, int ldm, const double* xi_x, double* xs, int* status,
                       hipStream_t st, const double* Ft = nullptr, const double* bt = nullptr,
                       double* Lc = nullptr, double* Et = nullptr);
void fill_egl_tree(const Layout& Lo, void* ws, EglTree* up, EglTree* down);
akf_status run_egl(const Layout& Lo, void* ws, const double* g, double* outL, double* outg,
                   int ldo, int dout, hipStream_t st);
const char* last_error();

}  // namespace akf
