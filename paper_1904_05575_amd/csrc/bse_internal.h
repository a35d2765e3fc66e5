// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/bse.h"

enum {
  BSE_INFO_BAD_QMAP = -1,
  BSE_INFO_NONFINITE = -2,
  BSE_INFO_NOT_PD_PLUS = -3,
  BSE_INFO_NO_CONVERGE = -4,
};

// Largest number of W slices (momentum-transfer classes) of one problem.
constexpr int64_t kMaxQ = 8192;

// Carves aligned sub-buffers out of one workspace (or only sums their sizes).
struct WsLayout {
  char* base = nullptr;
  size_t total = 0;
  WsLayout() = default;
  explicit WsLayout(void* b) : base((char*)b) {}
  void* add(int64_t bytes) {
    total = (total + 255) & ~(size_t)255;
    void* p = base ? base + total : nullptr;
    total += (size_t)std::max<int64_t>(bytes, 0);
    return p;
  }
};

inline void bse_gamma(int type, double* gx, double* gc) {
  switch (type) {
    case BSE_SINGLET: *gx = 1.0; *gc = 1.0; break;
    case BSE_TRIPLET: *gx = 0.0; *gc = 1.0; break;
    case BSE_RPA: *gx = 1.0; *gc = 0.0; break;
    default: *gx = 0.0; *gc = 0.0; break;
  }
}

// assembly.hip
size_t build_workspace_fp64(const bse_desc* d);
bse_status build_fp64(const bse_desc* d, const bse_inputs* in, void* out0, void* out1, void* ws,
                      int32_t* info, hipStream_t s);

// stage1.hip: class-grouped T = conj(L) W(q) on the real view of the complex data
bool launch_stage1(const double2* left, int R, int ng, const double2* W, const int32_t* perm,
                   const int32_t* cls, int nq, int nk, double2* T, const int32_t* info,
                   hipStream_t s);

// direct.hip: both direct-term contractions in one pass, added into the
// outputs (false: shape not handled, nothing launched)
bool first_product_fits(int ng, int R);
bool launch_first_product(int shape, const double2* left, int R, int ng, int nk,
                          const double2* W, const int32_t* perm, const int32_t* cls, int nq,
                          double2* Tout, const int32_t* info, hipStream_t s);
bool launch_direct_onepass(int prec, const double2* left, const double2* right, int R, int N2,
                           int ng, int nk, int nv, int nc, const double2* W, const int32_t* perm,
                           const int32_t* cls, int nq, int ra, double coef, double2* out0,
                           double2* out1, int64_t ld, int32_t* tmap, const int32_t* info,
                           hipStream_t s);
bool launch_direct_fused(int prec, int variant, const double2* left, const double2* right, int R,
                         int N2, int ng, int nk, int nv, int nc, const double2* W,
                         const int32_t* perm, const int32_t* cls, int nq, int ra, double coef,
                         double2* out0, double2* out1, int64_t ld, double2* Tout,
                         const int32_t* info, hipStream_t s);

// gemm_lp.hip: reduced-precision products of the assembly
size_t split_w_bytes(int nq, int ng);
bool launch_split_w(int prec, const double2* W, int nq, int ng, void* Wsp, hipStream_t s);
bool launch_stage1_lp(int prec, int nterms, const double2* left, int R, int ng, const void* Wsp,
                      const int32_t* perm, const int32_t* cls, int nq, int nk, double2* T,
                      const int32_t* info, hipStream_t s);
bool launch_exchange_lp(int prec, int nterms, const double2* Mcv, int n, int ng,
                        const double* vbar, double alpha, double2* C, int64_t ld,
                        const int32_t* info, hipStream_t s);

// tune.cpp: tile choice for a call site and size (deflt when no entry applies)
int tune_choice(int site, int64_t size, int deflt);

// solve.hip
void launch_zero_ints(int32_t* p, int n, hipStream_t s);
size_t solve_workspace(const bse_desc* d);
// Stages of solve_run: before the Cholesky factorisation (counters, the
// copy of A+B), the factorisation, from it to the sweep (the squared form, the
// probe's projection), the Householder sweep, everything after it.
constexpr int SOLVE_PRE1 = 1, SOLVE_CHOL = 8, SOLVE_PRE2 = 16, SOLVE_SWEEP = 2, SOLVE_POST = 4;
constexpr int SOLVE_PRE = SOLVE_PRE1 | SOLVE_CHOL | SOLVE_PRE2;
constexpr int SOLVE_ALL = SOLVE_PRE | SOLVE_SWEEP | SOLVE_POST;
bse_status solve_run(const bse_desc* d, void* H0, void* H1, double* E, void* XpY, void* XmY,
                     int64_t ldx, const void* probe, double* osc, void* ws, int32_t* info,
                     hipStream_t s, int phase = SOLVE_ALL);
// Cholesky factorisation A - B = U^H U of several problems in step (the
// factorisation of the full solve): each problem's matrix (upper triangle,
// leading dimension ld, order n), its U11 staging (solve workspace) and status.
struct CholItem {
  double2* A;
  int64_t ld, n;
  double2* u11;
  int32_t* info;
};
constexpr int CHOL_GROUP_MAX = 16;
// Up to CHOL_GROUP_MAX problems whose tuned Cholesky GEMM tile is the same;
// each problem's values are those of its own factorisation in solve_run.
bool cholesky_batch(const CholItem* it, int np, hipStream_t s);
// The factorisation's arguments for problem d (full coupling) in workspace ws.
CholItem solve_chol_item(const bse_desc* d, void* H1, void* ws, int32_t* info);

// The sweep's arguments for problem d in workspace ws (as solve_run passes
// them; `project`: spectrum-only run with a probe).
struct TrdItem;
TrdItem solve_sweep_item(const bse_desc* d, void* H0, void* ws, bool project, int32_t* info);

// screening.hip
size_t screening_workspace(const bse_screen_desc* d);
bool screening_desc_ok(const bse_screen_desc* d);
bse_status screening_run(const bse_screen_desc* d, const double* eps_v, const double* eps_c,
                         const int32_t* kqmap, const double2* Svc, const double2* Scv,
                         const double* vsqrt, double2* W, void* ws, int32_t* info,
                         hipStream_t s);

// spectrum.hip
hipError_t launch_oscillator(int64_t n, const double2* XpY, int64_t ldx, const double2* probe,
                             double* osc, hipStream_t s);
hipError_t launch_spectrum(int64_t n, const double* E, const double* osc, double pref, double eta,
                           int64_t nw, const double* omega, double2* eps, hipStream_t s);
hipError_t launch_transitions(int64_t n, const double2* XpY, int64_t ldx, int nprobe,
                              const double2* probe, int64_t ldp, double2* t, int64_t ldt,
                              hipStream_t s);
hipError_t launch_dielectric_tensor(int64_t n, const double* E, int nd, const double2* t,
                                    int64_t ldt, double pref, double eta, int64_t nw,
                                    const double* omega, double2* eps, hipStream_t s);
hipError_t launch_loss(int64_t nw, const double2* eps, int64_t inc, double vinv, double* loss,
                       double* sqw, hipStream_t s);
