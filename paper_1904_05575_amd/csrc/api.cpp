// C ABI of the BSE library: argument checks, workspace sizing, dispatch.
#include <math.h>

#include "bse_internal.h"
#include "timing.h"

namespace {

bool desc_ok(const bse_desc* d) {
  if (!d) return false;
  if (d->nk <= 0 || d->nv <= 0 || d->nc <= 0 || d->ng <= 0) return false;
  const int64_t n = (int64_t)d->nk * d->nv * d->nc;
  if (n > (1LL << 30) || d->nk > 46340) return false;
  if (d->ld < n) return false;
  if (d->coupling != BSE_TDA && d->coupling != BSE_FULL) return false;
  if (d->type < BSE_SINGLET || d->type > BSE_IP) return false;
  if (d->prec != BSE_PREC_FP64 && d->prec != BSE_PREC_FP32 && d->prec != BSE_PREC_BF16X3)
    return false;
  if (d->split_terms != 0 && d->split_terms != 3 && d->split_terms != 6) return false;
  if (!isfinite(d->kappa) || !isfinite(d->scissor)) return false;
  return true;
}

}  // namespace

extern "C" {

size_t bse_workspace_size(const bse_desc* desc, int32_t stage) {
  if (!desc_ok(desc)) return 0;
  if (stage == BSE_STAGE_BUILD) return build_workspace_fp64(desc);
  if (stage == BSE_STAGE_SOLVE) return solve_workspace(desc);
  return 0;
}

bse_status bse_build(const bse_desc* d, const bse_inputs* in, void* H0, void* H1, void* ws,
                     size_t ws_bytes, int32_t* info, hipStream_t stream) {
  launch_failure_reset();
  if (!desc_ok(d) || !in || !H0 || !info || !ws) return BSE_ERR_ARG;
  const bool full = d->coupling == BSE_FULL;
  if (!in->eps_v || !in->eps_c || !in->Mcv || !in->Mvv || (!in->Mcc && !in->mcc_env) ||
      !in->W || !in->vbar || !in->qmap)
    return BSE_ERR_ARG;
  if (full && (!in->Ncv || !in->Nvc || !in->qramap || !H1)) return BSE_ERR_ARG;
  if (in->nq <= 0 || in->nq > kMaxQ) return BSE_ERR_ARG;
  // the W split holds nk slices (2 nk for the full BSE)
  if (d->prec != BSE_PREC_FP64 && in->nq > (full ? 2 : 1) * d->nk) return BSE_ERR_ARG;
  if (ws_bytes < build_workspace_fp64(d)) return BSE_ERR_WORKSPACE;
  return build_fp64(d, in, H0, H1, ws, info, stream);
}

bse_status bse_solve(const bse_desc* d, void* H0, void* H1, double* E, void* XpY, void* XmY,
                     int64_t ldx, const void* probe, double* osc, void* ws, size_t ws_bytes,
                     int32_t* info, hipStream_t stream) {
  launch_failure_reset();
  if (!desc_ok(d) || !H0 || !E || !info || !ws) return BSE_ERR_ARG;
  const int64_t n = (int64_t)d->nk * d->nv * d->nc;
  if (d->coupling == BSE_FULL && !H1) return BSE_ERR_ARG;
  if (XpY && ldx < n) return BSE_ERR_ARG;
  if (XmY && (!XpY || XmY == XpY)) return BSE_ERR_ARG;  // X-Y comes with X+Y, in its own buffer
  if ((probe == nullptr) != (osc == nullptr)) return BSE_ERR_ARG;
  if (!XpY && !probe) return BSE_ERR_ARG;  // nothing but eigenvalues: pass a probe or XpY
  if (ws_bytes < solve_workspace(d)) return BSE_ERR_WORKSPACE;
  return solve_run(d, H0, H1, E, XpY, XmY, ldx, probe, osc, ws, info, stream);
}

bse_status bse_oscillator(int64_t n, const void* XpY, int64_t ldx, const void* probe, double* osc,
                          hipStream_t stream) {
  launch_failure_reset();
  if (n <= 0 || !XpY || !probe || !osc || ldx < n) return BSE_ERR_ARG;
  return launch_oscillator(n, (const double2*)XpY, ldx, (const double2*)probe, osc, stream) ==
                 hipSuccess
             ? BSE_OK
             : BSE_ERR_HIP;
}

bse_status bse_spectrum(int64_t n, const double* E, const double* osc, double pref, double eta,
                        int64_t nw, const double* omega, void* eps, hipStream_t stream) {
  launch_failure_reset();
  if (n <= 0 || nw <= 0 || !E || !osc || !omega || !eps) return BSE_ERR_ARG;
  if (!isfinite(pref) || !(eta > 0.0) || !isfinite(eta)) return BSE_ERR_ARG;
  return launch_spectrum(n, E, osc, pref, eta, nw, omega, (double2*)eps, stream) == hipSuccess
             ? BSE_OK
             : BSE_ERR_HIP;
}

bse_status bse_transitions(int64_t n, const void* XpY, int64_t ldx, int32_t nprobe,
                           const void* probe, int64_t ldp, void* t, int64_t ldt,
                           hipStream_t stream) {
  launch_failure_reset();
  if (n <= 0 || nprobe < 1 || nprobe > 4 || !XpY || !probe || !t) return BSE_ERR_ARG;
  if (ldx < n || ldp < n || ldt < n) return BSE_ERR_ARG;
  return launch_transitions(n, (const double2*)XpY, ldx, nprobe, (const double2*)probe, ldp,
                            (double2*)t, ldt, stream) == hipSuccess
             ? BSE_OK
             : BSE_ERR_HIP;
}

bse_status bse_dielectric_tensor(int64_t n, const double* E, int32_t nd, const void* t,
                                 int64_t ldt, double pref, double eta, int64_t nw,
                                 const double* omega, void* eps, hipStream_t stream) {
  launch_failure_reset();
  if (n <= 0 || nw <= 0 || nd < 1 || nd > 3 || !E || !t || !omega || !eps) return BSE_ERR_ARG;
  if (ldt < n || !isfinite(pref) || !(eta > 0.0) || !isfinite(eta)) return BSE_ERR_ARG;
  return launch_dielectric_tensor(n, E, nd, (const double2*)t, ldt, pref, eta, nw, omega,
                                  (double2*)eps, stream) == hipSuccess
             ? BSE_OK
             : BSE_ERR_HIP;
}

bse_status bse_loss(int64_t nw, const void* eps, int64_t inc, double vinv, double* loss,
                    double* sqw, hipStream_t stream) {
  launch_failure_reset();
  if (nw <= 0 || inc < 1 || !eps || !loss) return BSE_ERR_ARG;
  if (sqw && (!isfinite(vinv) || !(vinv > 0.0))) return BSE_ERR_ARG;
  return launch_loss(nw, (const double2*)eps, inc, vinv, loss, sqw, stream) == hipSuccess
             ? BSE_OK
             : BSE_ERR_HIP;
}

size_t bse_screening_workspace_size(const bse_screen_desc* d) {
  return screening_desc_ok(d) ? screening_workspace(d) : 0;
}

bse_status bse_screening(const bse_screen_desc* d, const double* eps_v, const double* eps_c,
                         const int32_t* kqmap, const void* Svc, const void* Scv,
                         const double* vsqrt, void* W, void* ws, size_t ws_bytes, int32_t* info,
                         hipStream_t stream) {
  launch_failure_reset();
  if (!screening_desc_ok(d)) return BSE_ERR_ARG;
  if (!eps_v || !eps_c || !kqmap || !Svc || !Scv || !vsqrt || !W || !ws || !info)
    return BSE_ERR_ARG;
  if (ws_bytes < screening_workspace(d)) return BSE_ERR_WORKSPACE;
  return screening_run(d, eps_v, eps_c, kqmap, (const double2*)Svc, (const double2*)Scv, vsqrt,
                       (double2*)W, ws, info, stream);
}

const char* bse_status_string(bse_status s) {
  switch (s) {
    case BSE_OK: return "ok";
    case BSE_ERR_ARG: return "invalid argument";
    case BSE_ERR_WORKSPACE: return "workspace too small";
    case BSE_ERR_HIP: {
      const char* m = launch_failure();
      return m ? m : "HIP launch failed";
    }
  }
  return "unknown status";
}

}  // extern "C"
