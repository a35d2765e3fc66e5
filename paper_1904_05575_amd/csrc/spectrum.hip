// Oscillator strengths and the Lorentzian eigen-sum of the macroscopic
// dielectric function (paper Sec. 4.4, eqs. chir and osci); the optical-limit
// transition coefficients and dielectric tensor (eqs. tlambdai, epsmij), the
// loss function and the dynamic structure factor (eq. Lofeps).
#include "bse_internal.h"
#include "common.h"
#include "timing.h"

namespace {

// osc[l] = |sum_a conj(XpY[a, l]) probe[a]|^2, one wavefront per column l.
__global__ __launch_bounds__(256) void k_oscillator(int64_t n, const double2* __restrict__ X,
                                                    int64_t ldx, const double2* __restrict__ p,
                                                    double* __restrict__ osc) {
  const int64_t l = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (l >= n) return;
  const double2* col = X + l * ldx;
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t a = lane; a < n; a += 64) acc = cadd(acc, cmulc(col[a], p[a]));
  acc = wave_sum2(acc);
  if (lane == 0) osc[l] = cabs2(acc);
}

// eps[j] = 1 - pref sum_l osc[l] [1/(w_j - E_l + i eta) - 1/(w_j + E_l + i eta)],
// one wavefront per frequency; fixed summation order.
__global__ __launch_bounds__(256) void k_spectrum(int64_t n, const double* __restrict__ E,
                                                  const double* __restrict__ osc, double pref,
                                                  double eta, int64_t nw,
                                                  const double* __restrict__ omega,
                                                  double2* __restrict__ eps) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= nw) return;
  const double w = omega[j], eta2 = eta * eta;
  double sr = 0.0, si = 0.0;
  for (int64_t l = lane; l < n; l += 64) {
    const double f = osc[l], e = E[l];
    const double x1 = w - e, x2 = w + e;
    const double i1 = 1.0 / (x1 * x1 + eta2), i2 = 1.0 / (x2 * x2 + eta2);
    // 1/(x + i eta) = (x - i eta) / (x^2 + eta^2)
    sr += f * (x1 * i1 - x2 * i2);
    si += f * (-eta * i1 + eta * i2);
  }
  sr = wave_sum(sr);
  si = wave_sum(si);
  if (lane == 0) eps[j] = make_double2(1.0 - pref * sr, -pref * si);
}


// t[l + i ldt] = -i sum_a conj(X[a, l]) p[a + i ldp] for TC consecutive
// columns l per block.  Thread tid takes rows tid, tid + 256, ...: per row it
// loads the NP probe values once and the row's element of each of the TC
// columns (256 consecutive elements of a column per block and step, so every
// column is read once, coalesced).  Sums: per wavefront, then the four
// wavefronts' partials in order (deterministic).
constexpr int TR_THREADS = 256, TR_COLS = 8;
template <int NP>
__global__ __launch_bounds__(TR_THREADS) void k_transitions(int64_t n,
                                                         const double2* __restrict__ X,
                                                         int64_t ldx,
                                                         const double2* __restrict__ p,
                                                         int64_t ldp, double2* __restrict__ t,
                                                         int64_t ldt) {
  __shared__ double2 part[TR_THREADS / 64][TR_COLS * NP];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t l0 = (int64_t)blockIdx.x * TR_COLS;
  const int ncol = (int)std::min<int64_t>(TR_COLS, n - l0);
  double2 acc[TR_COLS][NP];
#pragma unroll
  for (int c = 0; c < TR_COLS; ++c)
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[c][i] = make_double2(0.0, 0.0);
  for (int64_t a = tid; a < n; a += TR_THREADS) {
    double2 pv[NP], xv[TR_COLS];
#pragma unroll
    for (int i = 0; i < NP; ++i) pv[i] = p[a + i * ldp];
#pragma unroll
    for (int c = 0; c < TR_COLS; ++c)
      xv[c] = X[a + (l0 + std::min(c, ncol - 1)) * ldx];  // clamped column, masked below
#pragma unroll
    for (int c = 0; c < TR_COLS; ++c)
#pragma unroll
      for (int i = 0; i < NP; ++i) acc[c][i] = cadd(acc[c][i], cmulc(xv[c], pv[i]));
  }
#pragma unroll
  for (int c = 0; c < TR_COLS; ++c)
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const double2 v = wave_sum2(acc[c][i]);
      if (lane == 0) part[wid][c * NP + i] = v;
    }
  __syncthreads();
  if (tid < ncol * NP) {
    const int c = tid / NP, i = tid % NP;
    double2 v = part[0][tid];
#pragma unroll
    for (int w = 1; w < TR_THREADS / 64; ++w) v = cadd(v, part[w][tid]);
    t[(l0 + c) + i * ldt] = make_double2(v.y, -v.x);  // times -i
  }
}

// eps[(j ND + a) ND + b] = delta_ab - pref sum_l conj(t_la) t_lb g_l(w_j),
// g_l(w) = 1/(w - E_l + i eta) - 1/(w + E_l + i eta); one wavefront per
// frequency, fixed summation order.
template <int ND>
__global__ __launch_bounds__(256) void k_dielectric_tensor(int64_t n, const double* __restrict__ E,
                                                           const double2* __restrict__ t,
                                                           int64_t ldt, double pref, double eta,
                                                           int64_t nw,
                                                           const double* __restrict__ omega,
                                                           double2* __restrict__ eps) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= nw) return;
  const double w = omega[j], eta2 = eta * eta;
  double2 acc[ND][ND];
#pragma unroll
  for (int a = 0; a < ND; ++a)
#pragma unroll
    for (int b = 0; b < ND; ++b) acc[a][b] = make_double2(0.0, 0.0);
  for (int64_t l = lane; l < n; l += 64) {
    const double e = E[l];
    double2 tv[ND];
#pragma unroll
    for (int a = 0; a < ND; ++a) tv[a] = t[l + a * ldt];
    const double x1 = w - e, x2 = w + e;
    const double i1 = 1.0 / (x1 * x1 + eta2), i2 = 1.0 / (x2 * x2 + eta2);
    // 1/(x + i eta) = (x - i eta) / (x^2 + eta^2)
    const double2 g = make_double2(x1 * i1 - x2 * i2, -eta * i1 + eta * i2);
#pragma unroll
    for (int a = 0; a < ND; ++a)
#pragma unroll
      for (int b = 0; b < ND; ++b) acc[a][b] = cadd(acc[a][b], cmul(cmulc(tv[a], tv[b]), g));
  }
#pragma unroll
  for (int a = 0; a < ND; ++a)
#pragma unroll
    for (int b = 0; b < ND; ++b) {
      const double2 v = wave_sum2(acc[a][b]);
      if (lane == 0)
        eps[(j * ND + a) * ND + b] = make_double2((a == b ? 1.0 : 0.0) - pref * v.x, -pref * v.y);
    }
}

// loss[j] = -Im 1/eps[j inc] = Im eps / |eps|^2; sqw[j] = loss[j] vinv / pi.
__global__ __launch_bounds__(256) void k_loss(int64_t nw, const double2* __restrict__ eps,
                                              int64_t inc, double vinv,
                                              double* __restrict__ loss,
                                              double* __restrict__ sqw) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= nw) return;
  const double2 e = eps[j * inc];
  const double L = e.y / cabs2(e);
  loss[j] = L;
  if (sqw) sqw[j] = L * vinv * (1.0 / M_PI);
}

}  // namespace

hipError_t launch_oscillator(int64_t n, const double2* XpY, int64_t ldx, const double2* probe,
                             double* osc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  BSE_LAUNCH(k_oscillator, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, XpY, ldx,
                     probe, osc);
  return hipGetLastError();
}

hipError_t launch_spectrum(int64_t n, const double* E, const double* osc, double pref, double eta,
                           int64_t nw, const double* omega, double2* eps, hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  BSE_LAUNCH(k_spectrum, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, n, E, osc, pref,
                     eta, nw, omega, eps);
  return hipGetLastError();
}

hipError_t launch_transitions(int64_t n, const double2* XpY, int64_t ldx, int nprobe,
                              const double2* probe, int64_t ldp, double2* t, int64_t ldt,
                              hipStream_t s) {
  const dim3 grid((unsigned)cdiv(n, TR_COLS)), block(TR_THREADS);
  switch (nprobe) {
    case 1: BSE_LAUNCH(k_transitions<1>, grid, block, 0, s, n, XpY, ldx, probe, ldp, t, ldt); break;
    case 2: BSE_LAUNCH(k_transitions<2>, grid, block, 0, s, n, XpY, ldx, probe, ldp, t, ldt); break;
    case 3: BSE_LAUNCH(k_transitions<3>, grid, block, 0, s, n, XpY, ldx, probe, ldp, t, ldt); break;
    case 4: BSE_LAUNCH(k_transitions<4>, grid, block, 0, s, n, XpY, ldx, probe, ldp, t, ldt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dielectric_tensor(int64_t n, const double* E, int nd, const double2* t,
                                    int64_t ldt, double pref, double eta, int64_t nw,
                                    const double* omega, double2* eps, hipStream_t s) {
  const dim3 grid((unsigned)((nw + 3) / 4)), block(256);
  switch (nd) {
    case 1: BSE_LAUNCH(k_dielectric_tensor<1>, grid, block, 0, s, n, E, t, ldt, pref, eta, nw, omega, eps); break;
    case 2: BSE_LAUNCH(k_dielectric_tensor<2>, grid, block, 0, s, n, E, t, ldt, pref, eta, nw, omega, eps); break;
    case 3: BSE_LAUNCH(k_dielectric_tensor<3>, grid, block, 0, s, n, E, t, ldt, pref, eta, nw, omega, eps); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_loss(int64_t nw, const double2* eps, int64_t inc, double vinv, double* loss,
                       double* sqw, hipStream_t s) {
  BSE_LAUNCH(k_loss, dim3((unsigned)cdiv(nw, 256)), dim3(256), 0, s, nw, eps, inc, vinv, loss,
             sqw);
  return hipGetLastError();
}
