// Oscillator strengths and the Lorentzian eigen-sum of the macroscopic
// dielectric function (paper Sec. 4.4, eqs. chir and osci).
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
