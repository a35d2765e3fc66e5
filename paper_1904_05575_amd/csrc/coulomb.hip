// The Coulomb potential of the exchange term without its macroscopic part
// (paper Sec. 4.2, eq. vbar_def) and the probe vector of the spectrum (Sec.
// 4.4, eq. osci) on the device: the last host-side arithmetic of a problem's
// inputs.
#include <cmath>

#include "bse_internal.h"
#include "common.h"
#include "timing.h"

namespace {

constexpr int CB_THREADS = 256;

// One block.  G_Q is the G nearest to Q (smallest |G - Q|^2, the lowest index
// among equals); q = Q - G_Q; vbar[G] = 4 pi / |G + q|^2 for G != G_Q and 0 at
// G_Q.  Cartesian G = gvec * (2 pi / alat), component sums in x, y, z order.
__global__ __launch_bounds__(CB_THREADS) void k_coulomb(int ng, const int32_t* __restrict__ gvec,
                                                        double scale, double qx, double qy,
                                                        double qz, double* __restrict__ vbar,
                                                        int32_t* __restrict__ gq_out) {
  __shared__ double bd[CB_THREADS];
  __shared__ int bi[CB_THREADS];
  __shared__ int gq_s;
  const int tid = threadIdx.x;
  double best = INFINITY;
  int ib = ng;
  for (int g = tid; g < ng; g += CB_THREADS) {
    const double dx = gvec[3 * g] * scale - qx, dy = gvec[3 * g + 1] * scale - qy,
                 dz = gvec[3 * g + 2] * scale - qz;
    const double d2 = dx * dx + dy * dy + dz * dz;
    if (d2 < best) {  // g increases: the first of equals stays
      best = d2;
      ib = g;
    }
  }
  bd[tid] = best;
  bi[tid] = ib;
  __syncthreads();
  for (int h = CB_THREADS / 2; h > 0; h >>= 1) {
    if (tid < h) {
      const double o = bd[tid + h];
      const int oi = bi[tid + h];
      if (o < bd[tid] || (o == bd[tid] && oi < bi[tid])) {
        bd[tid] = o;
        bi[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    gq_s = bi[0];
    *gq_out = bi[0];
  }
  __syncthreads();
  const int gq = gq_s;
  const double rx = qx - gvec[3 * gq] * scale, ry = qy - gvec[3 * gq + 1] * scale,
               rz = qz - gvec[3 * gq + 2] * scale;
  for (int g = tid; g < ng; g += CB_THREADS) {
    const double px = gvec[3 * g] * scale + rx, py = gvec[3 * g + 1] * scale + ry,
                 pz = gvec[3 * g + 2] * scale + rz;
    const double p2 = px * px + py * py + pz * pz;
    vbar[g] = g == gq ? 0.0 : 4.0 * M_PI / p2;
  }
}

// probe[a] = conj(Mcv[a][gq]) (eq. osci: the plane-wave element at G_Q).
__global__ __launch_bounds__(256) void k_probe(int64_t n, int ng, const double2* __restrict__ Mcv,
                                               const int32_t* __restrict__ gq,
                                               double2* __restrict__ probe) {
  const int64_t a = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (a >= n) return;
  const int g = *gq;
  probe[a] = cconj(Mcv[a * ng + g]);
}

}  // namespace

extern "C" {

bse_status bse_coulomb(int32_t ng, const int32_t* gvec, double alat, const double* Q,
                       double* vbar, int32_t* gq, hipStream_t stream) {
  launch_failure_reset();
  if (ng <= 0 || !gvec || !Q || !vbar || !gq || !(alat > 0.0) || !std::isfinite(alat))
    return BSE_ERR_ARG;
  if (!std::isfinite(Q[0]) || !std::isfinite(Q[1]) || !std::isfinite(Q[2])) return BSE_ERR_ARG;
  BSE_LAUNCH(k_coulomb, dim3(1), dim3(CB_THREADS), 0, stream, (int)ng, gvec, 2.0 * M_PI / alat,
             Q[0], Q[1], Q[2], vbar, gq);
  return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
}

bse_status bse_probe(int64_t n, int32_t ng, const void* Mcv, const int32_t* gq, void* probe,
                     hipStream_t stream) {
  launch_failure_reset();
  if (n <= 0 || ng <= 0 || !Mcv || !gq || !probe) return BSE_ERR_ARG;
  BSE_LAUNCH(k_probe, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, stream, n, (int)ng,
             (const double2*)Mcv, gq, (double2*)probe);
  return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
}

}  // extern "C"
