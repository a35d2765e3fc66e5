// Static RPA screening (paper Sec. 4.2, the RPA dielectric matrix and eq.
// wggq): for every q of the mesh
//   Xt[G, G'] = (1/V_c) sum_t |F_t| conj(M_t(G)) M_t(G')          (MFMA zgemm)
//   W = v^1/2 (I + v^1/2 Xt v^1/2)^-1 v^1/2                          (one block per q)
// with t over the pairs (occupied at k, unoccupied at k+q) and (unoccupied
// at k, occupied at k+q) and |F_t| = 1 / |e_j,k+q - e_i,k| in 1/Hartree.  The
// printed eps = I - v_G' X (X = -Xt) is brought to the Hermitian form
// I + v^1/2 Xt v^1/2 = v^1/2 eps v^-1/2, so that w = v eps^-1 =
// v^1/2 (v^1/2 eps v^-1/2)^-1 v^1/2.
#include "bse_internal.h"
#include "common.h"
#include "timing.h"
#include "zgemm.h"

namespace {

constexpr int SCR_MAX_NG = 512;

// w[q][r] = inv_vc * units / de for the rows r of both pair sets; de <= 0 (no
// gap) is an error (info = -5) and gives a zero weight.
__global__ __launch_bounds__(256) void k_screen_weights(int nk, int nv, int nc,
                                                        const double* __restrict__ eps_v,
                                                        const double* __restrict__ eps_c,
                                                        const int32_t* __restrict__ kqmap,
                                                        double scale, double* __restrict__ w1,
                                                        double* __restrict__ w2,
                                                        int32_t* info) {
  const int64_t k1 = (int64_t)nk * nv * nc;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= 2 * nk * k1) return;
  const int set = (int)(e / (nk * k1));      // 0: (v at k, c at k+q); 1: (c at k, v at k+q)
  const int64_t rem = e % (nk * k1);
  const int q = (int)(rem / k1);
  const int64_t r = rem % k1;
  const int k = (int)(r / (nv * nc)), b = (int)(r % (nv * nc));
  const int kq = kqmap[(int64_t)q * nk + k];
  double de;
  if (set == 0) {
    const int v = b / nc, c = b % nc;
    de = eps_c[(int64_t)kq * nc + c] - eps_v[(int64_t)k * nv + v];
  } else {
    const int c = b / nv, v = b % nv;
    de = eps_c[(int64_t)k * nc + c] - eps_v[(int64_t)kq * nv + v];
  }
  double wt = 0.0;
  if (de > 0.0 && isfinite(de))
    wt = scale / de;
  else
    set_info(info, -5);
  (set == 0 ? w1 : w2)[rem] = wt;
}

// In place on W[q] (row-major ng x ng, holding the upper triangle of the
// Hermitian Xt): A = I + s Xt s, mirrored onto the lower triangle, then the
// sweep operator over every pivot (Goodnight, The American Statistician 33,
// 1979), which leaves -A^-1, then W = -s (-A^-1) s = s A^-1 s.  One block per
// q; A is Hermitian positive definite, so no pivoting is needed; a pivot
// whose real part is not positive is an error (info = -6).
__global__ __launch_bounds__(256) void k_screen_invert(double2* __restrict__ W,
                                                       const double* __restrict__ vsqrt, int ng,
                                                       int32_t* info) {
  __shared__ double2 col[SCR_MAX_NG], row[SCR_MAX_NG];
  __shared__ double s[SCR_MAX_NG];
  if (failed(info)) return;
  const int tid = threadIdx.x;
  const int64_t q = blockIdx.x;
  double2* A = W + q * ng * ng;
  const int nn = ng * ng;
  for (int i = tid; i < ng; i += 256) s[i] = vsqrt[q * ng + i];
  __syncthreads();
  for (int e = tid; e < nn; e += 256) {
    const int i = e / ng, j = e % ng;
    if (i > j) continue;
    const double2 x = A[e];
    A[e] = make_double2((i == j ? 1.0 : 0.0) + s[i] * x.x * s[j], i == j ? 0.0 : s[i] * x.y * s[j]);
  }
  __syncthreads();
  for (int e = tid; e < nn; e += 256) {  // reads the upper triangle only
    const int i = e / ng, j = e % ng;
    if (i > j) A[e] = cconj(A[(int64_t)j * ng + i]);
  }
  __syncthreads();
  for (int k = 0; k < ng; ++k) {
    for (int i = tid; i < ng; i += 256) {
      col[i] = A[(int64_t)i * ng + k];
      row[i] = A[(int64_t)k * ng + i];
    }
    __syncthreads();
    const double2 d = row[k];
    if (!(d.x > 0.0) || !isfinite(d.x)) {
      if (tid == 0) set_info(info, -6);
      return;  // uniform: every thread reads the same pivot
    }
    const double dn = 1.0 / cabs2(d);
    const double2 rd = make_double2(d.x * dn, -d.y * dn);  // 1 / d
    for (int e = tid; e < nn; e += 256) {
      const int i = e / ng, j = e % ng;
      double2 a;
      if (i == k && j == k)
        a = make_double2(-rd.x, -rd.y);
      else if (i == k)
        a = cmul(row[j], rd);
      else if (j == k)
        a = cmul(col[i], rd);
      else
        a = csub(A[e], cmul(cmul(col[i], row[j]), rd));
      A[e] = a;
    }
    __syncthreads();
  }
  for (int e = tid; e < nn; e += 256) {
    const int i = e / ng, j = e % ng;
    const double2 a = A[e];
    A[e] = make_double2(-s[i] * a.x * s[j], -s[i] * a.y * s[j]);
  }
}

}  // namespace

size_t screening_workspace(const bse_screen_desc* d) {
  return (size_t)2 * d->nk * d->nk * d->nv * d->nc * sizeof(double);
}

bse_status screening_run(const bse_screen_desc* d, const double* eps_v, const double* eps_c,
                         const int32_t* kqmap, const double2* Svc, const double2* Scv,
                         const double* vsqrt, double2* W, void* ws, int32_t* info,
                         hipStream_t s) {
  const int nk = d->nk, ng = d->ng;
  const int64_t k1 = (int64_t)nk * d->nv * d->nc;
  double* w1 = (double*)ws;
  double* w2 = w1 + (int64_t)nk * k1;
  BSE_LAUNCH(k_screen_weights, dim3((unsigned)cdiv(2 * nk * k1, 256)), dim3(256), 0, s, nk,
             d->nv, d->nc, eps_v, eps_c, kqmap, d->inv_vc * d->units_per_hartree, w1, w2, info);
  // the tile edge that pads the ng x ng output least (64 unless 32 saves > 15 %)
  const int64_t p64 = (int64_t)cdiv(ng, 64) * 64, p32 = (int64_t)cdiv(ng, 32) * 32;
  const int tile = (p64 * p64 * 100 <= p32 * p32 * 115) ? 64 : 32;
  for (int set = 0; set < 2; ++set) {
    ZgemmParams g;  // upper triangle of Xt[q] (+)= M_q^H diag(w_q) M_q
    g.M = ng;
    g.N = ng;
    g.K = (int)k1;
    g.A = set == 0 ? Svc : Scv;
    g.a_rs = 1;
    g.a_cs = ng;
    g.a_bs = k1 * ng;
    g.conjA = 1;
    g.kscale = set == 0 ? w1 : w2;
    g.ks_bs = k1;
    g.B = g.A;
    g.b_rs = ng;
    g.b_cs = 1;
    g.b_bs = k1 * ng;
    g.C = W;
    g.c_rs = ng;
    g.c_cs = 1;
    g.c_bs = (int64_t)ng * ng;
    g.c_uplo = 1;
    g.alpha = make_double2(1.0, 0.0);
    g.beta = set == 0 ? 0.0 : 1.0;
    g.info = info;
    g.tag = "zgemm_screen_chi";
    g.tile = tile;
    if (zgemm(g, nk, s) != hipSuccess) return BSE_ERR_HIP;
  }
  BSE_LAUNCH(k_screen_invert, dim3((unsigned)nk), dim3(256), 0, s, W, vsqrt, ng, info);
  return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
}

bool screening_desc_ok(const bse_screen_desc* d) {
  if (!d || d->nk < 1 || d->nv < 1 || d->nc < 1 || d->ng < 1 || d->ng > SCR_MAX_NG) return false;
  if ((int64_t)2 * d->nk * d->nk * d->nv * d->nc >= (int64_t)1 << 31) return false;
  return std::isfinite(d->inv_vc) && d->inv_vc > 0.0 && std::isfinite(d->units_per_hartree) &&
         d->units_per_hartree > 0.0;
}
