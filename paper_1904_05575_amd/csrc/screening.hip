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

// Upper triangle of Xt[q] = sum over both pair sets of w_t conj(M_t) M_t^T for
// N_G <= 16 NT, one block per q: the rows of q stream once through LDS (16
// rows per slice, the next slice prefetched into registers, one barrier per
// slice) and every wavefront accumulates its share of the NT(NT+1)/2 upper
// 16 x 16 output tiles on MFMA (the A and B operands are the same rows, A
// conjugated and weighted).  Each pair element is read from HBM once.
template <int NT>
__global__ __launch_bounds__(256) void k_screen_chi(const double2* __restrict__ S1,
                                                    const double2* __restrict__ S2,
                                                    const double* __restrict__ w1,
                                                    const double* __restrict__ w2, int64_t k1,
                                                    int ng, double2* __restrict__ W,
                                                    const int32_t* info) {
  constexpr int NP = NT * 16, PITCH = NP + 2, RS = 16;  // rows per slice
  constexpr int T = NT * (NT + 1) / 2, TW = (T + 3) / 4, EL = NT;  // EL = RS * NP / 256
  __shared__ double sre[2][RS][PITCH], sim[2][RS][PITCH];
  __shared__ double sw[2][RS];
  if (failed(info)) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int64_t q = blockIdx.x;
  // the columns beyond N_G stay zero in both buffers
  for (int e = tid; e < 2 * RS * NP; e += 256) {
    const int b = e / (RS * NP), r = (e / NP) % RS, c = e % NP;
    if (c >= ng) {
      sre[b][r][c] = 0.0;
      sim[b][r][c] = 0.0;
    }
  }
  // this wavefront's tiles: t = wid, wid + 4, ... in row-major order over I <= J
  int tI[TW], tJ[TW];
  bool tok[TW];
  d4 cr[TW], ci[TW];
#pragma unroll
  for (int u = 0; u < TW; ++u) {
    const int t = wid + 4 * u;
    tok[u] = t < T;
    int I = 0, rem = tok[u] ? t : 0;
    while (rem >= NT - I) {
      rem -= NT - I;
      ++I;
    }
    tI[u] = I;
    tJ[u] = I + rem;
    cr[u] = d4{0, 0, 0, 0};
    ci[u] = d4{0, 0, 0, 0};
  }
  const int slice_el = RS * ng;
  double2 pre[EL];
  double pw = 0.0;
  for (int set = 0; set < 2; ++set) {
    const double2* M = (set == 0 ? S1 : S2) + q * k1 * ng;
    const double* wq = (set == 0 ? w1 : w2) + q * k1;
    const int64_t ns = (k1 + RS - 1) / RS;
    auto fetch = [&](int64_t sl) {
      const int64_t row0 = sl * RS;
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int idx = tid + 256 * e;
        const int r = idx / ng;
        const bool ok = idx < slice_el && row0 + r < k1;
        pre[e] = ok ? M[row0 * ng + idx] : make_double2(0.0, 0.0);
      }
      pw = (tid < RS && row0 + tid < k1) ? wq[row0 + tid] : 0.0;
    };
    auto put = [&](int b) {
#pragma unroll
      for (int e = 0; e < EL; ++e) {
        const int idx = tid + 256 * e;
        if (idx < slice_el) {
          const int r = idx / ng, c = idx % ng;
          sre[b][r][c] = pre[e].x;
          sim[b][r][c] = pre[e].y;
        }
      }
      if (tid < RS) sw[b][tid] = pw;
    };
    fetch(0);
    int buf = 0;
    for (int64_t sl = 0; sl < ns; ++sl) {
      put(buf);
      __syncthreads();
      if (sl + 1 < ns) fetch(sl + 1);
#pragma unroll
      for (int ks = 0; ks < RS / 4; ++ks) {
        const int k = ks * 4 + (lane >> 4);
        const double wk = sw[buf][k];
#pragma unroll
        for (int u = 0; u < TW; ++u) {
          if (!tok[u]) continue;  // uniform in the wavefront
          const int ca = tI[u] * 16 + (lane & 15), cb = tJ[u] * 16 + (lane & 15);
          const double are = wk * sre[buf][k][ca], aim = -wk * sim[buf][k][ca];
          const double bre = sre[buf][k][cb], bim = sim[buf][k][cb];
          cr[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(are, bre, cr[u], 0, 0, 0);
          cr[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-aim, bim, cr[u], 0, 0, 0);
          ci[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(are, bim, ci[u], 0, 0, 0);
          ci[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(aim, bre, ci[u], 0, 0, 0);
        }
      }
      buf ^= 1;
    }
    __syncthreads();  // the next set's first put reuses buffer 0
  }
  double2* Wq = W + q * ng * ng;
#pragma unroll
  for (int u = 0; u < TW; ++u) {
    if (!tok[u]) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = tI[u] * 16 + (lane >> 4) + 4 * r, gj = tJ[u] * 16 + (lane & 15);
      if (gi < ng && gj < ng) Wq[(int64_t)gi * ng + gj] = make_double2(cr[u][r], ci[u][r]);
    }
  }
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

// The same inversion for N_G <= 128 with the matrix in registers.  Thread
// (ti, tj) of a 16 x 32 grid holds the elements (ti + 16 a, tj + 32 b),
// a < 8, b < 4, so a thread needs 8 entries of the pivot column and 4 of the
// pivot row per step.  Per pivot k the owners publish row k and column k in
// LDS and every thread updates its own elements: two barriers per pivot and
// no global traffic between the load and the final store.  The lower
// triangle is formed from the conjugate of the upper one when it is loaded.
constexpr int INV_NGMAX = 128, INV_TI = 16, INV_TJ = 32;
constexpr int INV_A = INV_NGMAX / INV_TI, INV_B = INV_NGMAX / INV_TJ;
__global__ __launch_bounds__(INV_TI * INV_TJ) void k_screen_invert_reg(
    double2* __restrict__ W, const double* __restrict__ vsqrt, int ng, int32_t* info) {
  __shared__ double2 col[INV_NGMAX], row[INV_NGMAX];
  __shared__ double s[INV_NGMAX];
  if (failed(info)) return;
  const int tid = threadIdx.x, ti = tid % INV_TI, tj = tid / INV_TI;
  const int64_t q = blockIdx.x;
  double2* A = W + q * ng * ng;
  for (int i = tid; i < ng; i += INV_TI * INV_TJ) s[i] = vsqrt[q * ng + i];
  __syncthreads();
  double2 a[INV_A][INV_B];
#pragma unroll
  for (int x = 0; x < INV_A; ++x)
#pragma unroll
    for (int y = 0; y < INV_B; ++y) {
      const int i = ti + INV_TI * x, j = tj + INV_TJ * y;
      a[x][y] = make_double2(0.0, 0.0);
      if (i < ng && j < ng) {
        const double2 v = i <= j ? A[(int64_t)i * ng + j] : cconj(A[(int64_t)j * ng + i]);
        a[x][y] = make_double2((i == j ? 1.0 : 0.0) + s[i] * v.x * s[j],
                               i == j ? 0.0 : s[i] * v.y * s[j]);
      }
    }
  for (int k = 0; k < ng; ++k) {
#pragma unroll
    for (int x = 0; x < INV_A; ++x)
#pragma unroll
      for (int y = 0; y < INV_B; ++y) {
        const int i = ti + INV_TI * x, j = tj + INV_TJ * y;
        if (j == k && i < ng) col[i] = a[x][y];
        if (i == k && j < ng) row[j] = a[x][y];
      }
    __syncthreads();
    const double2 d = row[k];
    if (!(d.x > 0.0) || !isfinite(d.x)) {
      if (tid == 0) set_info(info, -6);
      return;  // uniform: every thread reads the same pivot
    }
    const double dn = 1.0 / cabs2(d);
    const double2 rd = make_double2(d.x * dn, -d.y * dn);  // 1 / d
    double2 cd[INV_A], rw[INV_B];
#pragma unroll
    for (int x = 0; x < INV_A; ++x) cd[x] = cmul(col[min(ti + INV_TI * x, INV_NGMAX - 1)], rd);
#pragma unroll
    for (int y = 0; y < INV_B; ++y) rw[y] = row[min(tj + INV_TJ * y, INV_NGMAX - 1)];
#pragma unroll
    for (int x = 0; x < INV_A; ++x)
#pragma unroll
      for (int y = 0; y < INV_B; ++y) {
        const int i = ti + INV_TI * x, j = tj + INV_TJ * y;
        if (i >= ng || j >= ng) continue;
        if (i == k && j == k)
          a[x][y] = make_double2(-rd.x, -rd.y);
        else if (i == k || j == k)
          a[x][y] = cmul(a[x][y], rd);
        else
          a[x][y] = csub(a[x][y], cmul(cd[x], rw[y]));
      }
    __syncthreads();  // col and row are rewritten for the next pivot
  }
#pragma unroll
  for (int x = 0; x < INV_A; ++x)
#pragma unroll
    for (int y = 0; y < INV_B; ++y) {
      const int i = ti + INV_TI * x, j = tj + INV_TJ * y;
      if (i < ng && j < ng)
        A[(int64_t)i * ng + j] = make_double2(-s[i] * a[x][y].x * s[j], -s[i] * a[x][y].y * s[j]);
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
  const dim3 g1((unsigned)nk), b1(256);
  switch (cdiv(ng, 16)) {  // one block per q streams its rows once (N_G <= 128)
    case 1: BSE_LAUNCH(k_screen_chi<1>, g1, b1, 0, s, Svc, Scv, w1, w2, k1, ng, W, info); break;
    case 2: BSE_LAUNCH(k_screen_chi<2>, g1, b1, 0, s, Svc, Scv, w1, w2, k1, ng, W, info); break;
    case 3: BSE_LAUNCH(k_screen_chi<3>, g1, b1, 0, s, Svc, Scv, w1, w2, k1, ng, W, info); break;
    case 4: BSE_LAUNCH(k_screen_chi<4>, g1, b1, 0, s, Svc, Scv, w1, w2, k1, ng, W, info); break;
    case 5: BSE_LAUNCH(k_screen_chi<5>, g1, b1, 0, s, Svc, Scv, w1, w2, k1, ng, W, info); break;
    case 6: BSE_LAUNCH(k_screen_chi<6>, g1, b1, 0, s, Svc, Scv, w1, w2, k1, ng, W, info); break;
    case 7: BSE_LAUNCH(k_screen_chi<7>, g1, b1, 0, s, Svc, Scv, w1, w2, k1, ng, W, info); break;
    case 8: BSE_LAUNCH(k_screen_chi<8>, g1, b1, 0, s, Svc, Scv, w1, w2, k1, ng, W, info); break;
    default: break;
  }
  if (ng <= 128) {
    BSE_LAUNCH(k_screen_invert_reg, dim3((unsigned)nk), dim3(INV_TI * INV_TJ), 0, s, W, vsqrt, ng,
               info);
    return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
  }
  // larger N_G: the batched GEMM, the tile edge that pads the output least
  // (64 unless 32 saves > 15 %)
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
