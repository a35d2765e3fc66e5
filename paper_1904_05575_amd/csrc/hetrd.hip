// Householder reduction of a Hermitian matrix to real symmetric tridiagonal
// form, T = Q^H S Q with Q = H_0 H_1 ... H_{n-2}, H_c = I - tau_c v_c v_c^H
// (blocked, lower, panel width TRD_NB), for the eigenproblem of Sec. 4.3.
//
// Per column c (local index i of its panel) two kernels run:
//   k_trd_col   finishes reflector c-1 (its v, its W column, and H_{c-1}^H
//               applied to an optional probe vector), applies the panel's
//               earlier reflectors to column c and writes block partial sums
//               of |x|^2, V^H x, W^H x;
//   k_trd_hemv  every block reduces those partials (same order everywhere)
//               and forms reflector c, then y = S v_c - V (W^H v_c) -
//               W (V^H v_c), one wavefront per output row reading column r
//               of the trailing matrix, and block partials of y^H v_c.
// The next column kernel reduces the y^H v partials into alpha.  Kernel
// boundaries order every exchange between blocks: no atomics, no fences.
// After each panel, one MFMA GEMM applies S -= [V W][W V]^H to the trailing
// matrix (both triangles).  The panel's V and W live in two n x 2*TRD_NB
// buffers, VW = [V | W] and WV = [W | V], which make that update one product.
#include "bse_internal.h"
#include "common.h"
#include "solve_internal.h"
#include "timing.h"
#include "zgemm.h"

namespace {

constexpr int ROWS_A = 256;     // rows per block of the column kernel
constexpr int COL_THREADS = 1024;
constexpr int HEMV_WAVES = 8;   // output rows per hemv block
constexpr int VCHUNK = 2048;    // v staged in LDS in chunks of this many entries
constexpr int NVAL = 2 + 2 * TRD_NB;  // |x|^2, conj(x) y_probe, V^H x (i), W^H x (i)

// Deterministic block-wide complex sum (wavefront butterflies, then waves in
// order); every thread gets the result.  sh needs blockDim.x / 64 entries.
BSE_DEV double2 block_sum2(double2 v, double2* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum2(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  for (int k = 0; k < nw; ++k) s = cadd(s, sh[k]);
  return s;
}

// alpha of reflector c-1: -|tau|^2 / 2 times sum of the nb hemv partials of y^H v
BSE_DEV double2 reduce_alpha(const double2* __restrict__ partB, int nb, double2 tc, double2* sh) {
  double2 acc = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc = cadd(acc, partB[b]);
  const double2 s = block_sum2(acc, sh);
  const double t2 = cabs2(tc);
  return make_double2(-0.5 * t2 * s.x, -0.5 * t2 * s.y);
}

// x -= a conj(b)
BSE_DEV double2 sub_mulc(double2 x, double2 a, double2 b) {
  return make_double2(x.x - (a.x * b.x + a.y * b.y), x.y - (a.y * b.x - a.x * b.y));
}

__global__ __launch_bounds__(COL_THREADS) void k_trd_col(
    double2* __restrict__ M, int64_t ld, int n, double2* __restrict__ VW, double2* __restrict__ WV,
    int j0, int i, int has_new, double2* __restrict__ hs, const double2* __restrict__ ybuf,
    double2* __restrict__ partA, const double2* __restrict__ partB, double2* __restrict__ yp,
    const int32_t* info) {
  constexpr int QP = COL_THREADS / ROWS_A;        // threads sharing one row in step 1
  constexpr int RG = COL_THREADS / 64;            // row groups of step 2
  constexpr int RPG = ROWS_A / RG;                // rows per group
  __shared__ double2 xs[ROWS_A], vps[ROWS_A], wps[ROWS_A], x0s[ROWS_A];
  __shared__ double2 xpart[QP][ROWS_A];
  __shared__ double2 vcs[TRD_NB], wcs[TRD_NB];
  __shared__ double2 red[RG][2 * TRD_NB];
  __shared__ double2 red0[ROWS_A / 64][2];
  __shared__ double2 shb[COL_THREADS / 64];
  (void)info;  // no data-dependent indexing: runs even after an earlier failure
  const int c = j0 + i;
  const int64_t N = n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int rbase = c + blockIdx.x * ROWS_A;

  // ---- 0. finish reflector c-1 (row-mapped threads) and stage row c of the panel.
  // Every load of this step is issued before the reduction that forms alpha.
  const int r0 = rbase + tid;
  const bool row_thread = tid < ROWS_A, act = row_thread && r0 < n;
  double2 x0 = make_double2(0.0, 0.0), xv = x0, yb = x0, ypr = x0, vcl = x0, wcl = x0;
  if (act) {
    if (has_new) x0 = M[r0 + (int64_t)c * ld];
    if (yp) ypr = yp[r0];
    if (i > 0) {
      xv = M[r0 + (int64_t)(c - 1) * ld];
      yb = ybuf[r0];
    }
  }
  const int ipc = tid - ROWS_A;
  if (!row_thread && has_new && ipc < i - 1) {
    vcl = VW[c + (int64_t)ipc * N];
    wcl = VW[c + (int64_t)(TRD_NB + ipc) * N];
  }
  double2 tc = make_double2(0.0, 0.0), al = tc, scal_p = tc, pdot = tc, ybc = tc;
  if (i > 0) {
    tc = hs[HS_TAU];
    scal_p = hs[HS_SCAL];
    pdot = hs[HS_PDOT];
    ybc = ybuf[c];
    al = reduce_alpha(partB, cdiv(n - c, HEMV_WAVES), tc, shb);
  }
  if (row_thread) {
    const int r = r0;
    double2 vprev_r = make_double2(0.0, 0.0), wprev_r = make_double2(0.0, 0.0);
    if (i > 0 && act) {
      const int cp = c - 1;
      vprev_r = (r == c) ? make_double2(1.0, 0.0) : cmul(scal_p, xv);
      M[r + (int64_t)cp * ld] = vprev_r;
      wprev_r = cadd(cmul(tc, yb), cmul(al, vprev_r));
      VW[r + (int64_t)(i - 1) * N] = vprev_r;
      VW[r + (int64_t)(TRD_NB + i - 1) * N] = wprev_r;
      WV[r + (int64_t)(i - 1) * N] = wprev_r;
      WV[r + (int64_t)(TRD_NB + i - 1) * N] = vprev_r;
      if (yp) {
        // y <- H^H y = y - conj(tau) (v^H y) v
        const double2 f = cmulc(tc, pdot);
        ypr = csub(ypr, cmul(f, vprev_r));
        yp[r] = ypr;
      }
    }
    vps[tid] = vprev_r;
    wps[tid] = wprev_r;
    x0s[tid] = x0;
  } else if (has_new && ipc < i - 1) {
    vcs[ipc] = vcl;
    wcs[ipc] = wcl;
  }
  if (!has_new) return;
  __syncthreads();

  // ---- 1. apply the panel's earlier reflectors to column c: QP threads per row
  {
    const int rr = tid % ROWS_A, qq = tid / ROWS_A;
    const int r = rbase + rr;
    double2 acc = make_double2(0.0, 0.0);
    if (r < n) {
      constexpr int PER = (TRD_NB + QP - 1) / QP;
      double2 vr[PER], wr[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int ip = qq + u * QP;
        if (ip < i - 1) {
          vr[u] = VW[r + (int64_t)ip * N];
          wr[u] = VW[r + (int64_t)(TRD_NB + ip) * N];
        }
      }
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int ip = qq + u * QP;
        if (ip < i - 1) {
          acc = cadd(acc, cmulc(wcs[ip], vr[u]));   // v_ip[r] conj(w_ip[c])
          acc = cadd(acc, cmulc(vcs[ip], wr[u]));   // w_ip[r] conj(v_ip[c])
        }
      }
    }
    xpart[qq][rr] = acc;
  }
  __syncthreads();
  if (tid < ROWS_A) {
    const int r = rbase + tid;
    double2 x = make_double2(0.0, 0.0);
    bool tail = false;
    if (r < n) {
      x = x0s[tid];
#pragma unroll
      for (int q = 0; q < QP; ++q) x = csub(x, xpart[q][tid]);
      if (i > 0) {
        // reflector c-1: v[c] = 1, w[c] = tau y[c] + alpha
        const double2 wprev_c = cadd(cmul(tc, ybc), al);
        x = sub_mulc(x, vps[tid], wprev_c);
        x = csub(x, wps[tid]);
      }
      if (r == c) x.y = 0.0;
      M[r + (int64_t)c * ld] = x;
      tail = r >= c + 2;
    }
    xs[tid] = tail ? x : make_double2(0.0, 0.0);
    const double2 s0 = wave_sum2(make_double2(tail ? cabs2(x) : 0.0, 0.0));
    const double2 s1 = wave_sum2((tail && yp) ? cmulc(x, ypr) : make_double2(0.0, 0.0));
    if (lane == 0) {
      red0[wid][0] = s0;
      red0[wid][1] = s1;
    }
  }
  __syncthreads();

  // ---- 2. V^H x and W^H x over this block's rows: thread = (panel column, row group)
  {
    const int col = tid & 63;  // 0..31 -> V column, 32..63 -> W column
    const int ip = col & (TRD_NB - 1);
    const int g = tid >> 6;
    double2 acc = make_double2(0.0, 0.0);
    if (ip < i) {
      const int lo = g * RPG, hi = lo + RPG;
      if (ip < i - 1) {
        const double2* src = VW + (int64_t)col * N + rbase;
        double2 sv[RPG];
#pragma unroll
        for (int u = 0; u < RPG; ++u)
          sv[u] = (rbase + lo + u < n) ? src[lo + u] : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < RPG; ++u) acc = cadd(acc, cmulc(sv[u], xs[lo + u]));
      } else {
        const double2* src = (col < TRD_NB) ? vps : wps;
        for (int u = lo; u < hi; ++u) acc = cadd(acc, cmulc(src[u], xs[u]));
      }
    }
    red[g][col] = acc;
  }
  __syncthreads();
  // block partials, compact layout [|x|^2, conj(x) y, V^H x (i), W^H x (i)]
  const int nvals = 2 + 2 * i;
  if (tid < nvals) {
    const int t = tid;
    double2 sb = make_double2(0.0, 0.0);
    if (t < 2) {
      for (int w = 0; w < ROWS_A / 64; ++w) sb = cadd(sb, red0[w][t]);
    } else {
      const int src = (t < 2 + i) ? (t - 2) : (TRD_NB + t - 2 - i);
      for (int g = 0; g < RG; ++g) sb = cadd(sb, red[g][src]);
    }
    partA[(int64_t)blockIdx.x * NVAL + t] = sb;
  }
}

// Reflector c from the column kernel's partials (every block, same order),
// then y[r] = sum_j S[r, j] v[j] - V[r,:] (W^H v) - W[r,:] (V^H v),  r in (c, n).
// S is Hermitian with both triangles stored, so S[r, j] v[j] = conj(S[j, r]) v[j]
// reads column r contiguously.  v is staged in LDS; eight loads in flight per lane.
__global__ __launch_bounds__(HEMV_WAVES * 64) void k_trd_hemv(
    const double2* __restrict__ M, int64_t ld, int n, const double2* __restrict__ VW, int j0,
    int i, double2* __restrict__ hs, double2* __restrict__ ybuf,
    const double2* __restrict__ partA, double2* __restrict__ partB, double* __restrict__ dd,
    double* __restrict__ ee, double2* __restrict__ tau, const double2* __restrict__ yp,
    const int32_t* info) {
  constexpr int NTH = HEMV_WAVES * 64;
  constexpr int SLC = NTH / 128;
  __shared__ double2 vs[VCHUNK];
  __shared__ double2 red[HEMV_WAVES];
  __shared__ double2 sl[SLC][128];
  __shared__ double2 sums[NVAL];
  __shared__ double2 sVv[TRD_NB], sWv[TRD_NB];
  __shared__ double2 sh_scal;
  (void)info;  // no data-dependent indexing: runs even after an earlier failure
  const int c = j0 + i;
  const int64_t N = n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  // ---- reflector c from the column kernel's block partials
  const int nvals = 2 + 2 * i;
  const int nbA = cdiv(n - c, ROWS_A);
  {
    const int t = tid & 127, slice = tid >> 7;
    if (t < nvals) {
      double2 sb = make_double2(0.0, 0.0);
      for (int b = slice; b < nbA; b += SLC) sb = cadd(sb, partA[(int64_t)b * NVAL + t]);
      sl[slice][t] = sb;
    }
  }
  __syncthreads();
  if (tid < nvals) {
    double2 sb = make_double2(0.0, 0.0);
    for (int q = 0; q < SLC; ++q) sb = cadd(sb, sl[q][tid]);
    sums[tid] = sb;
  }
  __syncthreads();
  if (tid == 0) {
    const double2 ax = M[(c + 1) + (int64_t)c * ld];
    const double xn2 = sums[0].x;
    double2 tv, scal;
    double beta;
    if (xn2 == 0.0 && ax.y == 0.0) {
      tv = make_double2(0.0, 0.0);
      beta = ax.x;
      scal = make_double2(0.0, 0.0);
    } else {
      beta = -copysign(sqrt(ax.x * ax.x + ax.y * ax.y + xn2), ax.x);
      tv = make_double2((beta - ax.x) / beta, -ax.y / beta);
      const double2 dnm = make_double2(ax.x - beta, ax.y);
      const double q = 1.0 / cabs2(dnm);
      scal = make_double2(dnm.x * q, -dnm.y * q);
    }
    sh_scal = scal;
    if (blockIdx.x == 0) {
      ee[c] = beta;
      tau[c] = tv;
      dd[c] = M[c + (int64_t)c * ld].x;
      hs[HS_SCAL] = scal;
      hs[HS_TAU] = tv;
      // v^H y = y[c+1] + conj(scal) sum_{r >= c+2} conj(x_r) y_r
      if (yp) hs[HS_PDOT] = cadd(yp[c + 1], cmulc(scal, sums[1]));
    }
  }
  __syncthreads();
  const double2 scal = sh_scal;
  if (tid < i) {
    const double2 v1 = VW[(c + 1) + (int64_t)tid * N];
    const double2 w1 = VW[(c + 1) + (int64_t)(TRD_NB + tid) * N];
    sVv[tid] = cadd(cconj(v1), cmul(scal, sums[2 + tid]));
    sWv[tid] = cadd(cconj(w1), cmul(scal, sums[2 + i + tid]));
  }

  // ---- y = S v - V (W^H v) - W (V^H v)
  const int r = c + 1 + blockIdx.x * HEMV_WAVES + wid;
  const double2* vcol = M + (int64_t)c * ld;
  const double2* col = M + (int64_t)(r < n ? r : c) * ld;
  double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
  for (int js = c + 1; js < n; js += VCHUNK) {
    const int je = min(n, js + VCHUNK);
    __syncthreads();
    for (int j = js + tid; j < je; j += NTH)
      vs[j - js] = (j == c + 1) ? make_double2(1.0, 0.0) : cmul(scal, vcol[j]);
    __syncthreads();
    if (r < n) {
      int j = js + lane;
      for (; j + 7 * 64 < je; j += 8 * 64) {
        const double2 s0 = col[j], s1 = col[j + 64], s2 = col[j + 128], s3 = col[j + 192];
        const double2 s4 = col[j + 256], s5 = col[j + 320], s6 = col[j + 384], s7 = col[j + 448];
        const int b = j - js;
        a0 = cadd(a0, cmulc(s0, vs[b]));
        a1 = cadd(a1, cmulc(s1, vs[b + 64]));
        a2 = cadd(a2, cmulc(s2, vs[b + 128]));
        a3 = cadd(a3, cmulc(s3, vs[b + 192]));
        a0 = cadd(a0, cmulc(s4, vs[b + 256]));
        a1 = cadd(a1, cmulc(s5, vs[b + 320]));
        a2 = cadd(a2, cmulc(s6, vs[b + 384]));
        a3 = cadd(a3, cmulc(s7, vs[b + 448]));
      }
      for (; j < je; j += 64) a0 = cadd(a0, cmulc(col[j], vs[j - js]));
    }
  }
  double2 contrib = make_double2(0.0, 0.0);
  if (r < n) {
    double2 acc = cadd(cadd(a0, a1), cadd(a2, a3));
    if (lane < i) {
      const double2 vr = VW[r + (int64_t)lane * N];
      const double2 wr = VW[r + (int64_t)(TRD_NB + lane) * N];
      acc = csub(acc, cadd(cmul(vr, sWv[lane]), cmul(wr, sVv[lane])));
    }
    acc = wave_sum2(acc);
    if (lane == 0) {
      ybuf[r] = acc;
      const double2 vr = (r == c + 1) ? make_double2(1.0, 0.0) : cmul(scal, vcol[r]);
      contrib = cmulc(acc, vr);  // conj(y[r]) v[r]
    }
  }
  if (lane == 0) red[wid] = contrib;
  __syncthreads();
  if (tid == 0) {
    double2 sb = make_double2(0.0, 0.0);
    for (int w = 0; w < HEMV_WAVES; ++w) sb = cadd(sb, red[w]);
    partB[blockIdx.x] = sb;
  }
}

__global__ void k_trd_last(const double2* M, int64_t ld, int n, double* dd, const int32_t* info) {
  if (failed(info)) return;
  if (threadIdx.x == 0) dd[n - 1] = M[(n - 1) + (int64_t)(n - 1) * ld].x;
}

// zero columns [c0, 2*TRD_NB) pattern of the panel buffers (short last panel)
__global__ void k_trd_zero_cols(double2* VW, double2* WV, int64_t n, int jb) {
  const int64_t total = n * 2 * TRD_NB;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int colidx = (int)(e / n);
    if ((colidx % TRD_NB) >= jb) {
      VW[e] = make_double2(0.0, 0.0);
      WV[e] = make_double2(0.0, 0.0);
    }
  }
}

}  // namespace

int64_t trd_part_elems(int64_t n) {
  const int64_t a = ((n + ROWS_A - 1) / ROWS_A + 1) * NVAL;
  const int64_t b = (n + HEMV_WAVES - 1) / HEMV_WAVES + 1;
  return a + b;
}

bool tridiagonalise(double2* M, int64_t n, int64_t ld, const TrdBufs& w, int32_t* info,
                    hipStream_t s) {
  for (int64_t j0 = 0; j0 < n - 1; j0 += TRD_NB) {
    const int jb = (int)std::min<int64_t>(TRD_NB, n - 1 - j0);
    if (jb < TRD_NB)
      BSE_LAUNCH(k_trd_zero_cols, dim3(256), dim3(256), 0, s, w.VW, w.WV, n, jb);
    double2* partA = w.part;
    double2* partB = w.part + ((n + ROWS_A - 1) / ROWS_A + 1) * NVAL;
    for (int i = 0; i < jb; ++i) {
      const int64_t c = j0 + i;
      BSE_LAUNCH(k_trd_col, dim3(cdiv(n - c, ROWS_A)), dim3(COL_THREADS), 0, s, M, ld, (int)n, w.VW,
                 w.WV, (int)j0, i, 1, w.hs, w.ybuf, partA, partB, w.yproj, info);
      BSE_LAUNCH(k_trd_hemv, dim3(cdiv(n - c - 1, HEMV_WAVES)), dim3(HEMV_WAVES * 64), 0, s, M,
                 ld, (int)n, w.VW, (int)j0, i, w.hs, w.ybuf, partA, partB, w.dd, w.ee, w.tau,
                 w.yproj, info);
    }
    // finish the panel's last reflector
    BSE_LAUNCH(k_trd_col, dim3(cdiv(n - (j0 + jb), ROWS_A)), dim3(COL_THREADS), 0, s, M, ld, (int)n,
               w.VW, w.WV, (int)j0, jb, 0, w.hs, w.ybuf, partA, partB, w.yproj, info);
    const int64_t t = j0 + jb;
    if (t < n) {
      ZgemmParams g;  // S[t:, t:] -= [V W] [W V]^H
      g.M = (int)(n - t);
      g.N = (int)(n - t);
      g.K = 2 * TRD_NB;
      g.A = w.VW + t;
      g.a_rs = 1;
      g.a_cs = n;
      g.B = w.WV + t;
      g.b_rs = n;
      g.b_cs = 1;
      g.conjB = 1;
      g.C = M + t + t * ld;
      g.c_rs = 1;
      g.c_cs = ld;
      g.alpha = make_double2(-1.0, 0.0);
      g.beta = 1.0;
      g.info = info;
      g.tag = "zgemm_her2k";
      if (zgemm(g, 1, s) != hipSuccess) return false;
    }
  }
  BSE_LAUNCH(k_trd_last, dim3(1), dim3(64), 0, s, M, ld, (int)n, w.dd, info);
  return hipGetLastError() == hipSuccess;
}
