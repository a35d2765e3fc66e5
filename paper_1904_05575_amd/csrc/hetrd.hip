// Householder reduction of a Hermitian matrix to real symmetric tridiagonal
// form, T = Q^H S Q with Q = H_0 H_1 ... H_{n-2}, H_c = I - tau_c v_c v_c^H
// (blocked, lower, panel width TRD_NB), for the eigenproblem of Sec. 4.3.
//
// Per column c (local index i of its panel) two kernels run:
//   k_trd_col   finishes reflector c-1 (its v, its W column, and H_{c-1}^H
//               applied to an optional probe vector), applies the panel's
//               earlier reflectors to column c, and forms reflector c (the
//               last block to finish reduces the block partial sums);
//   k_trd_hemv  y = S v_c - V (W^H v_c) - W (V^H v_c), one wavefront per
//               output row, reading column r of the trailing matrix.
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
constexpr int HEMV_WAVES = 8;   // output rows per hemv block
constexpr int VCHUNK = 2048;    // v staged in LDS in chunks of this many entries
constexpr int NVAL = 2 + 2 * TRD_NB;  // |x|^2, conj(x) y_probe, V^H x (i), W^H x (i)

BSE_DEV double2 ld_acq(const double2* p) {
  double2 v;
  v.x = __hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.y = __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

// x -= a conj(b)
BSE_DEV double2 sub_mulc(double2 x, double2 a, double2 b) {
  return make_double2(x.x - (a.x * b.x + a.y * b.y), x.y - (a.y * b.x - a.x * b.y));
}

__global__ __launch_bounds__(ROWS_A) void k_trd_col(
    double2* __restrict__ M, int64_t ld, int n, double2* __restrict__ VW, double2* __restrict__ WV,
    int j0, int i, int has_new, double2* __restrict__ hs, const double2* __restrict__ ybuf,
    double2* __restrict__ part, int32_t* counter, double* __restrict__ dd,
    double* __restrict__ ee, double2* __restrict__ tau, double2* __restrict__ yp,
    const int32_t* info) {
  constexpr int NG = ROWS_A / 64;
  __shared__ double2 xs[ROWS_A], vps[ROWS_A], wps[ROWS_A];
  __shared__ double2 vcs[TRD_NB], wcs[TRD_NB];
  __shared__ double2 red[NG][2 * TRD_NB + 2];
  __shared__ double2 sums[NVAL];
  __shared__ double2 sh_scal;
  __shared__ int is_last;
  if (failed(info)) return;
  const int c = j0 + i;
  const int64_t N = n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int rbase = c + blockIdx.x * ROWS_A;
  const int r = rbase + tid;
  const bool act = r < n;

  // ---- 0. finish reflector c-1
  double2 vprev_r = make_double2(0.0, 0.0), wprev_r = make_double2(0.0, 0.0);
  double2 wprev_c = make_double2(0.0, 0.0);
  if (i > 0) {
    const int cp = c - 1;
    const double2 scal = hs[HS_SCAL], tc = hs[HS_TAU], al = hs[HS_ALPHA];
    if (act) {
      const double2 xv = M[r + (int64_t)cp * ld];
      vprev_r = (r == c) ? make_double2(1.0, 0.0) : cmul(scal, xv);
      M[r + (int64_t)cp * ld] = vprev_r;
      wprev_r = cadd(cmul(tc, ybuf[r]), cmul(al, vprev_r));
      VW[r + (int64_t)(i - 1) * N] = vprev_r;
      VW[r + (int64_t)(TRD_NB + i - 1) * N] = wprev_r;
      WV[r + (int64_t)(i - 1) * N] = wprev_r;
      WV[r + (int64_t)(TRD_NB + i - 1) * N] = vprev_r;
      if (yp) {
        // y <- H^H y = y - conj(tau) (v^H y) v
        const double2 f = cmulc(tc, hs[HS_PDOT]);
        yp[r] = csub(yp[r], cmul(f, vprev_r));
      }
    }
    wprev_c = cadd(cmul(tc, ybuf[c]), al);
  }
  if (!has_new) return;

  // ---- 1. apply the panel's earlier reflectors to column c (one row per thread);
  // row c of the panel is the same for every thread and is staged in LDS
  for (int ip = tid; ip < i - 1; ip += ROWS_A) {
    vcs[ip] = VW[c + (int64_t)ip * N];
    wcs[ip] = VW[c + (int64_t)(TRD_NB + ip) * N];
  }
  __syncthreads();
  double2 x = make_double2(0.0, 0.0);
  if (act) {
    x = M[r + (int64_t)c * ld];
    for (int ip0 = 0; ip0 < i - 1; ip0 += 8) {
      double2 vr[8], wr[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (ip0 + u < i - 1) {
          vr[u] = VW[r + (int64_t)(ip0 + u) * N];
          wr[u] = VW[r + (int64_t)(TRD_NB + ip0 + u) * N];
        }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (ip0 + u < i - 1) {
          x = sub_mulc(x, vr[u], wcs[ip0 + u]);
          x = sub_mulc(x, wr[u], vcs[ip0 + u]);
        }
    }
    if (i > 0) {
      x = sub_mulc(x, vprev_r, wprev_c);
      x = sub_mulc(x, wprev_r, make_double2(1.0, 0.0));
    }
    if (r == c) x.y = 0.0;
    M[r + (int64_t)c * ld] = x;
  }
  const bool tail = act && (r >= c + 2);
  xs[tid] = tail ? x : make_double2(0.0, 0.0);
  vps[tid] = vprev_r;  // column i-1 of the panel, just formed by this thread
  wps[tid] = wprev_r;
  {
    const double2 s0 = wave_sum2(make_double2(tail ? cabs2(x) : 0.0, 0.0));
    const double2 s1 = wave_sum2((tail && yp) ? cmulc(x, yp[r]) : make_double2(0.0, 0.0));
    if (lane == 0) {
      red[wid][2 * TRD_NB] = s0;
      red[wid][2 * TRD_NB + 1] = s1;
    }
  }
  __syncthreads();

  // ---- 2. V^H x and W^H x over this block's rows: thread = (panel column, row group)
  {
    const int col = tid & 63;  // 0..31 -> V column, 32..63 -> W column
    const int ip = col & (TRD_NB - 1);
    double2 acc = make_double2(0.0, 0.0);
    const int r0 = rbase + wid * 64;
    const int rlim = min(n, r0 + 64);
    if (ip < i - 1) {
      const double2* src = VW + (int64_t)col * N;
      for (int rr0 = max(r0, c + 2); rr0 < rlim; rr0 += 16) {
        double2 sv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (rr0 + u < rlim) sv[u] = src[rr0 + u];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (rr0 + u < rlim) acc = cadd(acc, cmulc(sv[u], xs[rr0 + u - rbase]));
      }
    } else if (ip == i - 1) {
      const double2* src = (col < TRD_NB) ? vps : wps;
      for (int rr = max(r0, c + 2); rr < rlim; ++rr)
        acc = cadd(acc, cmulc(src[rr - rbase], xs[rr - rbase]));
    }
    red[wid][col] = acc;
  }
  __syncthreads();
  // block partials, compact layout [|x|^2, conj(x) y, V^H x (i), W^H x (i)]
  const int nvals = 2 + 2 * i;
  for (int t = tid; t < nvals; t += ROWS_A) {
    const int src = (t == 0) ? 2 * TRD_NB : (t == 1) ? 2 * TRD_NB + 1
                  : (t < 2 + i) ? (t - 2) : (TRD_NB + t - 2 - i);
    double2 sb = make_double2(0.0, 0.0);
    for (int g = 0; g < NG; ++g) sb = cadd(sb, red[g][src]);
    part[(int64_t)blockIdx.x * NVAL + t] = sb;
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) is_last = (atomicAdd(counter, 1) == (int)gridDim.x - 1);
  __syncthreads();
  if (!is_last) return;
  __threadfence();

  // ---- 3. last block: reflector c
  const int nb = gridDim.x;
  for (int t = tid; t < nvals; t += ROWS_A) {
    double2 sb = make_double2(0.0, 0.0);
    int b = 0;
    for (; b + 8 <= nb; b += 8) {
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = ld_acq(part + (int64_t)(b + u) * NVAL + t);
#pragma unroll
      for (int u = 0; u < 8; ++u) sb = cadd(sb, v[u]);
    }
    for (; b < nb; ++b) sb = cadd(sb, ld_acq(part + (int64_t)b * NVAL + t));
    sums[t] = sb;
  }
  __syncthreads();
  if (tid == 0) {
    const double2 ax = ld_acq(M + (c + 1) + (int64_t)c * ld);
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
    ee[c] = beta;
    tau[c] = tv;
    dd[c] = ld_acq(M + c + (int64_t)c * ld).x;
    hs[HS_SCAL] = scal;
    hs[HS_TAU] = tv;
    if (yp) {
      // v^H y = y[c+1] + conj(scal) sum_{r >= c+2} conj(x_r) y_r
      const double2 y1 = ld_acq(yp + (c + 1));
      hs[HS_PDOT] = cadd(y1, cmulc(scal, sums[1]));
    }
    sh_scal = scal;
  }
  __syncthreads();
  const double2 scal = sh_scal;
  for (int ip = tid; ip < i; ip += ROWS_A) {
    const double2 v1 = ld_acq(VW + (c + 1) + (int64_t)ip * N);
    const double2 w1 = ld_acq(VW + (c + 1) + (int64_t)(TRD_NB + ip) * N);
    hs[HS_VV + ip] = cadd(cconj(v1), cmul(scal, sums[2 + ip]));
    hs[HS_WV + ip] = cadd(cconj(w1), cmul(scal, sums[2 + i + ip]));
  }
  if (tid == 0) *counter = 0;
}

// y[r] = sum_j S[r, j] v[j] - V[r,:] (W^H v) - W[r,:] (V^H v),  r in (c, n).
// S is Hermitian with both triangles stored, so S[r, j] v[j] = conj(S[j, r]) v[j]
// reads column r contiguously.  v is staged in LDS; eight loads in flight per lane.
__global__ __launch_bounds__(HEMV_WAVES * 64) void k_trd_hemv(
    const double2* __restrict__ M, int64_t ld, int n, const double2* __restrict__ VW, int j0,
    int i, double2* __restrict__ hs, double2* __restrict__ ybuf, double2* __restrict__ part,
    int32_t* counter, const int32_t* info) {
  __shared__ double2 vs[VCHUNK];
  __shared__ double2 red[HEMV_WAVES];
  __shared__ int is_last;
  if (failed(info)) return;
  const int c = j0 + i;
  const int64_t N = n;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int r = c + 1 + blockIdx.x * HEMV_WAVES + wid;
  const double2 scal = hs[HS_SCAL];
  const double2* vcol = M + (int64_t)c * ld;
  const double2* col = M + (int64_t)(r < n ? r : c) * ld;
  double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0, a3 = a0;
  for (int js = c + 1; js < n; js += VCHUNK) {
    const int je = min(n, js + VCHUNK);
    __syncthreads();
    for (int j = js + (int)threadIdx.x; j < je; j += HEMV_WAVES * 64)
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
      acc = csub(acc, cadd(cmul(vr, hs[HS_WV + lane]), cmul(wr, hs[HS_VV + lane])));
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
  if (threadIdx.x == 0) {
    double2 sb = make_double2(0.0, 0.0);
    for (int w = 0; w < HEMV_WAVES; ++w) sb = cadd(sb, red[w]);
    part[blockIdx.x] = sb;
    __threadfence();
    is_last = (atomicAdd(counter, 1) == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (wid == 0) {
    double2 sb = make_double2(0.0, 0.0);
    for (int b = lane; b < (int)gridDim.x; b += 64) sb = cadd(sb, ld_acq(part + b));
    sb = wave_sum2(sb);
    if (lane == 0) {
      const double t2 = cabs2(hs[HS_TAU]);
      hs[HS_ALPHA] = make_double2(-0.5 * t2 * sb.x, -0.5 * t2 * sb.y);
      *counter = 0;
    }
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
  return std::max(a, b);
}

bool tridiagonalise(double2* M, int64_t n, int64_t ld, const TrdBufs& w, int32_t* info,
                    hipStream_t s) {
  for (int64_t j0 = 0; j0 < n - 1; j0 += TRD_NB) {
    const int jb = (int)std::min<int64_t>(TRD_NB, n - 1 - j0);
    if (jb < TRD_NB)
      BSE_LAUNCH(k_trd_zero_cols, dim3(256), dim3(256), 0, s, w.VW, w.WV, n, jb);
    for (int i = 0; i < jb; ++i) {
      const int64_t c = j0 + i;
      BSE_LAUNCH(k_trd_col, dim3(cdiv(n - c, ROWS_A)), dim3(ROWS_A), 0, s, M, ld, (int)n, w.VW,
                 w.WV, (int)j0, i, 1, w.hs, w.ybuf, w.part, w.counters + 0, w.dd, w.ee, w.tau,
                 w.yproj, info);
      BSE_LAUNCH(k_trd_hemv, dim3(cdiv(n - c - 1, HEMV_WAVES)), dim3(HEMV_WAVES * 64), 0, s, M,
                 ld, (int)n, w.VW, (int)j0, i, w.hs, w.ybuf, w.part, w.counters + 1, info);
    }
    // finish the panel's last reflector
    BSE_LAUNCH(k_trd_col, dim3(cdiv(n - (j0 + jb), ROWS_A)), dim3(ROWS_A), 0, s, M, ld, (int)n,
               w.VW, w.WV, (int)j0, jb, 0, w.hs, w.ybuf, w.part, w.counters + 0, w.dd, w.ee,
               w.tau, w.yproj, info);
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
