// Householder reduction of a Hermitian matrix to real symmetric tridiagonal
// form, T = Q^H S Q with Q = H_0 H_1 ... H_{n-2}, H_c = I - tau_c v_c v_c^H
// (blocked, lower, panel width TRD_NB), for the eigenproblem of Sec. 4.3.
// Only the lower triangle of S is read or updated.
//
// Per column c (local index i of its panel) two kernels run:
//   k_trd_col   finishes reflector c-1: y = S v - V (W^H v) - W (V^H v) from
//               the hemv kernel's partial sums, its W column, and H_{c-1}^H
//               applied to an optional probe vector; then applies the panel's
//               earlier reflectors to column c and writes block partial sums
//               of |x|^2, V^H x, W^H x;
//   k_trd_hemv  every block reduces |x|^2 (same order everywhere) and forms
//               reflector c; the blocks then cover the lower triangle of the
//               trailing matrix in square tiles, each tile (I, J) giving the
//               partial products S_IJ v_J (rows of I) and S_IJ^H v_I (rows
//               of J, off-diagonal tiles) plus its share of y^H v.
// Kernel boundaries order every exchange between blocks: no atomics, no
// fences.  After each panel one MFMA GEMM applies S -= [V W][W V]^H to the
// lower triangle of the trailing matrix.  The panel's V and W live in two
// n x 2*TRD_NB buffers, VW = [V | W] and WV = [W | V], which make that update
// one product.
#include "bse_internal.h"
#include "common.h"
#include "solve_internal.h"
#include "timing.h"
#include "zgemm.h"

namespace {

constexpr int ROWS_A = 128;     // rows per block of the column kernel
constexpr int COL_THREADS = 1024;
constexpr int HEMV_THREADS = 256;
constexpr int NVAL = 2 + 2 * TRD_NB;  // |x|^2, conj(x) y_probe, V^H x (i), W^H x (i)

// Square tile of the hemv kernel for a trailing matrix of order m.
__host__ __device__ inline int hemv_tile(int64_t m) { return m < 4096 ? 64 : (m < 12288 ? 128 : 256); }

// Partial sums of y = S v for a trailing matrix of order m starting at row b0,
// cut into nI x nI tiles of size t (lower triangle, tile-row I >= tile-column J):
// row r (tile index Ir) collects nI + 1 slots,
//   slot k <= Ir : Y[k][r]          = (S_{Ir,k} v_k)[r]
//   slot k >  Ir : Y[ycs + k-1][r]  = (S_{k-1,Ir}^H v_{k-1})[r]
BSE_DEV int64_t yslot(int k, int Ir, int ycs, int64_t n, int r) {
  return (int64_t)(k <= Ir ? k : ycs + k - 1) * n + r;
}

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

// x -= a conj(b)
BSE_DEV double2 sub_mulc(double2 x, double2 a, double2 b) {
  return make_double2(x.x - (a.x * b.x + a.y * b.y), x.y - (a.y * b.x - a.x * b.y));
}

// Full wavefront sum with DPP lane moves on the vector ALU (no LDS traffic);
// the total lands in lane 63.  Steps: quad swaps, half-row and row mirrors,
// then row 0 + 1 and row 2 + 3 through row_bcast:15, all four through
// row_bcast:31.  Lanes outside a step's row mask add zero.
template <int CTRL, int ROWS = 0xf>
BSE_DEV double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
BSE_DEV double wave_total63(double v) {
  v += dpp_d<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);       // row_half_mirror
  v += dpp_d<0x140>(v);       // row_mirror
  v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

__global__ __launch_bounds__(COL_THREADS) void k_trd_col(
    double2* __restrict__ M, int64_t ld, int n, double2* __restrict__ VW, double2* __restrict__ WV,
    int j0, int i, int has_new, const double2* __restrict__ hs, const double2* __restrict__ Y,
    int ycs, int tprev, double2* __restrict__ partA, const double2* __restrict__ partB,
    double2* __restrict__ yp) {
  constexpr int QP = COL_THREADS / ROWS_A;        // threads sharing one row
  constexpr int PER = TRD_NB / QP;                // panel columns per thread
  constexpr int YCH = 8;                          // y slots loaded per round
  constexpr int HW = ROWS_A / 64;                 // wavefronts per thread group qq
  __shared__ double2 vps[ROWS_A], wps[ROWS_A], x0s[ROWS_A], xs[ROWS_A];
  __shared__ double2 xpart[QP][ROWS_A];
  __shared__ double2 vcs[TRD_NB], wcs[TRD_NB];
  __shared__ double2 red[QP][HW][2 * PER];
  __shared__ double2 red0[HW][2];
  __shared__ double2 shb[COL_THREADS / 64];
  __shared__ double2 yc_s;
  __shared__ double2 svw[2 * TRD_NB];  // V^H v | W^H v of reflector c-1
  const int c = j0 + i;
  const int64_t N = n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int rbase = c + blockIdx.x * ROWS_A;
  const int rr = tid % ROWS_A, qq = tid / ROWS_A;  // qq is uniform in a wavefront
  const int r = rbase + rr;
  const bool act = r < n;

  // ---- 0. issue every global load of the kernel
  double2 x0 = make_double2(0.0, 0.0), xv = x0, ypr = x0;
  if (qq == 0 && act) {
    if (has_new) x0 = M[r + (int64_t)c * ld];
    if (yp) ypr = yp[r];
    if (i > 0) xv = M[r + (int64_t)(c - 1) * ld];
  }
  // panel reflectors 0..i-2 on this row: the correction of y_{c-1}, step 2, step 3
  double2 vr[PER], wr[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int ip = qq + u * QP;
    vr[u] = wr[u] = make_double2(0.0, 0.0);
    if (ip < i - 1 && act) {
      vr[u] = VW[r + (int64_t)ip * N];
      wr[u] = VW[r + (int64_t)(TRD_NB + ip) * N];
    }
  }
  if (tid < 2 * TRD_NB && tid % TRD_NB < i - 1) svw[tid] = hs[HS_SVV + tid];
  // y_{c-1}[r]: the previous hemv kernel's slots, QP threads per row
  const int nIp = i > 0 ? cdiv(n - c, tprev) : 0;
  double2 yq = make_double2(0.0, 0.0);
  if (i > 0 && act) {
    const int Ir = (r - c) / tprev;
    for (int k0 = qq; k0 <= nIp; k0 += YCH * QP) {
      double2 t[YCH];
#pragma unroll
      for (int u = 0; u < YCH; ++u) t[u] = Y[yslot(min(k0 + u * QP, nIp), Ir, ycs, N, r)];
#pragma unroll
      for (int u = 0; u < YCH; ++u)
        if (k0 + u * QP <= nIp) yq = cadd(yq, t[u]);
    }
  }
  // row c of the panel's earlier reflectors, and the slots of y_{c-1}[c] (wave 2)
  double2 vcl = make_double2(0.0, 0.0), wcl = vcl;
  if (qq == 1 && rr < i - 1) {
    vcl = VW[c + (int64_t)rr * N];
    wcl = VW[c + (int64_t)(TRD_NB + rr) * N];
  }
  double2 ycq = make_double2(0.0, 0.0);
  if (wid == 2 && i > 0)
    for (int k = lane; k <= nIp; k += 64) ycq = cadd(ycq, Y[yslot(k, 0, ycs, N, c)]);
  // the hemv blocks' partials of y^H v
  double2 pa = make_double2(0.0, 0.0);
  if (i > 0)
    for (int b = tid; b < nIp * (nIp + 1) / 2; b += COL_THREADS) pa = cadd(pa, partB[b]);
  double2 tc = make_double2(0.0, 0.0), scal_p = tc, pdot = tc;
  if (i > 0) {
    tc = hs[HS_TAU];
    scal_p = hs[HS_SCAL];
    pdot = hs[HS_PDOT];
  }
  __syncthreads();  // svw staged

  // ---- 1. y_{c-1} = S v - V (W^H v) - W (V^H v) and alpha
  double2 al = make_double2(0.0, 0.0);
  if (i > 0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int ip = qq + u * QP;
      if (ip < i - 1 && act)
        yq = csub(yq, cadd(cmul(vr[u], svw[TRD_NB + ip]), cmul(wr[u], svw[ip])));
    }
    if (wid == 2) {
      if (lane < i - 1)
        ycq = csub(ycq, cadd(cmul(vcl, svw[TRD_NB + lane]), cmul(wcl, svw[lane])));
      ycq = wave_sum2(ycq);
      if (lane == 0) yc_s = ycq;
    }
    xpart[qq][rr] = yq;
    const double2 s = block_sum2(pa, shb);  // y^H v; synchronises the block
    const double t2 = cabs2(tc);
    al = make_double2(-0.5 * t2 * s.x, -0.5 * t2 * s.y);
  }

  // ---- finish reflector c-1 (row threads) and stage row c of the panel
  if (qq == 0) {
    double2 vprev_r = make_double2(0.0, 0.0), wprev_r = make_double2(0.0, 0.0);
    if (i > 0 && act) {
      double2 y = make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < QP; ++q) y = cadd(y, xpart[q][rr]);
      vprev_r = (r == c) ? make_double2(1.0, 0.0) : cmul(scal_p, xv);
      M[r + (int64_t)(c - 1) * ld] = vprev_r;
      wprev_r = cadd(cmul(tc, y), cmul(al, vprev_r));
      VW[r + (int64_t)(i - 1) * N] = vprev_r;
      VW[r + (int64_t)(TRD_NB + i - 1) * N] = wprev_r;
      WV[r + (int64_t)(i - 1) * N] = wprev_r;
      WV[r + (int64_t)(TRD_NB + i - 1) * N] = vprev_r;
      if (yp) {
        // y_probe <- H^H y_probe = y_probe - conj(tau) (v^H y_probe) v
        const double2 f = cmulc(tc, pdot);
        ypr = csub(ypr, cmul(f, vprev_r));
        yp[r] = ypr;
      }
    }
    vps[rr] = vprev_r;
    wps[rr] = wprev_r;
    x0s[rr] = x0;
  } else if (qq == 1 && has_new && rr < i - 1) {
    vcs[rr] = vcl;
    wcs[rr] = wcl;
  }
  if (!has_new) return;
  __syncthreads();

  // ---- 2. apply the panel's earlier reflectors to column c: QP threads per row
  {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int ip = qq + u * QP;
      if (ip < i - 1) {
        acc = cadd(acc, cmulc(wcs[ip], vr[u]));   // v_ip[r] conj(w_ip[c])
        acc = cadd(acc, cmulc(vcs[ip], wr[u]));   // w_ip[r] conj(v_ip[c])
      }
    }
    xpart[qq][rr] = acc;
  }
  __syncthreads();
  if (qq == 0) {
    double2 x = make_double2(0.0, 0.0);
    bool tail = false;
    if (act) {
      x = x0s[rr];
#pragma unroll
      for (int q = 0; q < QP; ++q) x = csub(x, xpart[q][rr]);
      if (i > 0) {
        // reflector c-1: v[c] = 1, w[c] = tau y[c] + alpha
        const double2 wprev_c = cadd(cmul(tc, yc_s), al);
        x = sub_mulc(x, vps[rr], wprev_c);
        x = csub(x, wps[rr]);
      }
      if (r == c) x.y = 0.0;
      M[r + (int64_t)c * ld] = x;
      tail = r >= c + 2;
    }
    xs[rr] = tail ? x : make_double2(0.0, 0.0);
    const double2 s0 = wave_sum2(make_double2(tail ? cabs2(x) : 0.0, 0.0));
    const double2 s1 = wave_sum2((tail && yp) ? cmulc(x, ypr) : make_double2(0.0, 0.0));
    if (lane == 0) {
      red0[wid][0] = s0;
      red0[wid][1] = s1;
    }
  }
  __syncthreads();

  // ---- 3. V^H x and W^H x over this block's rows from the panel values each
  // thread holds (column ip = qq + u QP; column i-1 from LDS), wavefront sums
  {
    const double2 x = xs[rr];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int ip = qq + u * QP;
      if (ip < i) {  // uniform in the wavefront
        double2 v = vr[u], w = wr[u];
        if (ip == i - 1) {
          v = vps[rr];
          w = wps[rr];
        }
        double2 pv = cmulc(v, x), pw = cmulc(w, x);
        pv.x = wave_total63(pv.x);
        pv.y = wave_total63(pv.y);
        pw.x = wave_total63(pw.x);
        pw.y = wave_total63(pw.y);
        if (lane == 63) {
          red[qq][wid % HW][2 * u] = pv;
          red[qq][wid % HW][2 * u + 1] = pw;
        }
      }
    }
  }
  __syncthreads();
  // block partials, compact layout [|x|^2, conj(x) y, V^H x (i), W^H x (i)]
  const int nvals = 2 + 2 * i;
  if (tid < nvals) {
    const int t = tid;
    double2 sb = make_double2(0.0, 0.0);
    if (t < 2) {
      for (int w = 0; w < HW; ++w) sb = cadd(sb, red0[w][t]);
    } else {
      const bool isw = t >= 2 + i;
      const int ip = isw ? t - 2 - i : t - 2;
      for (int h = 0; h < HW; ++h) sb = cadd(sb, red[ip % QP][h][2 * (ip / QP) + (isw ? 1 : 0)]);
    }
    partA[(int64_t)blockIdx.x * NVAL + t] = sb;
  }
}

// Reflector c from the column kernel's partials, then the Hermitian product
// S v over the lower triangle of the trailing matrix (rows and columns c+1..n-1)
// in t x t tiles, one block per tile (I >= J), tiles numbered column-major.
// Wavefront w reads columns w, w+4, ... of the tile, lane l rows l, l+64, ...:
// each load is a contiguous 1 KB column segment.  The first two load batches
// of the tile are issued before the reflector is formed (every thread forms it
// from the same reduced |x|^2, so no broadcast round trip is needed).  Block 0
// also stores the reflector, V^H v and W^H v for the next column kernel.
template <int TT>
__global__ __launch_bounds__(HEMV_THREADS) void k_trd_hemv(
    const double2* __restrict__ M, int64_t ld, int n, const double2* __restrict__ VW, int j0,
    int i, double2* __restrict__ hs, const double2* __restrict__ partA,
    double2* __restrict__ partB, double2* __restrict__ Y, int ycs, double* __restrict__ dd,
    double* __restrict__ ee, double2* __restrict__ tau, const double2* __restrict__ yp) {
  constexpr int U = TT / 64;              // rows per lane
  constexpr int CPW = TT / 4;             // columns per wavefront
  constexpr int CB = (8 / U) < CPW ? (8 / U) : CPW;  // columns per load batch
  constexpr int SLC = HEMV_THREADS / 128;
  __shared__ double2 sl[SLC][128];
  __shared__ double2 sums[NVAL];
  __shared__ double2 vrow[TT], vcol[TT], csum[TT];
  __shared__ double2 racc[HEMV_THREADS / 64][TT];
  __shared__ double2 red[HEMV_THREADS / 64];
  const int c = j0 + i, b0 = c + 1;
  const int64_t N = n;
  const int m = n - b0;
  const int nI = cdiv(m, TT);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int bid = blockIdx.x;

  // ---- tile of this block: largest J with J*nI - J(J-1)/2 <= bid
  int J = 0;
  {
    int lo = 0, hi = nI - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      const int64_t pre = (int64_t)mid * nI - (int64_t)mid * (mid - 1) / 2;
      if (pre <= bid) lo = mid; else hi = mid - 1;
    }
    J = lo;
  }
  const int Ib = J + (bid - (J * nI - J * (J - 1) / 2));
  const int cj0 = b0 + J * TT, rb0 = b0 + Ib * TT;
  const bool diag = Ib == J;
  const int nlast = n - 1;

  auto load = [&](double2 (&s)[CB][U], int q0) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int jl = wid + 4 * (q0 + cb);
      const int64_t jc = min(cj0 + jl, nlast);
#pragma unroll
      for (int u = 0; u < U; ++u) s[cb][u] = M[min(rb0 + lane + 64 * u, nlast) + jc * ld];
    }
  };

  // ---- issue the first tile batches and every load of the reflector
  double2 ba[CB][U], bb[CB][U];
  load(ba, 0);
  if (CB < CPW) load(bb, CB);
  const double2* xcol = M + (int64_t)c * ld;
  const double2 ax = xcol[b0];
  double2 xc = make_double2(0.0, 0.0), xr = xc;
  if (tid < TT) {
    if (cj0 + tid < n) xc = xcol[cj0 + tid];
    if (rb0 + tid < n) xr = xcol[rb0 + tid];
  }
  const int nbA = cdiv(n - c, ROWS_A);
  const int nvals = 2 + 2 * i;
  if (wid == 0) {
    double2 a = make_double2(0.0, 0.0);
    for (int b = lane; b < nbA; b += 64) a = cadd(a, partA[(int64_t)b * NVAL]);
    a = wave_sum2(a);
    if (lane == 0) sums[0] = a;
  }
  if (bid == 0) {
    const int t = tid & 127, slice = tid >> 7;
    if (t >= 1 && t < nvals) {
      double2 sb = make_double2(0.0, 0.0);
      for (int b = slice; b < nbA; b += SLC) sb = cadd(sb, partA[(int64_t)b * NVAL + t]);
      sl[slice][t] = sb;
    }
  }
  __syncthreads();
  if (bid == 0 && tid >= 1 && tid < nvals) {
    double2 sb = make_double2(0.0, 0.0);
    for (int q = 0; q < SLC; ++q) sb = cadd(sb, sl[q][tid]);
    sums[tid] = sb;
  }
  __syncthreads();

  // ---- reflector c (the same arithmetic in every thread)
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
  // block 0: the reflector, V^H v and W^H v of the panel, and their share of
  // y^H v: sum_r conj(V (W^H v) + W (V^H v))[r] v[r] = sum_ip conj(sWv) sVv + conj(sVv) sWv
  double2 corr = make_double2(0.0, 0.0);
  if (bid == 0) {
    if (tid == 0) {
      ee[c] = beta;
      tau[c] = tv;
      dd[c] = M[c + (int64_t)c * ld].x;
      hs[HS_SCAL] = scal;
      hs[HS_TAU] = tv;
      // v^H y = y[c+1] + conj(scal) sum_{r >= c+2} conj(x_r) y_r
      if (yp) hs[HS_PDOT] = cadd(yp[b0], cmulc(scal, sums[1]));
    }
    if (tid < i) {
      const double2 v1 = VW[b0 + (int64_t)tid * N];
      const double2 w1 = VW[b0 + (int64_t)(TRD_NB + tid) * N];
      const double2 svv = cadd(cconj(v1), cmul(scal, sums[2 + tid]));
      const double2 swv = cadd(cconj(w1), cmul(scal, sums[2 + i + tid]));
      hs[HS_SVV + tid] = svv;
      hs[HS_SWV + tid] = swv;
      corr = cadd(cmulc(swv, svv), cmulc(svv, swv));
    }
  }
  // ---- v on the tile's rows and columns
  if (tid < TT) {
    const int j = cj0 + tid, r = rb0 + tid;
    vcol[tid] = (j < n) ? ((j == b0) ? make_double2(1.0, 0.0) : cmul(scal, xc)) : make_double2(0.0, 0.0);
    vrow[tid] = (r < n) ? ((r == b0) ? make_double2(1.0, 0.0) : cmul(scal, xr)) : make_double2(0.0, 0.0);
  }
  __syncthreads();

  // ---- tile product: rows S_IJ v_J (lane-local), columns S_IJ^H v_I (wave sums)
  double2 vr[U], racc_l[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    vr[u] = vrow[lane + 64 * u];
    racc_l[u] = make_double2(0.0, 0.0);
  }
  auto use = [&](const double2 (&s)[CB][U], int q0) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      const int jl = wid + 4 * (q0 + cb);
      const bool jok = cj0 + jl < n;
      const double2 vj = vcol[jl];
      double2 cacc = make_double2(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rl = lane + 64 * u;
        const bool ok = jok && (rb0 + rl < n) && (!diag || rl >= jl);
        const bool strict = !diag || rl > jl;
        double2 sr = ok ? s[cb][u] : make_double2(0.0, 0.0);
        if (diag && rl == jl) sr.y = 0.0;  // the diagonal of a Hermitian matrix is real
        racc_l[u] = cadd(racc_l[u], cmul(sr, vj));
        if (ok && strict) cacc = cadd(cacc, cmulc(s[cb][u], vr[u]));
      }
      cacc.x = wave_total63(cacc.x);
      cacc.y = wave_total63(cacc.y);
      if (lane == 63) csum[jl] = cacc;
    }
  };
#pragma unroll 1
  for (int q0 = 0; q0 < CPW; q0 += 2 * CB) {
    use(ba, q0);
    if (q0 + 2 * CB < CPW) load(ba, q0 + 2 * CB);
    if (q0 + CB < CPW) {
      use(bb, q0 + CB);
      if (q0 + 3 * CB < CPW) load(bb, q0 + 3 * CB);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) racc[wid][lane + 64 * u] = racc_l[u];
  __syncthreads();

  // ---- slots and this block's share of y^H v
  double2 pb = make_double2(0.0, 0.0);
  if (tid < TT) {
    const int r = rb0 + tid, j = cj0 + tid;
    if (r < n) {
      double2 rp = make_double2(0.0, 0.0);
#pragma unroll
      for (int w = 0; w < HEMV_THREADS / 64; ++w) rp = cadd(rp, racc[w][tid]);
      Y[(int64_t)J * N + r] = rp;
      pb = cadd(pb, cmulc(rp, vrow[tid]));
    }
    if (j < n) {
      const double2 cp = csum[tid];
      Y[(int64_t)(ycs + Ib) * N + j] = cp;
      pb = cadd(pb, cmulc(cp, vcol[tid]));
    }
  }
  pb = csub(pb, corr);
  pb = block_sum2(pb, red);
  if (tid == 0) partB[bid] = pb;
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

// Largest hemv grid over the sweep (tiles of the largest trailing order in
// each tile-size range).
int64_t hemv_blocks_max(int64_t n) {
  int64_t best = 1;
  for (int64_t m : {std::min<int64_t>(n - 1, 4095), std::min<int64_t>(n - 1, 12287), n - 1}) {
    if (m < 1) continue;
    const int64_t t = hemv_tile(m), nI = (m + t - 1) / t;
    best = std::max(best, nI * (nI + 1) / 2);
  }
  return best;
}

int64_t ycs_of(int64_t n) { return (n + 63) / 64; }

template <int TT>
void launch_hemv(int nb, double2* M, int64_t ld, int64_t n, const TrdBufs& w, int j0, int i,
                 double2* partA, double2* partB, double2* Y, int ycs, hipStream_t s) {
  BSE_LAUNCH(k_trd_hemv<TT>, dim3(nb), dim3(HEMV_THREADS), 0, s, M, ld, (int)n, w.VW, j0, i, w.hs,
             partA, partB, Y, ycs, w.dd, w.ee, w.tau, w.yproj);
}

}  // namespace

// [partA: column-kernel partials | partB: hemv partials of y^H v | Y: hemv slots]
int64_t trd_part_elems(int64_t n) {
  const int64_t a = ((n + ROWS_A - 1) / ROWS_A + 1) * NVAL;
  return a + hemv_blocks_max(n) + 2 * ycs_of(n) * n;
}

bool tridiagonalise(double2* M, int64_t n, int64_t ld, const TrdBufs& w, int32_t* info,
                    hipStream_t s) {
  double2* partA = w.part;
  double2* partB = w.part + ((n + ROWS_A - 1) / ROWS_A + 1) * NVAL;
  double2* Y = partB + hemv_blocks_max(n);
  const int ycs = (int)ycs_of(n);
  for (int64_t j0 = 0; j0 < n - 1; j0 += TRD_NB) {
    const int jb = (int)std::min<int64_t>(TRD_NB, n - 1 - j0);
    if (jb < TRD_NB)
      BSE_LAUNCH(k_trd_zero_cols, dim3(256), dim3(256), 0, s, w.VW, w.WV, n, jb);
    for (int i = 0; i < jb; ++i) {
      const int64_t c = j0 + i, m = n - c - 1;
      BSE_LAUNCH(k_trd_col, dim3(cdiv(n - c, ROWS_A)), dim3(COL_THREADS), 0, s, M, ld, (int)n, w.VW,
                 w.WV, (int)j0, i, 1, w.hs, Y, ycs, hemv_tile(n - c), partA, partB, w.yproj);
      const int tt = hemv_tile(m);
      const int nI = cdiv(m, tt), nb = nI * (nI + 1) / 2;
      if (tt == 64) launch_hemv<64>(nb, M, ld, n, w, (int)j0, i, partA, partB, Y, ycs, s);
      else if (tt == 128) launch_hemv<128>(nb, M, ld, n, w, (int)j0, i, partA, partB, Y, ycs, s);
      else launch_hemv<256>(nb, M, ld, n, w, (int)j0, i, partA, partB, Y, ycs, s);
    }
    // finish the panel's last reflector
    const int64_t cl = j0 + jb;
    BSE_LAUNCH(k_trd_col, dim3(cdiv(n - cl, ROWS_A)), dim3(COL_THREADS), 0, s, M, ld, (int)n,
               w.VW, w.WV, (int)j0, jb, 0, w.hs, Y, ycs, hemv_tile(n - cl), partA, partB, w.yproj);
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
      g.c_uplo = 2;  // lower triangle only
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
