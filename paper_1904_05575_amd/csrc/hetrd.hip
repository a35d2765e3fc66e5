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
//               trailing matrix in square tiles, each block an equal run of
//               consecutive tiles, each tile (I, J) giving the partial
//               products S_IJ v_J (rows of I) and S_IJ^H v_I (rows of J,
//               off-diagonal tiles) plus its share of y^H v.
// Kernel boundaries order every exchange between blocks: no atomics, no
// fences.  After each panel one MFMA GEMM applies S -= [V W][W V]^H to the
// lower triangle of the trailing matrix.  The panel's V and W live in two
// n x 2*TRD_NB buffers, VW = [V | W] and WV = [W | V], which make that update
// one product.
#include <algorithm>
#include <vector>

#include "bse_internal.h"
#include "common.h"
#include "solve_internal.h"
#include "timing.h"
#include "zgemm.h"

namespace {

constexpr int ROWS_A = 64;      // rows per block of the column kernel
constexpr int COL_THREADS = 1024;
constexpr int HT = 64;          // square tile of the hemv kernel
constexpr int HV_THREADS = 1024; // hemv block: 16 wavefronts, 4 tile columns each
constexpr int NVAL = 2 + 2 * TRD_NB;  // |x|^2, conj(x) y_probe, V^H x (i), W^H x (i)

// The hemv tiling of the trailing matrix (rows and columns b0..n-1) starts at
// org = b0 rounded down to 8 elements (128 bytes), so that every column segment
// of a tile covers whole cache lines (unaligned segments fetch one line more in
// eight); rows and columns org..b0-1 are masked (v = 0 there).
__host__ __device__ inline int trd_org(int b0) { return b0 & ~7; }

// Partial sums of y = S v for a trailing matrix of order m starting at row org,
// cut into nI x nI tiles of order HT (lower triangle: tile-row I >= tile-column
// J).  Tile (I, J) has index I (I + 1) / 2 + J (tile-rows in order); block b
// of a launch with G blocks over T tiles takes the run [T b / G, T (b+1) / G),
// so that no block has more than one tile above the mean.  The part of a
// tile-row inside one block's run is a piece; piece p of tile-row I (p counted
// from the block that holds the row's first tile) leaves its row sums in slot
// p.  Row r, in tile-row Ir, collects
//   Y[p][r]        p = 0 .. nrs - 1   (the pieces of tile-row Ir: S v over them)
//   Y[ycs + I][r]  I = Ir .. nI - 1   (tile (I, Ir): S_{I,Ir}^H v_I)
// i.e. nrs + nI - Ir slots, nrs = block_of(last tile of Ir) - block_of(first) + 1.
__host__ __device__ inline int64_t hemv_tile_start(int64_t T, int G, int b) {
  return T * b / G;
}
__host__ __device__ inline int hemv_block_of(int64_t T, int G, int64_t t) {
  return (int)(((t + 1) * G - 1) / T);
}
BSE_DEV int64_t yslot(int q, int Ir, int nrs, int ycs, int64_t n, int r) {
  return (int64_t)(q < nrs ? q : ycs + Ir + (q - nrs)) * n + r;
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

// Wavefront sum of a complex value, every lane gets it (DPP, then lane 63
// broadcast).
BSE_DEV double bcast63(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
BSE_DEV double2 wave_sum2_dpp(double2 v) {
  return make_double2(bcast63(wave_total63(v.x)), bcast63(wave_total63(v.y)));
}

// v where ok, else 0 (component selects: a select of the whole vector type
// would send register arrays to scratch)
BSE_DEV double2 keep(bool ok, double2 v) { return make_double2(ok ? v.x : 0.0, ok ? v.y : 0.0); }

// x -= a conj(b)
BSE_DEV double2 sub_mulc(double2 x, double2 a, double2 b) {
  return make_double2(x.x - (a.x * b.x + a.y * b.y), x.y - (a.y * b.x - a.x * b.y));
}

BSE_DEV void trd_col_dev(
    double2* __restrict__ M, int64_t ld, int n, double2* __restrict__ VW, double2* __restrict__ WV,
    int j0, int i, int has_new, const double2* __restrict__ hs, const double2* __restrict__ Y,
    int ycs, int gprev, double2* __restrict__ partA, const double2* __restrict__ partB,
    double2* __restrict__ yp, int bx) {
  constexpr int QP = COL_THREADS / ROWS_A;        // threads sharing one row
  constexpr int PER = TRD_NB / QP;                // panel columns per thread
  constexpr int YCH = 8;                          // y slots loaded per round
  constexpr int HW = ROWS_A / 64;                 // wavefronts per thread group qq
  __shared__ double2 vps[ROWS_A], wps[ROWS_A], xs[ROWS_A];
  __shared__ double2 xpart[QP][ROWS_A], xpart2[QP][ROWS_A];
  __shared__ double2 vcs[TRD_NB], wcs[TRD_NB];
  static_assert(HW == 1, "one wavefront per row group: its sums are the block's partials");
  __shared__ double2 yc_s;     // y_{c-1}[c]
  __shared__ double2 yt_s;     // (S xt)[c]: row c of the unscaled product
  __shared__ double scc_s;     // S[c][c]
  __shared__ double2 svw[2 * TRD_NB];  // V^H v | W^H v of reflector c-1
  const int c = j0 + i;
  const int64_t N = n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int rbase = c + bx * ROWS_A;
  const int rr = tid % ROWS_A, qq = tid / ROWS_A;  // qq is uniform in a wavefront
  const int r = rbase + rr;
  const bool act = r < n;

  // ---- 0. issue every global load of the kernel before any arithmetic on
  // them: addresses are clamped and the values masked afterwards, so that the
  // loads go out together and are waited for once
  const double2 zero = make_double2(0.0, 0.0);
  const int rc = min(r, n - 1);
  static_assert(2 * TRD_NB == 64, "one wavefront stages V^H v | W^H v");
  double2 svl = zero, x0 = zero, xv = zero, ypr = zero;
  if (wid == 0) {
    svl = hs[HS_SVV + lane];
    x0 = M[rc + (int64_t)c * ld];
    xv = M[rc + (int64_t)max(c - 1, 0) * ld];
    ypr = (yp ? yp : (const double2*)M)[rc];
  }
  // panel reflectors 0..i-2 on this row: the correction of y_{c-1}, step 2, step 3
  const int ipmax = max(i - 2, 0);
  double2 vr[PER], wr[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int ip = min(qq + u * QP, ipmax);
    vr[u] = VW[rc + (int64_t)ip * N];
    wr[u] = VW[rc + (int64_t)(TRD_NB + ip) * N];
  }
  // y_{c-1}[r]: the previous hemv kernel's slots, QP threads per row
  const int orgp = trd_org(c);  // origin of the tiling of the hemv launch for reflector c-1
  const int nIp = i > 0 ? cdiv(n - orgp, HT) : 0;
  // pieces of tile-row Ir in the hemv launch (gprev blocks) that produced the slots
  const int Ir = (rc - orgp) / HT;
  const int64_t Tp = (int64_t)nIp * (nIp + 1) / 2, s_ir = (int64_t)Ir * (Ir + 1) / 2;
  const int nrs = Tp > 0 ? hemv_block_of(Tp, gprev, s_ir + Ir) - hemv_block_of(Tp, gprev, s_ir) + 1 : 1;
  const int tot = max(nrs + nIp - Ir, 1);
  double2 ysl[YCH];
#pragma unroll
  for (int u = 0; u < YCH; ++u) ysl[u] = Y[yslot(min(qq + u * QP, tot - 1), Ir, nrs, ycs, N, rc)];
  // the hemv blocks' partials of y^H v (wavefront 0 reduces them: only it
  // needs y^H v)
  constexpr int PB = 4;  // partials per lane issued together
  const int nun = i > 0 ? gprev : 0;  // one y^H v partial per hemv block
  double2 pbl[PB];
  if (wid == 0) {
#pragma unroll
    for (int u = 0; u < PB; ++u) pbl[u] = partB[min(lane + 64 * u, max(nun - 1, 0))];
  }
  const double2 tc = hs[HS_TAU], scal_p = hs[HS_SCAL], pdot = hs[HS_PDOT];
  // row c of the panel's earlier reflectors and the slots of y_{c-1}[c] (wavefront 1)
  constexpr int YC = 2;  // slots of row c per lane issued together
  double2 vcl = zero, wcl = zero, ycl[YC], scc = zero;
  if (wid == 1) {
    scc = hs[HS_S00];  // S[c][c] as the hemv kernel saw it (block 0 rewrites it here)
    const int ip = min(lane, ipmax);
    vcl = VW[c + (int64_t)ip * N];
    wcl = VW[c + (int64_t)(TRD_NB + ip) * N];
#pragma unroll
    for (int u = 0; u < YC; ++u) ycl[u] = Y[yslot(min(lane + 64 * u, nIp), 0, 1, ycs, N, c)];
  }

  // ---- masks and sums
  if (wid == 0 && lane % TRD_NB < i - 1) svw[lane] = svl;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const bool ok = qq + u * QP < i - 1 && act;
    vr[u] = keep(ok, vr[u]);
    wr[u] = keep(ok, wr[u]);
  }
  // y_{c-1}[r] = scal (S xt)[r] + S[r][c]: the hemv kernel multiplied the
  // unscaled reflector xt (v = scal xt + e_c); column c of S is x0
  double2 yq = zero;
  if (i > 0 && act) {
#pragma unroll
    for (int u = 0; u < YCH; ++u)
      if (qq + u * QP < tot) yq = cadd(yq, ysl[u]);
    for (int q0 = qq + YCH * QP; q0 < tot; q0 += QP)  // beyond the first round (very large n)
      yq = cadd(yq, Y[yslot(q0, Ir, nrs, ycs, N, r)]);
    yq = cmul(scal_p, yq);
    if (qq == 0) yq = cadd(yq, r == c ? make_double2(x0.x, 0.0) : x0);
  }
  double2 ycq = zero;
  if (wid == 1) {
    const bool ok = lane < i - 1;
    vcl = keep(ok, vcl);
    wcl = keep(ok, wcl);
    if (ok) {  // row c of the panel's earlier reflectors
      vcs[lane] = vcl;
      wcs[lane] = wcl;
    }
    if (i > 0) {
#pragma unroll
      for (int u = 0; u < YC; ++u)
        if (lane + 64 * u <= nIp) ycq = cadd(ycq, ycl[u]);
      for (int q = lane + 64 * YC; q <= nIp; q += 64) ycq = cadd(ycq, Y[yslot(q, 0, 1, ycs, N, c)]);
    }
  }
  double2 pa = zero;
  if (wid == 0) {
#pragma unroll
    for (int u = 0; u < PB; ++u)
      if (lane + 64 * u < nun) pa = cadd(pa, pbl[u]);
    for (int b = lane + 64 * PB; b < nun; b += 64) pa = cadd(pa, partB[b]);
  }
  __syncthreads();  // svw, vcs, wcs staged

  // ---- 1. y_{c-1} = S v - V (W^H v) - W (V^H v) and alpha; with it, step 2's
  // partial products: the panel's reflectors 0..i-2 applied to column c (they do
  // not depend on reflector c-1), QP threads per row
  double2 al = make_double2(0.0, 0.0);
  if (has_new && i > 1) {
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int ip = qq + u * QP;
      if (ip < i - 1) {
        acc = cadd(acc, cmulc(wcs[ip], vr[u]));   // v_ip[r] conj(w_ip[c])
        acc = cadd(acc, cmulc(vcs[ip], wr[u]));   // w_ip[r] conj(v_ip[c])
      }
    }
    xpart2[qq][rr] = acc;
  }
  if (i > 0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int ip = qq + u * QP;
      if (ip < i - 1 && act)
        yq = csub(yq, cadd(cmul(vr[u], svw[TRD_NB + ip]), cmul(wr[u], svw[ip])));
    }
    if (wid == ROWS_A / 64) {
      // row c: yt = (S xt)[c] (slots, unscaled); y = scal yt + S[c][c] - panel terms
      const double2 yt = wave_sum2_dpp(ycq);
      double2 corr = zero;
      if (lane < i - 1) corr = cadd(cmul(vcl, svw[TRD_NB + lane]), cmul(wcl, svw[lane]));
      corr = wave_sum2_dpp(corr);
      if (lane == 0) {
        yt_s = yt;
        scc_s = scc.x;
        yc_s = csub(cadd(cmul(scal_p, yt), make_double2(scc.x, 0.0)), corr);
      }
    }
    xpart[qq][rr] = yq;
    double2 s = zero;
    if (wid == 0) {
      // y^H v = v^H S v - panel terms, v^H S v = S[c][c] + 2 Re(scal yt[c])
      // + |scal|^2 xt^H S xt (the hemv blocks' partials sum to xt^H S xt); the
      // panel's share: -sum_ip conj(W^H v) V^H v + conj(V^H v) W^H v
      pa = cscale(pa, cabs2(scal_p));
      if (lane < i - 1) {
        const double2 sv = svw[lane], sw = svw[TRD_NB + lane];
        pa = csub(pa, cadd(cmulc(sw, sv), cmulc(sv, sw)));
      }
      s = wave_sum2_dpp(pa);
    }
    __syncthreads();  // xpart, xpart2, yc_s, yt_s and scc_s are read by wavefront 0
    if (wid == 0) {
      const double2 sy = cmul(scal_p, yt_s);
      const double t2 = cabs2(tc);
      al = make_double2(-0.5 * t2 * (s.x + scc_s + 2.0 * sy.x), -0.5 * t2 * s.y);
    }
  }

  // ---- finish reflector c-1 and update column c (row threads)
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
    if (has_new) {
      vps[rr] = vprev_r;
      wps[rr] = wprev_r;
      double2 x = make_double2(0.0, 0.0);
      bool tail = false;
      if (act) {
        x = x0;
        if (i > 1) {
#pragma unroll
          for (int q = 0; q < QP; ++q) x = csub(x, xpart2[q][rr]);
        }
        if (i > 0) {
          // reflector c-1: v[c] = 1, w[c] = tau y[c] + alpha
          const double2 wprev_c = cadd(cmul(tc, yc_s), al);
          x = sub_mulc(x, vprev_r, wprev_c);
          x = csub(x, wprev_r);
        }
        if (r == c) x.y = 0.0;
        M[r + (int64_t)c * ld] = x;
        tail = r >= c + 2;
      }
      xs[rr] = tail ? x : make_double2(0.0, 0.0);
      const double2 s0 = wave_sum2_dpp(make_double2(tail ? cabs2(x) : 0.0, 0.0));
      const double2 s1 = wave_sum2_dpp((tail && yp) ? cmulc(x, ypr) : make_double2(0.0, 0.0));
      if (has_new && lane == 0) {  // the block's |x|^2 and conj(x) y_probe
        partA[(int64_t)bx * NVAL + 0] = s0;
        partA[(int64_t)bx * NVAL + 1] = s1;
      }
    }
  }
  if (!has_new) return;
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
        // block partials, compact layout [|x|^2, conj(x) y, V^H x (i), W^H x (i)]
        if (lane == 63) {
          partA[(int64_t)bx * NVAL + 2 + ip] = pv;
          partA[(int64_t)bx * NVAL + 2 + i + ip] = pw;
        }
      }
    }
  }
}

__global__ __launch_bounds__(COL_THREADS) void k_trd_col(
    double2* __restrict__ M, int64_t ld, int n, double2* __restrict__ VW, double2* __restrict__ WV,
    int j0, int i, int has_new, const double2* __restrict__ hs, const double2* __restrict__ Y,
    int ycs, int gprev, double2* __restrict__ partA, const double2* __restrict__ partB,
    double2* __restrict__ yp) {
  trd_col_dev(M, ld, n, VW, WV, j0, i, has_new, hs, Y, ycs, gprev, partA, partB, yp,
              (int)blockIdx.x);
}

// Sum over the 16 lanes of each row of the wavefront (DPP within rows); every
// lane of a row gets its row's total.
BSE_DEV double row16_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}

// Reflector c from the column kernel's partials, then the Hermitian product
// S v over the lower triangle of the trailing matrix (rows and columns c+1..n-1)
// in HT x HT tiles.  Persistent blocks (at most one per compute unit) take
// equal runs of consecutive tiles in tile-row order, so that the most loaded
// block has at most one tile more than the mean (the launch lasts as long as
// its most loaded block).  Results are stored per tile or per piece (a
// tile-row's part of a run); each block also leaves one partial of y^H v.
// Tiles stream through three register buffers (two in flight while one is
// used) and their loads carry no conditions, so the wait for one tile never
// covers the next.  Within a piece no barrier is taken: each lane keeps its
// rows' partial sums in registers, and each tile's column sums go from the
// lanes straight to the slots.  A piece ends with one LDS reduction of its row
// sums.  Block 0 also stores the reflector; V^H v, W^H v and conj(v) y_probe
// for the next column kernel are spread over the blocks, one value each (the
// panel's share of y^H v follows from them in that kernel).  The column
// kernel's partial sums are loaded before the tile prefetch so that the
// reflector is not held up behind it.
//
// Wavefront w owns tile column 4w + l / 16 (lane l); load s of lane l reads
// row 16 s + l % 16: four contiguous 256-byte column segments per
// instruction.  A column's sum over the tile's rows is lane-local over s plus
// one 16-lane DPP reduction serving four columns.
BSE_DEV void trd_hemv_dev(
    const double2* __restrict__ M, int64_t ld, int n, const double2* __restrict__ VW, int j0,
    int i, double2* __restrict__ hs, const double2* __restrict__ partA,
    double2* __restrict__ partB, double2* __restrict__ Y, int ycs,
    double* __restrict__ dd, double* __restrict__ ee, double2* __restrict__ tau,
    const double2* __restrict__ yp, int bx, int G) {
  constexpr int NW = HV_THREADS / 64;     // 16 wavefronts
  constexpr int NL = 4;                   // matrix loads per lane per tile
  static_assert(NW * 4 == HT, "tile layout");
  struct Rec {        // one tile's loads
    double2 s[NL];    // elements (rows 16 s + lr, column jl)
    double2 xj;       // x at column jl
  };
  struct Pos {        // a tile: index in tile-row order and its (I, J)
    int64_t t;
    int I, J;
  };
  __shared__ double2 vrow[2][HT];
  __shared__ double2 rpart[NW * 4][HT];  // [wavefront x lane group][row]
  __shared__ double2 pred[NW];
  const int c = j0 + i, b0 = c + 1, org = trd_org(b0);
  const int64_t N = n;
  const int m = n - org;
  const int nI = cdiv(m, HT);
  const int64_t T = (int64_t)nI * (nI + 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;  // row in slab, column group
  const int jl = 4 * wid + lg;               // this lane's tile column
  const int nlast = n - 1;
  const int64_t t_end = hemv_tile_start(T, G, bx + 1);
  const double2* xcol = M + (int64_t)c * ld;
  const double2 zero = make_double2(0.0, 0.0);

  auto pos_of = [&](int64_t t) -> Pos {
    int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    I = ((int64_t)(I + 1) * (I + 2) / 2 <= t) ? I + 1 : I;
    I = ((int64_t)I * (I + 1) / 2 > t) ? I - 1 : I;
    return Pos{t, I, (int)(t - (int64_t)I * (I + 1) / 2)};
  };
  auto step = [&](Pos& q) {
    ++q.t;
    if (++q.J > q.I) {
      ++q.I;
      q.J = 0;
    }
  };
  // loads without conditions (indices clamped; past the run the cursor reads
  // tile (0, 0) again, which every block shares, so that the look-ahead costs
  // no memory traffic; those values are unused)
  auto load = [&](Rec& rc, const Pos& q) {
    const bool in = q.t < t_end;  // uniform
    const int rb0 = org + (in ? q.I : 0) * HT;
    const int64_t j = min(org + (in ? q.J : 0) * HT + jl, nlast);
#pragma unroll
    for (int s = 0; s < NL; ++s) rc.s[s] = M[min(rb0 + 16 * s + lr, nlast) + j * ld];
    rc.xj = xcol[j];
  };

  // ---- the small loads first, so that they are not queued behind the tile
  // prefetch of every block: x on the first tile-row's rows and, for
  // wavefront 1, the column kernel's |x|^2 partials and this block's share of
  // the other partial sums (value t = 1 + bx, + G, ...)
  const int nbA = cdiv(n - c, ROWS_A);
  const int nvals = 2 + 2 * i;
  Pos C = pos_of(hemv_tile_start(T, G, bx));
  const double2 xv0 = xcol[min(org + C.I * HT + (tid & (HT - 1)), nlast)];
  // x on the rows of the next tile-row, loaded one piece ahead of its use
  double2 xnx = xcol[min(org + (C.I + 1) * HT + lane, nlast)];
  constexpr int PQ = 4;  // partial sums per lane issued together
  double2 pq0[PQ], pq1[PQ];
  const int t0 = 1 + bx;  // first value of wavefront 1
  double2 ax = zero, vw1 = zero, yb0 = zero;
  if (wid == 1) {
    ax = xcol[b0];
    const int col1 = min(t0, NVAL - 1);
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      pq0[q] = partA[(int64_t)min(lane + 64 * q, nbA - 1) * NVAL];
      pq1[q] = partA[(int64_t)min(lane + 64 * q, nbA - 1) * NVAL + col1];
    }
    if (t0 < nvals) {
      if (t0 >= 2) {
        const int ip = (t0 - 2) % max(i, 1), w = (t0 - 2) / max(i, 1);
        vw1 = VW[b0 + (int64_t)(w * TRD_NB + ip) * N];
      } else if (yp) {
        yb0 = yp[b0];
      }
    }
  }
  Pos Lq = C;
  Rec r0, r1, r2;
  load(r0, Lq);
  step(Lq);
  load(r1, Lq);
  step(Lq);
  // The tiles multiply the unscaled reflector: v = scal xt + e_b0 with xt = x
  // below b0 and xt_b0 = 0, so S v = scal (S xt) + S e_b0.  The column kernel
  // applies scal and adds S e_b0, the column b0 of S that it reads anyway; the
  // product therefore does not wait for the reflector.
  auto vval = [&](int e, double2 x) -> double2 { return (e < n && e > b0) ? x : zero; };
  int ub = 0;  // vrow buffer of the current piece
  if (tid < HT) vrow[0][tid] = vval(org + C.I * HT + tid, xv0);
  __syncthreads();

  // ---- reflector c and the next column kernel's inputs: wavefront 1 of every
  // block, before its share of the tiles (the other wavefronts go ahead)
  if (wid == 1) {
    // sum over the column kernel's blocks of value col (lanes over blocks)
    auto colsum = [&](const double2(&pq)[PQ], int col) -> double2 {
      double2 a = zero;
#pragma unroll
      for (int q = 0; q < PQ; ++q)
        if (lane + 64 * q < nbA) a = cadd(a, pq[q]);
      for (int b = lane + 64 * PQ; b < nbA; b += 64) a = cadd(a, partA[(int64_t)b * NVAL + col]);
      return wave_sum2(a);
    };
    const double xn2 = colsum(pq0, 0).x;
    double2 tv, scal;
    double beta;
    if (xn2 == 0.0 && ax.y == 0.0) {
      tv = zero;
      beta = ax.x;
      scal = zero;
    } else {
      beta = -copysign(sqrt(ax.x * ax.x + ax.y * ax.y + xn2), ax.x);
      tv = make_double2((beta - ax.x) / beta, -ax.y / beta);
      const double2 dnm = make_double2(ax.x - beta, ax.y);
      const double q = 1.0 / cabs2(dnm);
      scal = make_double2(dnm.x * q, -dnm.y * q);
    }
    if (bx == 0 && lane == 0) {
      ee[c] = beta;
      tau[c] = tv;
      dd[c] = M[c + (int64_t)c * ld].x;
      hs[HS_SCAL] = scal;
      hs[HS_TAU] = tv;
      // S[b0][b0] for the next column kernel, which overwrites that element
      // while its other blocks would still read it
      hs[HS_S00] = make_double2(M[b0 + (int64_t)b0 * ld].x, 0.0);
    }
    const double2 s1 = (t0 < nvals) ? colsum(pq1, min(t0, NVAL - 1)) : zero;  // uniform
    // V^H v, W^H v of the panel and conj(v) y_probe: lane k takes value
    // t0 + k G (more than one only when there are fewer blocks than values,
    // i.e. for small trailing matrices)
    const int t = t0 + lane * G;
    if (t < nvals) {
      double2 st = s1, e1 = vw1, y0 = yb0;
      if (lane > 0) {
        st = zero;
        for (int b = 0; b < nbA; b += 4) {
          double2 pv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) pv[u] = partA[(int64_t)min(b + u, nbA - 1) * NVAL + t];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (b + u < nbA) st = cadd(st, pv[u]);
        }
        if (t >= 2) e1 = VW[b0 + (int64_t)(((t - 2) / i) * TRD_NB + (t - 2) % i) * N];
        else if (yp) y0 = yp[b0];
      }
      // v^H y_probe = y[c+1] + conj(scal) sum_{r >= c+2} conj(x_r) y_r
      if (t == 1) {
        if (yp) hs[HS_PDOT] = cadd(y0, cmulc(scal, st));
      } else if (t < 2 + i) {
        hs[HS_SVV + (t - 2)] = cadd(cconj(e1), cmul(scal, st));
      } else {
        hs[HS_SWV + (t - 2 - i)] = cadd(cconj(e1), cmul(scal, st));
      }
    }
  }

  double2 ra[NL] = {zero, zero, zero, zero};
  double2 pbl = zero;
  // slot of this block's piece of tile-row I: pieces are counted from the
  // block that holds the row's first tile
  auto row_slot = [&](int I) {
    return bx - hemv_block_of(T, G, (int64_t)I * (I + 1) / 2);
  };
  // cb: tile C; nb receives tile C + 2 (tile C + 1 is in flight in the third buffer)
  auto tile = [&](const Rec& cb, Rec& nb) {
    load(nb, Lq);
    step(Lq);
    const int I = C.I, J = C.J;
    const int rb0 = org + I * HT, cj0 = org + J * HT;
    const double2 vj = vval(cj0 + jl, cb.xj);
    // uniform; tiles touching the masked rows and columns take the masked path
    const bool plain = J != I && cj0 >= b0 && rb0 + HT <= n && cj0 + HT <= n;
    double2 ca = zero;
#pragma unroll
    for (int s = 0; s < NL; ++s) {
      const int rl = 16 * s + lr;
      const double2 sv = cb.s[s];
      const double2 vr = vrow[ub][rl];
      if (plain) {
        ra[s] = cadd(ra[s], cmul(sv, vj));
        ca = cadd(ca, cmulc(sv, vr));
      } else {
        const bool ok = (rb0 + rl < n) && (cj0 + jl < n) && (rb0 + rl >= b0) && (cj0 + jl >= b0) &&
                        (J != I || rl >= jl);
        const bool strict = J != I || rl > jl;
        double2 sr = ok ? sv : zero;
        if (J == I && rl == jl) sr.y = 0.0;  // the diagonal of a Hermitian matrix is real
        ra[s] = cadd(ra[s], cmul(sr, vj));
        if (ok && strict) ca = cadd(ca, cmulc(sv, vr));
      }
    }
    ca.x = row16_sum(ca.x);
    ca.y = row16_sum(ca.y);
    if (lr == 0 && cj0 + jl < n) {
      Y[(int64_t)(ycs + I) * N + cj0 + jl] = ca;
      pbl = cadd(pbl, cmulc(ca, vj));
    }
    const bool last = C.t + 1 == t_end;  // uniform
    if (J == I || last) {
      // ---- end of a piece: row sums over 64 partials (16 threads per row, then
      // a 16-lane reduction), the next tile-row's v rows, and its y^H v share
#pragma unroll
      for (int s = 0; s < NL; ++s) {
        rpart[4 * wid + lg][16 * s + lr] = ra[s];
        ra[s] = zero;
      }
      if (tid < HT && !last)  // the block goes on with tile-row I + 1
        vrow[ub ^ 1][tid] = vval(org + (I + 1) * HT + tid, xnx);
      __syncthreads();
      const int row = tid >> 4, part = tid & 15;
      double2 rs = zero;
#pragma unroll
      for (int q = 0; q < 4; ++q) rs = cadd(rs, rpart[part + 16 * q][row]);
      rs.x = row16_sum(rs.x);
      rs.y = row16_sum(rs.y);
      if (part == 0 && rb0 + row < n) {
        Y[(int64_t)row_slot(I) * N + rb0 + row] = rs;
        pbl = cadd(pbl, cmulc(rs, vrow[ub][row]));
      }
      __syncthreads();  // rpart and vrow[ub] are free again
      ub ^= 1;
      xnx = xcol[min(org + (I + 2) * HT + lane, nlast)];  // for the next piece's end
    }
    step(C);
  };
  while (C.t < t_end) {  // uniform
    tile(r0, r2);
    if (C.t >= t_end) break;
    tile(r1, r0);
    if (C.t >= t_end) break;
    tile(r2, r1);
  }
  // this block's share of y^H v
  pbl.x = wave_total63(pbl.x);
  pbl.y = wave_total63(pbl.y);
  if (lane == 63) pred[wid] = pbl;
  __syncthreads();
  if (tid == 0) {
    double2 t = zero;
#pragma unroll
    for (int w = 0; w < NW; ++w) t = cadd(t, pred[w]);
    partB[bx] = t;
  }
}

__global__ __launch_bounds__(HV_THREADS) void k_trd_hemv(
    const double2* __restrict__ M, int64_t ld, int n, const double2* __restrict__ VW, int j0,
    int i, double2* __restrict__ hs, const double2* __restrict__ partA,
    double2* __restrict__ partB, double2* __restrict__ Y, int ycs,
    double* __restrict__ dd, double* __restrict__ ee, double2* __restrict__ tau,
    const double2* __restrict__ yp) {
  trd_hemv_dev(M, ld, n, VW, j0, i, hs, partA, partB, Y, ycs, dd, ee, tau, yp, (int)blockIdx.x,
               (int)gridDim.x);
}

// ---- the same sweep over several independent problems at once: one launch
// per kernel and column step serves every problem still reducing (blockIdx.y
// selects the problem; blocks past a problem's grid return at once).  The
// kernel bodies are those of the single sweep, so with each problem's own hemv
// grid (the default) every problem gets the values it gets on its own.
// The problem that owns this block of a batched launch (a uniform scan of the
// block ranges in the kernel arguments).
BSE_DEV int batch_problem(const TrdFirst& f) {
  int p = 0;
  while (p + 1 < TRD_BATCH_MAX && (int)blockIdx.x >= f.b[p + 1]) ++p;
  return p;
}

__global__ __launch_bounds__(COL_THREADS) void k_trd_col_b(TrdBatchArgs a, TrdFirst f, int jg,
                                                           int i) {
  const int pi = batch_problem(f);
  const TrdProb p = a.p[pi];
  const int bx = (int)blockIdx.x - f.b[pi];  // block within the problem's column kernel
  const int n = p.n;
  const int j0 = jg - p.shift;  // this problem's panel at global panel step jg
  if (j0 < 0 || j0 >= n - 1) return;  // its sweep has not started or is over
  const int jb = min(TRD_NB, n - 1 - j0);
  if (i > jb) return;       // its last panel is shorter
  const int c = j0 + i;
  if (bx >= cdiv(n - c, ROWS_A)) return;
  // uniform: readfirstlane keeps it (and all index arithmetic on it) scalar
  const int gprev = __builtin_amdgcn_readfirstlane(c > 0 ? p.grids[c - 1] : 1);
  trd_col_dev(p.M, p.ld, n, p.VW, p.WV, j0, i, i < jb ? 1 : 0, p.hs, p.Y, p.ycs, gprev, p.partA,
              p.partB, p.yp, bx);
}

__global__ __launch_bounds__(HV_THREADS) void k_trd_hemv_b(TrdBatchArgs a, TrdFirst f, int jg,
                                                           int i) {
  const int pi = batch_problem(f);
  const TrdProb p = a.p[pi];
  const int bx = (int)blockIdx.x - f.b[pi];
  const int n = p.n;
  const int j0 = jg - p.shift;
  if (j0 < 0 || j0 >= n - 1 || i >= min(TRD_NB, n - 1 - j0)) return;
  const int G = f.b[pi + 1] - f.b[pi];  // the table's grid count for this step
  if (bx >= G) return;
  trd_hemv_dev(p.M, p.ld, n, p.VW, j0, i, p.hs, p.partA, p.partB, p.Y, p.ycs, p.dd, p.ee, p.tau,
               p.yp, bx, G);
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

int64_t ycs_of(int64_t n) { return (n + 63) / 64; }
int64_t hemv_tiles_max(int64_t n) {
  const int64_t nI = (n + HT - 1) / HT;  // the tiling starts at row 0 for the first column
  return nI * (nI + 1) / 2;
}

// Compute units of the current device (256 when the query fails).
int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
  }
  return cus;
}

// Blocks of a hemv launch over a trailing block of order m: one per compute
// unit, or fewer so that each takes at least the tuned number of tiles (1, 2,
// 4 or 8; fewer, longer runs can pay for small trailing matrices).
int hemv_grid(int64_t m) {
  const int cus = device_cus();
  const int64_t nI = (m + HT - 1) / HT, T = nI * (nI + 1) / 2;
  const int least = tune_choice(BSE_TUNE_HEMV_UNIT, m, 1);
  return (int)std::max<int64_t>(1, std::min<int64_t>(cus, (T + least - 1) / least));
}

}  // namespace

// [partA: column-kernel partials | partB: hemv block partials of y^H v (+ one
//  spare) | Y: hemv slots]
int64_t trd_part_elems(int64_t n) {
  const int64_t a = ((n + ROWS_A - 1) / ROWS_A + 1) * NVAL;
  return a + hemv_tiles_max(n) + 1 + 2 * ycs_of(n) * n;
}

bool tridiagonalise(double2* M, int64_t n, int64_t ld, const TrdBufs& w, int32_t* info,
                    hipStream_t s) {
  double2* partA = w.part;
  double2* partB = w.part + ((n + ROWS_A - 1) / ROWS_A + 1) * NVAL;
  double2* Y = partB + hemv_tiles_max(n) + 1;
  const int ycs = (int)ycs_of(n);
  int gprev = 1;  // blocks of the last hemv launch (read by the next column kernel)
  for (int64_t j0 = 0; j0 < n - 1; j0 += TRD_NB) {
    const int jb = (int)std::min<int64_t>(TRD_NB, n - 1 - j0);
    if (jb < TRD_NB)
      BSE_LAUNCH(k_trd_zero_cols, dim3(256), dim3(256), 0, s, w.VW, w.WV, n, jb);
    for (int i = 0; i < jb; ++i) {
      const int64_t c = j0 + i, m = n - trd_org((int)c + 1);  // order of the tiled block
      BSE_LAUNCH(k_trd_col, dim3(cdiv(n - c, ROWS_A)), dim3(COL_THREADS), 0, s, M, ld, (int)n, w.VW,
                 w.WV, (int)j0, i, 1, w.hs, Y, ycs, gprev, partA, partB, w.yproj);
      const int g = hemv_grid(m);
      BSE_LAUNCH(k_trd_hemv, dim3(g), dim3(HV_THREADS), 0, s, M, ld, (int)n, w.VW, (int)j0, i,
                 w.hs, partA, partB, Y, ycs, w.dd, w.ee, w.tau, w.yproj);
      gprev = g;
    }
    // finish the panel's last reflector
    const int64_t cl = j0 + jb;
    BSE_LAUNCH(k_trd_col, dim3(cdiv(n - cl, ROWS_A)), dim3(COL_THREADS), 0, s, M, ld, (int)n,
               w.VW, w.WV, (int)j0, jb, 0, w.hs, Y, ycs, gprev, partA, partB, w.yproj);
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
      g.tile = tune_choice(BSE_TUNE_GEMM_HER2K, n, 0);
      if (zgemm(g, 1, s) != hipSuccess) return false;
    }
  }
  BSE_LAUNCH(k_trd_last, dim3(1), dim3(64), 0, s, M, ld, (int)n, w.dd, info);
  return hipGetLastError() == hipSuccess;
}

namespace {

// Device pointers of problem `it`'s share of the partial-sum space.
void trd_parts(const TrdItem& it, double2** partA, double2** partB, double2** Y) {
  *partA = it.w.part;
  *partB = it.w.part + ((it.n + ROWS_A - 1) / ROWS_A + 1) * NVAL;
  *Y = *partB + hemv_tiles_max(it.n) + 1;
}

// Global panel step at which each problem of a group starts its sweep: 0 for
// all (BSE_TUNE_BATCH_ALIGN choice 0), or late by the largest multiple of
// TRD_NB that keeps it within the largest problem's steps (choice 1), so that
// the sweeps end together and every step reduces about the same bytes.
std::vector<int> batch_shifts(const TrdItem* it, int np) {
  int64_t nmax = 0;
  for (int p = 0; p < np; ++p) nmax = std::max(nmax, it[p].n);
  const int align = tune_choice(BSE_TUNE_BATCH_ALIGN, nmax, 0);
  std::vector<int> sh(np, 0);
  if (align == 1)
    for (int p = 0; p < np; ++p) sh[p] = (int)(((nmax - it[p].n) / TRD_NB) * TRD_NB);
  return sh;
}

// Blocks of every problem's hemv launch for its reflector c, c = 0 .. n - 2: by
// default hemv_grid() blocks, as in the problem's own sweep; in shared mode the
// launch of a global step has `per_cu` blocks per compute unit in all (at most
// one per CU per problem reducing at that step), each such problem getting a
// share proportional to its tiles (at least one, at most one per tile), so that
// all blocks take runs of about equal length.
std::vector<std::vector<int32_t>> batch_grids(const TrdItem* it, int np) {
  int64_t nmax = 0;
  for (int p = 0; p < np; ++p) nmax = std::max(nmax, it[p].n);
  const int per_cu = tune_choice(BSE_TUNE_BATCH_SWEEP, nmax, 0);
  const std::vector<int> sh = batch_shifts(it, np);
  auto tiles = [](int64_t n, int64_t c) {
    const int64_t nI = (n - trd_org((int)c + 1) + HT - 1) / HT;
    return nI * (nI + 1) / 2;
  };
  std::vector<std::vector<int32_t>> g(np);
  for (int p = 0; p < np; ++p) g[p].assign((size_t)std::max<int64_t>(it[p].n - 1, 0), 1);
  // global column cg: problem p reduces its column cg - shift_p (if it has one)
  for (int64_t cg = 0; cg + 1 < nmax; ++cg) {
    double sum = 0.0;
    int nact = 0;  // problems reducing at this step
    for (int p = 0; p < np; ++p) {
      const int64_t c = cg - sh[p];
      if (c >= 0 && c + 1 < it[p].n) {
        sum += (double)tiles(it[p].n, c);
        ++nact;
      }
    }
    // at most one block per CU per problem reducing: a problem alone keeps the
    // one-per-CU grid of its own sweep
    const double total = (double)std::min(per_cu, std::max(nact, 1)) * device_cus();
    for (int p = 0; p < np; ++p) {
      const int64_t c = cg - sh[p];
      if (c < 0 || c + 1 >= it[p].n) continue;
      const int64_t T = tiles(it[p].n, c);
      int64_t G;
      if (per_cu == 0) {
        G = hemv_grid(it[p].n - trd_org((int)c + 1));
      } else {
        G = std::llround(total * (double)T / sum);
        G = std::max<int64_t>(1, std::min(G, T));
      }
      g[p][c] = (int32_t)G;
    }
  }
  return g;
}

// The block ranges of the column-kernel and hemv launches of step (jg, i): per
// problem reducing at that step its column grid and its hemv grid, in problem
// order (compact grids: no block of a launch is idle).
struct StepGrids {
  TrdFirst col{}, hemv{};
};
StepGrids step_grids(const TrdItem* it, int np, const std::vector<std::vector<int32_t>>& grids,
                     const std::vector<int>& sh, int64_t jg, int i) {
  StepGrids g;
  int nc = 0, nh = 0;
  for (int p = 0; p < TRD_BATCH_MAX; ++p) {
    g.col.b[p] = nc;
    g.hemv.b[p] = nh;
    if (p >= np) continue;
    const int64_t n = it[p].n, j0 = jg - sh[p];
    if (j0 < 0 || j0 >= n - 1) continue;
    const int jb = (int)std::min<int64_t>(TRD_NB, n - 1 - j0);
    if (i > jb) continue;
    const int64_t c = j0 + i;
    nc += cdiv(n - c, ROWS_A);
    if (i < jb) nh += (int)grids[p][c];
  }
  g.col.b[TRD_BATCH_MAX] = nc;
  g.hemv.b[TRD_BATCH_MAX] = nh;
  return g;
}

}  // namespace

size_t trd_batch_table_bytes(const int64_t* n, int np) {
  size_t b = 0;
  for (int p = 0; p < np; ++p) b += (size_t)std::max<int64_t>(n[p], 1) * sizeof(int32_t);
  return b;
}

namespace {
// Offset (in int32 entries) of problem p's grid counts in the table.
std::vector<size_t> grid_offsets(const TrdItem* it, int np) {
  std::vector<size_t> off(np + 1, 0);
  for (int p = 0; p < np; ++p) off[p + 1] = off[p] + (size_t)std::max<int64_t>(it[p].n, 1);
  return off;
}
}  // namespace

bool trd_batch_table(const TrdItem* it, int np, void* dev, size_t bytes) {
  if (np <= 0 || !dev) return false;
  const std::vector<size_t> off = grid_offsets(it, np);
  if (bytes < off[np] * sizeof(int32_t)) return false;
  std::vector<int32_t> host(off[np], 0);
  for (int g0 = 0; g0 < np; g0 += TRD_BATCH_MAX) {  // groups as tridiagonalise_batch forms them
    const int ng = std::min(TRD_BATCH_MAX, np - g0);
    const auto grids = batch_grids(it + g0, ng);
    for (int p = 0; p < ng; ++p)
      std::copy(grids[p].begin(), grids[p].end(), host.begin() + off[g0 + p]);
  }
  return hipMemcpy(dev, host.data(), off[np] * sizeof(int32_t), hipMemcpyHostToDevice) ==
         hipSuccess;
}

bool tridiagonalise_batch(const TrdItem* it_all, int np_all, const void* dev, hipStream_t s) {
  const std::vector<size_t> off = grid_offsets(it_all, np_all);
  for (int g0 = 0; g0 < np_all; g0 += TRD_BATCH_MAX) {
    const TrdItem* it = it_all + g0;
    const int np = std::min(TRD_BATCH_MAX, np_all - g0);
    const auto grids = batch_grids(it, np);  // as written into the table
    const std::vector<int> sh = batch_shifts(it, np);
    TrdBatchArgs A{};
    int64_t nmax = 0;
    for (int p = 0; p < np; ++p) {
      const TrdItem& q = it[p];
      TrdProb& t = A.p[p];
      t.M = q.M;
      t.ld = q.ld;
      t.n = (int)q.n;
      t.ycs = (int)ycs_of(q.n);
      t.VW = q.w.VW;
      t.WV = q.w.WV;
      t.hs = q.w.hs;
      trd_parts(q, &t.partA, &t.partB, &t.Y);
      t.yp = q.w.yproj;
      t.tau = q.w.tau;
      t.dd = q.w.dd;
      t.ee = q.w.ee;
      t.grids = (const int32_t*)dev + off[g0 + p];
      t.shift = sh[p];
      nmax = std::max(nmax, q.n);
    }
    for (int64_t jg = 0; jg < nmax - 1; jg += TRD_NB) {  // global panel steps
      int jbmax = 0;
      for (int p = 0; p < np; ++p) {
        const TrdItem& q = it[p];
        const int64_t j0 = jg - sh[p];
        if (j0 < 0 || j0 >= q.n - 1) continue;
        const int jb = (int)std::min<int64_t>(TRD_NB, q.n - 1 - j0);
        jbmax = std::max(jbmax, jb);
        if (jb < TRD_NB)
          BSE_LAUNCH(k_trd_zero_cols, dim3(256), dim3(256), 0, s, q.w.VW, q.w.WV, q.n, jb);
      }
      for (int i = 0; i <= jbmax; ++i) {
        const StepGrids g = step_grids(it, np, grids, sh, jg, i);
        const int ncol = g.col.b[TRD_BATCH_MAX], nhemv = g.hemv.b[TRD_BATCH_MAX];
        if (ncol > 0)
          BSE_LAUNCH(k_trd_col_b, dim3(ncol), dim3(COL_THREADS), 0, s, A, g.col, (int)jg, i);
        if (nhemv > 0)
          BSE_LAUNCH(k_trd_hemv_b, dim3(nhemv), dim3(HV_THREADS), 0, s, A, g.hemv, (int)jg, i);
      }
      // S[t:, t:] -= [V W] [W V]^H for every problem, as one grouped GEMM per
      // tuned tile (each item with the tile the single sweep gives it)
      std::vector<ZgemmItem> up;
      std::vector<int> tiles;
      for (int p = 0; p < np; ++p) {
        const TrdItem& q = it[p];
        const int64_t j0 = jg - sh[p];
        if (j0 < 0 || j0 >= q.n - 1) continue;
        const int64_t t = j0 + std::min<int64_t>(TRD_NB, q.n - 1 - j0);
        const int64_t n = q.n;
        if (t >= n) continue;
        ZgemmItem g;
        g.M = (int)(n - t);
        g.N = (int)(n - t);
        g.K = 2 * TRD_NB;
        g.A = q.w.VW + t;
        g.a_rs = 1;
        g.a_cs = n;
        g.B = q.w.WV + t;
        g.b_rs = n;
        g.b_cs = 1;
        g.C = q.M + t + t * q.ld;
        g.c_rs = 1;
        g.c_cs = q.ld;
        g.info = q.info;
        up.push_back(g);
        tiles.push_back(tune_choice(BSE_TUNE_GEMM_HER2K, n, 0));
      }
      std::vector<char> done(up.size(), 0);
      std::vector<ZgemmItem> grp;
      for (size_t a = 0; a < up.size(); ++a) {
        if (done[a]) continue;
        grp.clear();
        for (size_t b = a; b < up.size(); ++b)
          if (!done[b] && tiles[b] == tiles[a]) {
            grp.push_back(up[b]);
            done[b] = 1;
          }
        ZgemmParams base;
        base.conjB = 1;
        base.c_uplo = 2;  // lower triangle only
        base.alpha = make_double2(-1.0, 0.0);
        base.beta = 1.0;
        base.tag = "zgemm_her2k";
        base.tile = tiles[a];
        if (zgemm_group(base, grp.data(), (int)grp.size(), s) != hipSuccess) return false;
      }
    }
    for (int p = 0; p < np; ++p)
      BSE_LAUNCH(k_trd_last, dim3(1), dim3(64), 0, s, it[p].M, it[p].ld, (int)it[p].n,
                 it[p].w.dd, it[p].info);
  }
  return hipGetLastError() == hipSuccess;
}
