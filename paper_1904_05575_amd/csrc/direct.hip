// Direct terms of the kernel (paper Sec. 4.2, eqs. wrrm and wrabar) in one
// pass per term, for pair elements given as arrays:
//   T_p[r][G'] = sum_G conj(L_p[r][G]) W[q][G][G']      (q = class of pair p)
//   blk_p[r][j] = sum_G' T_p[r][G'] Rt_p[j][G']
// and the blocks added straight into the outputs (A+B and A-B, or A).
//
// One block takes up to 64 rows of T (PPT whole pairs of one momentum-transfer
// class) and all N_G columns:
//  * the first product runs on the matrix cores (FP64, or FP32 in the
//    precision form) with complex products in three real products each
//    (Gauss: P1 = ar br, P2 = ai bi, P3 = (ar + ai)(br + bi); Re = P1 - P2,
//    Im = P3 - P1 - P2), the operands staged through LDS in chunks of 8 (16)
//    complex k with the next chunks' loads in flight in registers; in FP32
//    each chunk's products are added into FP64 sums;
//  * T then goes to LDS, 64 columns at a time, and the second product runs
//    on the vector ALU: each group of four lanes owns one (pair, j, row set)
//    and splits the G' sum four ways (reduced by DPP at the end); the right
//    operand Rt_p is read once from HBM;
//  * the finished entries are added into the outputs (column-major, ld).
// T never leaves the chip.  Requires N_G <= 128 and R <= 64 rows per pair.
#include "bse_internal.h"
#include "common.h"
#include "timing.h"

#include <type_traits>

namespace {

constexpr int DBM = 64;      // rows of T per block (whole pairs only)
constexpr int DMAXR = 8;     // rows of a pair one thread takes in the second product
constexpr int DPAD = 2;

// complex k per LDS chunk: two MFMA k-steps in FP64; in FP32 four, which is
// also the length of the FP32 partial sums added into FP64 accumulators
template <int PREC>
constexpr int dbk() { return PREC == BSE_PREC_FP32 ? 16 : 8; }

template <int PREC, int BN>
struct DSmem1 {
  using Real = typename std::conditional<PREC == BSE_PREC_FP32, float, double>::type;
  static constexpr int BK = dbk<PREC>();
  Real a_re[2][BK][DBM + DPAD], a_im[2][BK][DBM + DPAD];
  Real b_re[2][BK][BN + DPAD], b_im[2][BK][BN + DPAD];
};
struct DSmem2 {
  double2 t[DBM][64 + 1];
};
template <int PREC, int BN>
union DSmem {
  DSmem1<PREC, BN> s1;
  DSmem2 s2;
};

typedef float f4 __attribute__((ext_vector_type(4)));

// quad sum by DPP (lanes 4i .. 4i+3), every lane of the quad gets the total
template <int CTRL>
BSE_DEV double dpp_q(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
BSE_DEV double quad_sum(double v) {
  v += dpp_q<0xB1>(v);  // quad_perm [1,0,3,2]
  v += dpp_q<0x4E>(v);  // quad_perm [2,3,0,1]
  return v;
}

BSE_DEV int pair_row(int p, int nk) {  // ik of pair p = ik*nk - ik(ik-1)/2 + (jk - ik)
  int lo = 0, hi = nk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t start = (int64_t)mid * nk - (int64_t)mid * (mid - 1) / 2;
    if (start <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// WM x WN wavefronts; each wave TI x TJ tiles of 16 x 16 (WM*TI*16 = 64,
// WN*TJ*16 = BN).  ra = 0: resonant term (left Mvv, right Mcc); ra = 1:
// coupling term (left Ncv, right Nvc).  PREC: FP64, or FP32 (operands
// rounded to FP32, FP32 products summed over 16 complex k, FP64 across).
template <int PREC, int WM, int WN, int TI, int TJ, int BN, bool TOUT>
__global__ __launch_bounds__(WM* WN * 64) void k_direct_fused(
    const double2* __restrict__ Left, const double2* __restrict__ Right, int R, int N2, int ng,
    int nk, int nv, int nc, const double2* __restrict__ W, const int32_t* __restrict__ perm,
    const int32_t* __restrict__ cls, int tiles_per_class, int ra, double coef,
    double2* __restrict__ out0, double2* __restrict__ out1, int64_t ld, double2* __restrict__ Tout,
    const int32_t* info) {
  static_assert(WM * TI * 16 == DBM && WN * TJ * 16 == BN, "tile shape");
  constexpr bool F32 = PREC == BSE_PREC_FP32;
  using Real = typename DSmem1<PREC, BN>::Real;
  constexpr int DBK = dbk<PREC>();
  constexpr int NT = WM * WN * 64;
  constexpr int NA = DBM * DBK / NT > 0 ? DBM * DBK / NT : 1;   // A complex per thread
  constexpr int NB = DBK * BN / NT > 0 ? DBK * BN / NT : 1;     // B complex per thread
  static_assert(NA * NT >= DBM * DBK && NB * NT >= DBK * BN, "staging");
  __shared__ DSmem<PREC, BN> sm;
  if (failed(info)) return;
  const int q = blockIdx.x / tiles_per_class, mt = blockIdx.x % tiles_per_class;
  const int ppt = DBM / R;                   // whole pairs per block
  const int s0 = cls[q], np = cls[q + 1] - s0;
  const int pos0 = mt * ppt;                 // first pair (position in class q)
  if (pos0 >= np) return;
  const int npb = min(ppt, np - pos0);       // pairs of this block
  const int rows = npb * R;
  const double2* __restrict__ Wq = W + (int64_t)q * ng * ng;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm0 = (wid % WM) * (TI * 16), wn0 = (wid / WM) * (TJ * 16);

  // ---- first product (matrix cores, 3 real products per complex one)
  // A staging: element e -> (row mm = e / DBK, k = e % DBK): DBK threads read
  // DBK consecutive k of one row (contiguous bytes)
  const double2* arow[NA];
  bool aok[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int e = tid + NT * u;
    const int mm = e / DBK;
    aok[u] = e < DBM * DBK && mm < rows;
    const int m = aok[u] ? mm : 0;
    const int64_t p = perm[s0 + pos0 + m / R];
    arow[u] = Left + (p * R + m % R) * ng;
  }
  double2 ra0[NA], rb0[NB], ra1[NA], rb1[NB];
  auto fetch = [&](double2 (&ra_)[NA], double2 (&rb_)[NB], int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int k = k0 + (tid + NT * u) % DBK;
      ra_[u] = arow[u][k < ng ? k : ng - 1];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + NT * u;
      const int kk = e / BN, nn = e % BN;
      const int k = k0 + kk;
      rb_[u] = Wq[(int64_t)(k < ng ? k : ng - 1) * ng + (nn < ng ? nn : ng - 1)];
    }
  };
  auto put = [&](int buf, const double2 (&ra_)[NA], const double2 (&rb_)[NB], int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + NT * u;
      if (e < DBM * DBK) {
        const int mm = e / DBK, kk = e % DBK;
        const bool ok = aok[u] && k0 + kk < ng;
        sm.s1.a_re[buf][kk][mm] = ok ? (Real)ra_[u].x : (Real)0;
        sm.s1.a_im[buf][kk][mm] = ok ? (Real)(-ra_[u].y) : (Real)0;  // conj(L)
      }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + NT * u;
      if (e < DBK * BN) {
        const int kk = e / BN, nn = e % BN;
        const bool ok = k0 + kk < ng && nn < ng;
        sm.s1.b_re[buf][kk][nn] = ok ? (Real)rb_[u].x : (Real)0;
        sm.s1.b_im[buf][kk][nn] = ok ? (Real)rb_[u].y : (Real)0;
      }
    }
  };
  // FP64: the three products accumulate for the whole K; FP32: per chunk,
  // then added into the FP64 real and imaginary parts of T
  d4 p1[TI][TJ], p2[TI][TJ], p3[TI][TJ];
  d4 tre[TI][TJ], tim[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
      p1[i][j] = p2[i][j] = p3[i][j] = tre[i][j] = tim[i][j] = d4{0, 0, 0, 0};
  auto mma = [&](int buf, int k0) {
    if constexpr (F32) {
      f4 c1[TI][TJ], c2[TI][TJ], c3[TI][TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) c1[i][j] = c2[i][j] = c3[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < DBK / 4; ++ks) {
        if (k0 + ks * 4 < ng) {
          const int kr = ks * 4 + (lane >> 4);
          float ar[TI], ai[TI], as[TI], br[TJ], bi[TJ], bs[TJ];
#pragma unroll
          for (int i = 0; i < TI; ++i) {
            ar[i] = sm.s1.a_re[buf][kr][wm0 + i * 16 + (lane & 15)];
            ai[i] = sm.s1.a_im[buf][kr][wm0 + i * 16 + (lane & 15)];
            as[i] = ar[i] + ai[i];
          }
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
            br[j] = sm.s1.b_re[buf][kr][wn0 + j * 16 + (lane & 15)];
            bi[j] = sm.s1.b_im[buf][kr][wn0 + j * 16 + (lane & 15)];
            bs[j] = br[j] + bi[j];
          }
#pragma unroll
          for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
              c1[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[i], br[j], c1[i][j], 0, 0, 0);
              c2[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[i], bi[j], c2[i][j], 0, 0, 0);
              c3[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[i], bs[j], c3[i][j], 0, 0, 0);
            }
        }
      }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            tre[i][j][r] += (double)(c1[i][j][r] - c2[i][j][r]);
            tim[i][j][r] += (double)(c3[i][j][r] - c1[i][j][r] - c2[i][j][r]);
          }
    } else {
#pragma unroll
      for (int ks = 0; ks < DBK / 4; ++ks) {
        if (k0 + ks * 4 < ng) {
          const int kr = ks * 4 + (lane >> 4);
          double ar[TI], ai[TI], as[TI], br[TJ], bi[TJ], bs[TJ];
#pragma unroll
          for (int i = 0; i < TI; ++i) {
            ar[i] = sm.s1.a_re[buf][kr][wm0 + i * 16 + (lane & 15)];
            ai[i] = sm.s1.a_im[buf][kr][wm0 + i * 16 + (lane & 15)];
            as[i] = ar[i] + ai[i];
          }
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
            br[j] = sm.s1.b_re[buf][kr][wn0 + j * 16 + (lane & 15)];
            bi[j] = sm.s1.b_im[buf][kr][wn0 + j * 16 + (lane & 15)];
            bs[j] = br[j] + bi[j];
          }
#pragma unroll
          for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int j = 0; j < TJ; ++j) {
              p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], p1[i][j], 0, 0, 0);
              p2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bi[j], p2[i][j], 0, 0, 0);
              p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(as[i], bs[j], p3[i][j], 0, 0, 0);
            }
        }
      }
    }
  };
  const int nch = (ng + DBK - 1) / DBK;
  fetch(ra0, rb0, 0);
  put(0, ra0, rb0, 0);
  if (nch > 1) fetch(ra1, rb1, DBK);
  if (nch > 2) fetch(ra0, rb0, 2 * DBK);
  __syncthreads();
  // step ch: multiply chunk ch, stage chunk ch + 1 (held in `cur`) into the
  // other buffer, then reuse `cur` for the loads of chunk ch + 3
  auto step = [&](int ch, double2 (&ra_)[NA], double2 (&rb_)[NB]) {
    mma(ch & 1, ch * DBK);
    if (ch + 1 < nch) put((ch + 1) & 1, ra_, rb_, (ch + 1) * DBK);
    __syncthreads();
    if (ch + 3 < nch) fetch(ra_, rb_, (ch + 3) * DBK);
  };
  for (int ch = 0; ch < nch; ch += 2) {
    step(ch, ra1, rb1);
    if (ch + 1 < nch) step(ch + 1, ra0, rb0);
  }

  // FP64: T = P1 - P2 + i (P3 - P1 - P2); the three products are dead after this
  if constexpr (!F32) {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          tre[i][j][r] = p1[i][j][r] - p2[i][j][r];
          tim[i][j][r] = p3[i][j][r] - p1[i][j][r] - p2[i][j][r];
        }
  }
  // row of accumulator register r (f64: l/16 + 4r; f32: 4 (l/16) + r)
  auto acc_row = [&](int r) { return F32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r; };
  if constexpr (TOUT) {
    // first product only: T of the class's rows, [row][G'], for a separate
    // second pass
    double2* __restrict__ Tq = Tout + ((int64_t)s0 + pos0) * R * ng;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = wm0 + i * 16 + acc_row(r), n = wn0 + j * 16 + (lane & 15);
          if (m < rows && n < ng) Tq[(int64_t)m * ng + n] = make_double2(tre[i][j][r], tim[i][j][r]);
        }
    return;
  }

  // ---- second product (vector ALU), 64 columns of T at a time
  // item = ((pp * N2 + j) * RS + rs) * 4 + g4: pair pp of the block, right
  // index j, row set rs (DMAXR rows at most), quarter g4 of each 64-column
  // phase (G' = 64 ph + 4 gg + g4); the items go in rounds of NT
  const int RS = (R + DMAXR - 1) / DMAXR;
  const int rpt = (R + RS - 1) / RS;
  const int nitems = ppt * N2 * RS * 4;
  constexpr int NPH = BN / 64;
  const int nvnc = nv * nc;
  for (int base = 0; base < nitems; base += NT) {
    const int item = base + tid;
    const int g4 = item & 3;
    const int rs = (item >> 2) % RS;
    const int jj = (item >> 2) / RS % N2;
    const int pp = (item >> 2) / RS / N2;
    const int r0 = rs * rpt;
    const bool own = item < nitems && pp < npb;  // the same for the four lanes of a quad
    const double2* __restrict__ rt = Right;
    if (own) rt = Right + ((int64_t)perm[s0 + pos0 + pp] * N2 + jj) * ng;
    double2 acc[DMAXR];
#pragma unroll
    for (int r = 0; r < DMAXR; ++r) acc[r] = make_double2(0.0, 0.0);
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph) {
      // waves holding columns [64 ph, 64 ph + 64) store their part of T
      if (wn0 >= 64 * ph && wn0 < 64 * (ph + 1)) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int m = wm0 + i * 16 + acc_row(r);
              const int n = wn0 - 64 * ph + j * 16 + (lane & 15);
              sm.s2.t[m][n] = make_double2(tre[i][j][r], tim[i][j][r]);
            }
      }
      __syncthreads();
      if (own) {
#pragma unroll 4
        for (int gg = 0; gg < 16; ++gg) {
          const int gl = 4 * gg + g4, g = 64 * ph + gl;
          if (g < ng) {
            const double2 m = rt[g];
#pragma unroll
            for (int r = 0; r < DMAXR; ++r)
              if (r < rpt && r0 + r < R) {
                const double2 t = sm.s2.t[pp * R + r0 + r][gl];
                acc[r].x = fma(t.x, m.x, fma(-t.y, m.y, acc[r].x));
                acc[r].y = fma(t.x, m.y, fma(t.y, m.x, acc[r].y));
              }
          }
        }
      }
      __syncthreads();
    }
    // quad reduction: every lane of the block takes part
#pragma unroll
    for (int r = 0; r < DMAXR; ++r) {
      acc[r].x = quad_sum(acc[r].x);
      acc[r].y = quad_sum(acc[r].y);
    }
    if (own && g4 == 0) {
      const int p = perm[s0 + pos0 + pp];
      const int ik = pair_row(p, nk);
      const int jk = ik + (int)(p - ((int64_t)ik * nk - (int64_t)ik * (ik - 1) / 2));
#pragma unroll
      for (int r = 0; r < DMAXR; ++r) {
        if (r >= rpt || r0 + r >= R) continue;
        const int rr = r0 + r;
        int v, c, v2, c2;
        if (!ra) {  // rows (v, v'), columns j = (c, c')
          v = rr / nv; v2 = rr % nv; c = jj / nc; c2 = jj % nc;
        } else {    // rows (c, v'), columns j = (v, c')
          c = rr / nv; v2 = rr % nv; v = jj / nc; c2 = jj % nc;
        }
        const int64_t row = (int64_t)ik * nvnc + v * nc + c;
        const int64_t col = (int64_t)jk * nvnc + v2 * nc + c2;
        const double2 val = cscale(acc[r], coef);
        double2* d0 = out0 + row + col * ld;
        const double2 o = *d0;
        *d0 = make_double2(o.x + val.x, o.y + val.y);
        if (out1) {
          double2* d1 = out1 + row + col * ld;
          if (!ra) {
            *d1 = val;  // the resonant term writes A-B first
          } else {
            const double2 o1 = *d1;
            *d1 = make_double2(o1.x - val.x, o1.y - val.y);
          }
        }
      }
    }
  }
}

template <int PREC, int WM, int WN, int TI, int TJ, int BN>
void launch(const double2* left, const double2* right, int R, int N2, int ng, int nk, int nv,
            int nc, const double2* W, const int32_t* perm, const int32_t* cls, int nq, int ra,
            double coef, double2* out0, double2* out1, int64_t ld, double2* Tout,
            const int32_t* info, hipStream_t s) {
  const int ppt = DBM / R;
  const int tiles = cdiv(nk, ppt);  // a class holds at most nk pairs
  if (Tout)
    BSE_LAUNCH((k_direct_fused<PREC, WM, WN, TI, TJ, BN, true>), dim3((unsigned)(nq * tiles)),
               dim3(WM * WN * 64), 0, s, left, right, R, N2, ng, nk, nv, nc, W, perm, cls, tiles,
               ra, coef, out0, out1, ld, Tout, info);
  else
    BSE_LAUNCH((k_direct_fused<PREC, WM, WN, TI, TJ, BN, false>), dim3((unsigned)(nq * tiles)),
               dim3(WM * WN * 64), 0, s, left, right, R, N2, ng, nk, nv, nc, W, perm, cls, tiles,
               ra, coef, out0, out1, ld, Tout, info);
}

template <int PREC>
void dispatch(int variant, const double2* left, const double2* right, int R, int N2, int ng,
              int nk, int nv, int nc, const double2* W, const int32_t* perm, const int32_t* cls,
              int nq, int ra, double coef, double2* out0, double2* out1, int64_t ld,
              double2* Tout, const int32_t* info, hipStream_t s) {
#define BSE_DIRECT_ARGS left, right, R, N2, ng, nk, nv, nc, W, perm, cls, nq, ra, coef, out0, out1, ld, Tout, info, s
  if (ng <= 64) {
    if (variant == 1) launch<PREC, 4, 2, 1, 2, 64>(BSE_DIRECT_ARGS);
    else launch<PREC, 2, 2, 2, 2, 64>(BSE_DIRECT_ARGS);
  } else {
    if (variant == 1) launch<PREC, 4, 4, 1, 2, 128>(BSE_DIRECT_ARGS);
    else if (variant == 2) launch<PREC, 4, 2, 1, 4, 128>(BSE_DIRECT_ARGS);
    else launch<PREC, 2, 4, 2, 2, 128>(BSE_DIRECT_ARGS);
  }
#undef BSE_DIRECT_ARGS
}

// ---- First product alone, T = conj(L) W(q), with no padding of N_G on the
// matrix cores.  A block takes 64 consecutive rows of its class (pairs may
// straddle blocks: T's rows are independent), so no row slot is left empty
// except at the end of a class, and all N_G columns: NCT 16-column tiles on
// the matrix cores (Gauss's three real products), the columns past 16 NCT (VC,
// at most 3) and the k past the last multiple of 4 (at most 3) on the vector
// ALU.  4 wavefronts, wavefront w taking row tile w across all NCT column
// tiles (7 x 3 accumulator tiles at N_G = 113, so two wavefronts per SIMD, one
// from each of two blocks); the next chunk of operands is in flight in
// registers while one is multiplied.  (Dealing the tiles of one class to one
// XCD, for W(q) to stay in its L2, was measured slower: the blocks are
// handed out in order, and XCDs that finish their tiles early wait for the
// others.)
constexpr int FP_BM = 64;
constexpr int FP_BK = 8;

template <int NCT>
struct FpSmem {
  static constexpr int BW = NCT * 16 + 4;  // staged W columns
  double a_re[2][FP_BK][FP_BM + 2], a_im[2][FP_BK][FP_BM + 2];  // conj(L), [k][row]
  double b_re[2][FP_BK][BW + 2], b_im[2][FP_BK][BW + 2];        // W, [k][column]
  double2 ltail[3][FP_BM];                                      // conj(L[m][KF + t])
  double2 wtail[3][BW];                                         // W[KF + t][n]
  double2 vpart[4][FP_BM][3];                                   // vector-ALU columns, per k quarter
};

template <int NCT, int VC>
__global__ __launch_bounds__(256, 2) void k_first_product(
    const double2* __restrict__ Left, int R, int ng, const double2* __restrict__ W,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ cls, int nq, int spc,
    double2* __restrict__ Tout, const int32_t* info) {
  using S = FpSmem<NCT>;
  constexpr int BW = S::BW;
  constexpr int NA = FP_BM * FP_BK / 256;
  constexpr int NB = (FP_BK * BW + 255) / 256;
  __shared__ S sm;
  if (failed(info)) return;
  const int q = blockIdx.x / spc, sl = blockIdx.x % spc;
  if (q >= nq) return;
  const int s0 = cls[q], nr = (cls[q + 1] - s0) * R;
  const int m0 = sl * FP_BM;
  if (m0 >= nr) return;
  const int rows = min(FP_BM, nr - m0);
  const int KF = ng & ~3, remk = ng & 3;
  const double2* __restrict__ Wq = W + (int64_t)q * ng * ng;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = wid * 16;

  auto row_ptr = [&](int mm) {
    const int gm = m0 + mm, pos = gm / R;
    return Left + ((int64_t)perm[s0 + pos] * R + (gm - pos * R)) * ng;
  };
  const double2* arow[NA];
  bool aok[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int mm = (tid + 256 * u) >> 3;
    aok[u] = mm < rows;
    arow[u] = row_ptr(aok[u] ? mm : 0);
  }
  // K tail and the W rows it takes
  for (int e = tid; e < 3 * FP_BM; e += 256) {
    const int t = e / FP_BM, mm = e % FP_BM;
    double2 v = make_double2(0.0, 0.0);
    if (t < remk && mm < rows) v = row_ptr(mm)[KF + t];
    sm.ltail[t][mm] = make_double2(v.x, -v.y);
  }
  for (int e = tid; e < 3 * BW; e += 256) {
    const int t = e / BW, n = e % BW;
    sm.wtail[t][n] = (t < remk && n < ng) ? Wq[(int64_t)(KF + t) * ng + n] : make_double2(0.0, 0.0);
  }

  double2 ra[NA], rb[NB];  // the next chunk
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int k = k0 + ((tid + 256 * u) & 7);
      ra[u] = arow[u][k < KF ? k : 0];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + 256 * u;
      const int kk = e / BW, n = e % BW;
      const int k = k0 + kk;
      rb[u] = Wq[(int64_t)(k < KF ? k : 0) * ng + (n < ng ? n : 0)];
    }
  };
  auto put = [&](int buf, int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int e = tid + 256 * u;
      const int mm = e >> 3, kk = e & 7;
      const bool ok = aok[u] && k0 + kk < KF;
      sm.a_re[buf][kk][mm] = ok ? ra[u].x : 0.0;
      sm.a_im[buf][kk][mm] = ok ? -ra[u].y : 0.0;  // conj(L)
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int e = tid + 256 * u;
      if (e < FP_BK * BW) {
        const int kk = e / BW, n = e % BW;
        const bool ok = k0 + kk < KF && n < ng;
        sm.b_re[buf][kk][n] = ok ? rb[u].x : 0.0;
        sm.b_im[buf][kk][n] = ok ? rb[u].y : 0.0;
      }
    }
  };
  d4 p1[NCT], p2[NCT], p3[NCT];
#pragma unroll
  for (int j = 0; j < NCT; ++j) p1[j] = p2[j] = p3[j] = d4{0, 0, 0, 0};
  // vector-ALU columns 16 NCT + c: thread (row lane, k quarter wid)
  double2 vacc[VC > 0 ? VC : 1];
#pragma unroll
  for (int c = 0; c < (VC > 0 ? VC : 1); ++c) vacc[c] = make_double2(0.0, 0.0);
  auto mma = [&](int buf, int k0) {
#pragma unroll
    for (int ks = 0; ks < FP_BK / 4; ++ks) {
      if (k0 + ks * 4 < KF) {
        const int kr = ks * 4 + (lane >> 4);
        const double ar = sm.a_re[buf][kr][wm0 + (lane & 15)];
        const double ai = sm.a_im[buf][kr][wm0 + (lane & 15)];
        const double as = ar + ai;
#pragma unroll
        for (int j = 0; j < NCT; ++j) {
          const int n = j * 16 + (lane & 15);
          const double br = sm.b_re[buf][kr][n];
          const double bi = sm.b_im[buf][kr][n];
          p1[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, p1[j], 0, 0, 0);
          p2[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, p2[j], 0, 0, 0);
          p3[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, br + bi, p3[j], 0, 0, 0);
        }
      }
    }
    if constexpr (VC > 0) {
#pragma unroll
      for (int kq = 0; kq < 2; ++kq) {
        const int kk = wid * 2 + kq;
        const double xr = sm.a_re[buf][kk][lane], xi = sm.a_im[buf][kk][lane];
#pragma unroll
        for (int c = 0; c < VC; ++c) {
          const double yr = sm.b_re[buf][kk][16 * NCT + c], yi = sm.b_im[buf][kk][16 * NCT + c];
          vacc[c].x = fma(xr, yr, fma(-xi, yi, vacc[c].x));
          vacc[c].y = fma(xr, yi, fma(xi, yr, vacc[c].y));
        }
      }
    }
  };
  const int nch = (KF + FP_BK - 1) / FP_BK;
  if (nch > 0) {
    fetch(0);
    put(0, 0);
    if (nch > 1) fetch(FP_BK);
  }
  __syncthreads();
  for (int ch = 0; ch < nch; ++ch) {
    mma(ch & 1, ch * FP_BK);
    if (ch + 1 < nch) put((ch + 1) & 1, (ch + 1) * FP_BK);
    __syncthreads();
    if (ch + 2 < nch) fetch((ch + 2) * FP_BK);
  }

  double2* __restrict__ Tq = Tout + ((int64_t)s0 * R + m0) * ng;
  if constexpr (VC > 0) {
#pragma unroll
    for (int c = 0; c < VC; ++c) sm.vpart[wid][lane][c] = vacc[c];
  }
  // matrix-core columns: T = P1 - P2 + i (P3 - P1 - P2), plus the K tail
#pragma unroll
  for (int j = 0; j < NCT; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = wm0 + (lane >> 4) + 4 * r, n = j * 16 + (lane & 15);
      double2 v = make_double2(p1[j][r] - p2[j][r], p3[j][r] - p1[j][r] - p2[j][r]);
      for (int t = 0; t < remk; ++t) v = cadd(v, cmul(sm.ltail[t][m], sm.wtail[t][n]));
      if (m < rows && n < ng) Tq[(int64_t)m * ng + n] = v;
    }
  if constexpr (VC > 0) {
    __syncthreads();
    if (tid < FP_BM * VC) {
      const int m = tid & 63, c = tid >> 6;
      double2 v = make_double2(0.0, 0.0);
#pragma unroll
      for (int kq = 0; kq < 4; ++kq) v = cadd(v, sm.vpart[kq][m][c]);
      for (int t = 0; t < remk; ++t) v = cadd(v, cmul(sm.ltail[t][m], sm.wtail[t][16 * NCT + c]));
      if (m < rows) Tq[(int64_t)m * ng + 16 * NCT + c] = v;
    }
  }
}

template <int NCT, int VC>
void launch_fp(const double2* left, int R, int ng, int nk, const double2* W, const int32_t* perm,
               const int32_t* cls, int nq, double2* Tout, const int32_t* info, hipStream_t s) {
  const int spc = (int)cdiv((int64_t)nk * R, FP_BM);  // a class holds at most nk pairs
  BSE_LAUNCH((k_first_product<NCT, VC>), dim3((unsigned)((int64_t)nq * spc)), dim3(256), 0, s,
             left, R, ng, W, perm, cls, nq, spc, Tout, info);
}

// ---- The same product with the operand chunks copied from memory straight
// into LDS (global_load_lds, 16 bytes per lane: lane l's bytes land at the
// instruction's LDS base + 16 l), FP_NS chunks in flight, so that no register
// holds a chunk in transit.  4 wavefronts, each one 16-row tile across the NCT
// column tiles.  Layout of a chunk in LDS:
//  * L: 8 blocks of 8 rows x 8 k, slot(row, k) = 64 (row / 8) + 8 (row % 8) +
//    (k ^ row % 8): one load instruction fills a block (each row's 8 k are 128
//    contiguous bytes in memory), and the 16 rows x 1 k a matrix-core operand
//    takes hit distinct banks;
//  * W: [k][n] over the 16 NCT matrix-core columns.
// The conjugate of L is folded into the products: with Q2 = sum Li Wi and
// P3 = sum (Lr - Li)(Wr + Wi), T = P1 + Q2 + i (P3 - P1 + Q2).
constexpr int FP_NS = 3;
typedef __attribute__((address_space(3))) void lds_void_t;

constexpr int DF_MAXP = 7;  // pairs per block in the one-pass form (R >= 9)

template <int NCT>
struct Fp2Smem {
  static constexpr int BN = NCT * 16;
  union {
    struct {  // first product
      double2 a[FP_NS][FP_BM * FP_BK];
      double2 b[FP_NS][FP_BK * BN];
      double2 wcol[116][3];  // W[k][16 NCT + c]: the vector-ALU columns, all k
      double2 ltail[3][FP_BM];  // conj(L[m][KF + t])
    } s1;
    struct {  // second product of the one-pass form
      double2 t[FP_BM][17];            // T of one 16-column phase, [row][g]
      double2 rt[2][DF_MAXP][256];     // R_p[j][g] of the phase, g swizzled by j
      double2 dummy[64];
    } s2;
  };
};

template <int N>
BSE_DEV void wait_vmcnt() {  // s_waitcnt vmcnt(N), other counters untouched
  static_assert(N >= 0 && N < 64, "vmcnt");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// The compiler cannot tell which LDS bytes a copy in flight writes, so its own
// LDS reads and barriers wait for every copy (vmcnt(0)), which would stall each
// chunk on the loads of the chunks behind it.  Reads of the chunk buffers and
// the barrier between chunks are therefore written out, each read block ending
// with its own wait; the vmcnt waits are explicit (wait_vmcnt).
typedef double d2v __attribute__((ext_vector_type(2)));
BSE_DEV unsigned lds_off(const void* p) { return (unsigned)(uintptr_t)p; }  // low 32 bits
BSE_DEV void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
BSE_DEV d2v lds_read1(unsigned a) {
  d2v x;
  asm volatile("ds_read_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(x) : "v"(a) : "memory");
  return x;
}
// x at ax; y[j] at ab + 256 j (the seven 16-column tiles of one k).  The
// outputs are early-clobber: a read's destination must not be an address
// register that a later read of the block still takes.
BSE_DEV void lds_read_x_y7(d2v& x, d2v (&y)[7], unsigned ax, unsigned ab) {
  asm volatile(
      "ds_read_b128 %0, %8\n\t"
      "ds_read_b128 %1, %9\n\t"
      "ds_read_b128 %2, %9 offset:256\n\t"
      "ds_read_b128 %3, %9 offset:512\n\t"
      "ds_read_b128 %4, %9 offset:768\n\t"
      "ds_read_b128 %5, %9 offset:1024\n\t"
      "ds_read_b128 %6, %9 offset:1280\n\t"
      "ds_read_b128 %7, %9 offset:1536\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(x), "=&v"(y[0]), "=&v"(y[1]), "=&v"(y[2]), "=&v"(y[3]), "=&v"(y[4]), "=&v"(y[5]),
        "=&v"(y[6])
      : "v"(ax), "v"(ab)
      : "memory");
}

// FUSED = false: T written to Tout in class order (blocks of 64 rows).
// FUSED = true: blocks of whole pairs (ppt = 64 / R, R >= 9), and the second
// product follows on the matrix cores, 16 columns of T at a time: each
// wavefront puts its T tile of the phase into LDS, the block's pairs' second
// operands R_p[j][g] of the phase arrive by LDS copies (wavefront w owns pairs
// w and w + 4, and copies their rows for the next phase while multiplying
// this one), and blk_p = T_p R_p^T runs as one 16 x 16 Gauss tile per pair
// (rows r < R, columns j < N2 <= 16).  The blocks are then added into the
// outputs: out0 += coef blk, and out1 = coef blk (resonant) or out1 -= coef
// blk (coupling).  T never reaches memory.
// o[i] at a[i] (four reads, one wait)
BSE_DEV void lds_read_4(d2v (&o)[4], unsigned a0, unsigned a1, unsigned a2, unsigned a3) {
  asm volatile(
      "ds_read_b128 %0, %4\n\t"
      "ds_read_b128 %1, %5\n\t"
      "ds_read_b128 %2, %6\n\t"
      "ds_read_b128 %3, %7\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3])
      : "v"(a0), "v"(a1), "v"(a2), "v"(a3)
      : "memory");
}

// a[ks] at aa + 64 ks, b[ks] at ab[ks], ks = 0..3 (early-clobber outputs, as above)
BSE_DEV void lds_read_4x2(d2v (&a)[4], d2v (&b)[4], unsigned aa, const unsigned (&ab)[4]) {
  asm volatile(
      "ds_read_b128 %0, %8\n\t"
      "ds_read_b128 %1, %8 offset:64\n\t"
      "ds_read_b128 %2, %8 offset:128\n\t"
      "ds_read_b128 %3, %8 offset:192\n\t"
      "ds_read_b128 %4, %9\n\t"
      "ds_read_b128 %5, %10\n\t"
      "ds_read_b128 %6, %11\n\t"
      "ds_read_b128 %7, %12\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a[0]), "=&v"(a[1]), "=&v"(a[2]), "=&v"(a[3]), "=&v"(b[0]), "=&v"(b[1]),
        "=&v"(b[2]), "=&v"(b[3])
      : "v"(aa), "v"(ab[0]), "v"(ab[1]), "v"(ab[2]), "v"(ab[3])
      : "memory");
}

template <int NCT, int VC, bool FUSED, int PREC = BSE_PREC_FP64>
__global__ __launch_bounds__(256, 2) void k_first_product2(
    const double2* __restrict__ Left, int R, int ng, const double2* __restrict__ W,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ cls, int nq, int spc,
    double2* __restrict__ Tout, const int32_t* info, const double2* __restrict__ Right, int N2,
    int nk, int nv, int nc, int ra, double coef, double2* __restrict__ out0,
    double2* __restrict__ out1, int64_t ld, const int32_t* __restrict__ tmap) {
  using S = Fp2Smem<NCT>;
  constexpr int BN = S::BN;
  static_assert(NCT <= 7 && FP_NS == 3, "shape");
  __shared__ S sm;
  if (failed(info)) return;
  int q, sl;
  if (tmap) {  // the occupied tiles only, class by class
    const int v = tmap[blockIdx.x];
    if (v < 0) return;
    q = v & 8191;
    sl = v >> 13;
  } else {
    q = blockIdx.x / spc;
    sl = blockIdx.x % spc;
  }
  if (q >= nq) return;
  const int s0 = cls[q], nr = (cls[q + 1] - s0) * R;
  const int ppt = FUSED ? FP_BM / R : 0;
  const int m0 = FUSED ? sl * ppt * R : sl * FP_BM;
  if (m0 >= nr) return;
  const int rows = min(FUSED ? ppt * R : FP_BM, nr - m0);
  const int KF = ng & ~3, remk = ng & 3;
  const double2* __restrict__ Wq = W + (int64_t)q * ng * ng;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = wid * 16;

  auto row_ptr = [&](int mm) {
    const int gm = m0 + mm, pos = gm / R;
    return Left + ((int64_t)perm[s0 + pos] * R + (gm - pos * R)) * ng;
  };
  // the two L blocks this wavefront loads: rows 8 (2 wid + i) + lane / 8
  const double2* arow[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int mm = 8 * (2 * wid + i) + (lane >> 3);
    arow[i] = row_ptr(mm < rows ? mm : 0);
  }
  const int ka = (lane & 7) ^ (lane >> 3);  // k of the chunk this lane loads
  // vector-ALU columns and the K tail (plain loads, done before any copy to LDS)
  if constexpr (VC > 0)
    for (int e = tid; e < ng * VC; e += 256) {
      const int k = e / VC, c = e % VC;
      sm.s1.wcol[k][c] = Wq[(int64_t)k * ng + 16 * NCT + c];
    }
  for (int e = tid; e < 3 * FP_BM; e += 256) {
    const int t = e / FP_BM, mm = e % FP_BM;
    double2 v = make_double2(0.0, 0.0);
    if (t < remk && mm < rows) v = row_ptr(mm)[KF + t];
    sm.s1.ltail[t][mm] = make_double2(v.x, -v.y);
  }

  auto issue = [&](int st, int k0) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int k = min(k0 + ka, ng - 1);
      __builtin_amdgcn_global_load_lds((const void*)(arow[i] + k),
                                       (lds_void_t*)&sm.s1.a[st][(2 * wid + i) * 64], 16, 0, 0);
    }
    // W: the chunk's FP_BK x BN slots in 64-slot pieces, piece i on wavefront
    // i % 4.  Every lane of a copy loads: copies with some lanes switched off
    // (one per row, the row's tail masked) left parts of W unwritten in LDS
    // once a row took two copies.
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = wid + 4 * t;
      if (i < 2 * NCT) {  // wave-uniform; every lane of a piece loads
        const int e = 64 * i + lane, kk = e / BN, n = e % BN;
        const int kr = min(k0 + kk, ng - 1);
        __builtin_amdgcn_global_load_lds((const void*)(Wq + (int64_t)kr * ng + n),
                                         (lds_void_t*)&sm.s1.b[st][64 * i], 16, 0, 0);
      }
    }
  };
  // load instructions of one chunk on this wavefront: 2 of L, nbw of W
  const int nbw = (2 * NCT - wid + 3) / 4;

  // FP64: the three products in FP64 over the whole K.  FP32 (precision form):
  // operands rounded to FP32 as they leave LDS, products and sums in FP32
  constexpr bool F32 = PREC == BSE_PREC_FP32;
  using Acc = typename std::conditional<F32, f4, d4>::type;
  Acc p1[NCT], p2[NCT], p3[NCT];
#pragma unroll
  for (int j = 0; j < NCT; ++j) p1[j] = p2[j] = p3[j] = Acc{0, 0, 0, 0};
  // row of accumulator register r (f64: l/16 + 4r; f32: 4 (l/16) + r)
  auto acc_row = [&](int r) { return F32 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r; };
  double2 vacc[VC > 0 ? VC : 1];
#pragma unroll
  for (int c = 0; c < (VC > 0 ? VC : 1); ++c) vacc[c] = make_double2(0.0, 0.0);
  auto mma = [&](int st, int k0) {
#pragma unroll
    for (int ks = 0; ks < FP_BK / 4; ++ks) {
      if (k0 + ks * 4 < KF) {
        const int k = ks * 4 + (lane >> 4), row = wm0 + (lane & 15);
        const unsigned ax =
            lds_off(&sm.s1.a[st][(row >> 3) * 64 + (row & 7) * 8 + (k ^ (row & 7))]);
        const unsigned ab = lds_off(&sm.s1.b[st][k * BN + (lane & 15)]);
        d2v x, y[NCT];
        if constexpr (NCT == 7) {
          lds_read_x_y7(x, y, ax, ab);
        } else {
          x = lds_read1(ax);
#pragma unroll
          for (int j = 0; j < NCT; ++j) y[j] = lds_read1(ab + 256 * j);
        }
        if constexpr (F32) {
          const float xr = (float)x[0], xi = (float)x[1], xs = xr - xi;
#pragma unroll
          for (int j = 0; j < NCT; ++j) {
            const float yr = (float)y[j][0], yi = (float)y[j][1];
            p1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, yr, p1[j], 0, 0, 0);
            p2[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi, yi, p2[j], 0, 0, 0);
            p3[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs, yr + yi, p3[j], 0, 0, 0);
          }
        } else {
          const double xs = x[0] - x[1];
#pragma unroll
          for (int j = 0; j < NCT; ++j) {
            p1[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[0], y[j][0], p1[j], 0, 0, 0);
            p2[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[1], y[j][1], p2[j], 0, 0, 0);
            p3[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs, y[j][0] + y[j][1], p3[j], 0, 0, 0);
          }
        }
      }
    }
    if constexpr (VC > 0) {
      if constexpr (VC == 1) {  // the four values of the chunk in one read block
        const int kk0 = 2 * wid, kk1 = kk0 + 1;
        d2v o[4];
        lds_read_4(o, lds_off(&sm.s1.a[st][(lane >> 3) * 64 + (lane & 7) * 8 + (kk0 ^ (lane & 7))]),
                   lds_off(&sm.s1.a[st][(lane >> 3) * 64 + (lane & 7) * 8 + (kk1 ^ (lane & 7))]),
                   lds_off(&sm.s1.wcol[min(k0 + kk0, 115)][0]),
                   lds_off(&sm.s1.wcol[min(k0 + kk1, 115)][0]));
#pragma unroll
        for (int kq = 0; kq < 2; ++kq)
          if (k0 + kk0 + kq < KF) {
            const d2v x = o[kq], y = o[2 + kq];
            vacc[0].x = fma(x[0], y[0], fma(x[1], y[1], vacc[0].x));  // conj(x) y
            vacc[0].y = fma(x[0], y[1], fma(-x[1], y[0], vacc[0].y));
          }
      } else {
#pragma unroll
        for (int kq = 0; kq < 2; ++kq) {
          const int kk = 2 * wid + kq;
          if (k0 + kk < KF) {
            const d2v xv = lds_read1(
                lds_off(&sm.s1.a[st][(lane >> 3) * 64 + (lane & 7) * 8 + (kk ^ (lane & 7))]));
            const double2 x = make_double2(xv[0], xv[1]);
#pragma unroll
            for (int c = 0; c < VC; ++c) {
              const d2v yv = lds_read1(lds_off(&sm.s1.wcol[k0 + kk][c]));
              const double2 y = make_double2(yv[0], yv[1]);
              vacc[c].x = fma(x.x, y.x, fma(x.y, y.y, vacc[c].x));  // conj(x) y
              vacc[c].y = fma(x.x, y.y, fma(-x.y, y.x, vacc[c].y));
            }
          }
        }
      }
    }
  };

  const int nch = (KF + FP_BK - 1) / FP_BK;
  if (nch > 0) issue(0, 0);
  if (nch > 1) issue(1, FP_BK);
  for (int ch = 0; ch < nch; ++ch) {
    if (ch + 1 < nch) {  // chunk ch + 1 may still be in flight
      if (nbw == 4) wait_vmcnt<6>();
      else if (nbw == 3) wait_vmcnt<5>();
      else if (nbw == 2) wait_vmcnt<4>();
      else if (nbw == 1) wait_vmcnt<3>();
      else wait_vmcnt<2>();
    } else {
      wait_vmcnt<0>();
    }
    lds_barrier();  // chunk ch in LDS for every wavefront; chunk ch - 1 no longer read
    if (ch + 2 < nch) issue((ch + 2) % FP_NS, (ch + 2) * FP_BK);
    mma(ch % FP_NS, ch * FP_BK);
  }

  // T = P1 + Q2 + i (P3 - P1 + Q2) on the matrix-core columns, plus the K tail
  // (W rows from memory); no copy is in flight from here on
  double tre[NCT][4], tim[NCT][4];
#pragma unroll
  for (int j = 0; j < NCT; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = wm0 + acc_row(r), n = j * 16 + (lane & 15);
      double2 v = make_double2((double)(p1[j][r] + p2[j][r]),
                               (double)(p3[j][r] - p1[j][r] + p2[j][r]));
      for (int t = 0; t < remk; ++t)
        v = cadd(v, cmul(sm.s1.ltail[t][m], Wq[(int64_t)(KF + t) * ng + (n < ng ? n : 0)]));
      tre[j][r] = v.x;
      tim[j][r] = v.y;
    }
  // vector-ALU columns: the four k parts summed through LDS
  double2 vcv = make_double2(0.0, 0.0);  // T[tid % 64][16 NCT + tid / 64], tid < 64 VC
  if constexpr (VC > 0) {
    __syncthreads();  // every wavefront done with the chunk buffers and ltail
    double2(*vpart)[FP_BM][VC] = reinterpret_cast<double2(*)[FP_BM][VC]>(&sm.s2.t[0][0]);
    double2 lt[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) lt[t] = sm.s1.ltail[t][tid & 63];  // zero for t >= remk
    __syncthreads();
#pragma unroll
    for (int c = 0; c < VC; ++c) vpart[wid][lane][c] = vacc[c];
    __syncthreads();
    if (tid < FP_BM * VC) {
      const int m = tid & 63, c = tid >> 6;
#pragma unroll
      for (int kq = 0; kq < 4; ++kq) vcv = cadd(vcv, vpart[kq][m][c]);
#pragma unroll
      for (int t = 0; t < 3; ++t)
        if (t < remk) vcv = cadd(vcv, cmul(lt[t], Wq[(int64_t)(KF + t) * ng + 16 * NCT + c]));
    }
  }

  if constexpr (!FUSED) {
    double2* __restrict__ Tq = Tout + ((int64_t)s0 * R + m0) * ng;
#pragma unroll
    for (int j = 0; j < NCT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = wm0 + acc_row(r), n = j * 16 + (lane & 15);
        if (m < rows && n < ng) Tq[(int64_t)m * ng + n] = make_double2(tre[j][r], tim[j][r]);
      }
    if constexpr (VC > 0)
      if (tid < FP_BM * VC && (tid & 63) < rows)
        Tq[(int64_t)(tid & 63) * ng + 16 * NCT + (tid >> 6)] = vcv;
  } else {
    // ---- second product
    constexpr int NPH = NCT + (VC > 0 ? 1 : 0);
    const int npb = rows / R;                  // pairs of this block
    const int nq4 = (N2 + 3) >> 2;             // 4-row pieces of R_p
    __syncthreads();  // LDS free for the second product (vpart, ltail read)
    // copies of R_p for phase ph: 8 per wavefront and phase (unused ones land
    // in `dummy`), so that the waits count a fixed number
    // the second operands of this wavefront's pairs (loaded here, not between
    // the copies: a load the copies' addresses wait on would wait for them all)
    const double2* rbase[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int pp = wid + 4 * u;
      rbase[u] = pp < npb ? Right + (int64_t)perm[s0 + (m0 / R) + pp] * N2 * ng : Right;
    }
    auto issue_rt = [&](int buf, int ph) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int jq = 0; jq < 4; ++jq) {
          const int pp = wid + 4 * u;
          const bool real = pp < npb && jq < nq4;  // wave-uniform
          const int j = min(4 * jq + (lane >> 4), N2 - 1);
          const int g = min(16 * ph + ((lane & 15) ^ (j & 7)), ng - 1);
          const double2* src = real ? rbase[u] + (int64_t)j * ng + g : Right;
          lds_void_t* dst = real ? (lds_void_t*)&sm.s2.rt[buf][pp][64 * jq]
                                 : (lds_void_t*)&sm.s2.dummy[0];
          __builtin_amdgcn_global_load_lds((const void*)src, dst, 16, 0, 0);
        }
    };
    d4 q1[2], q2[2], q3[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) q1[u] = q2[u] = q3[u] = d4{0, 0, 0, 0};
    issue_rt(0, 0);
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph) {
      // this wavefront's copies for the next phase (into the buffer it read
      // in the previous phase)
      if (ph + 1 < NPH) issue_rt((ph + 1) & 1, ph + 1);
      if (ph > 0) lds_barrier();  // T of phase ph - 1 no longer read
      // T of this phase into LDS (columns past N_G as zeros)
      if (ph < NCT) {
        d2v v[4];
        unsigned wa[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = wm0 + acc_row(r), n = 16 * ph + (lane & 15);
          v[r][0] = n < ng ? tre[ph][r] : 0.0;
          v[r][1] = n < ng ? tim[ph][r] : 0.0;
          wa[r] = lds_off(&sm.s2.t[m][lane & 15]);
        }
        asm volatile(
            "ds_write_b128 %0, %4\n\tds_write_b128 %1, %5\n\t"
            "ds_write_b128 %2, %6\n\tds_write_b128 %3, %7\n\ts_waitcnt lgkmcnt(0)"
            ::"v"(wa[0]), "v"(wa[1]), "v"(wa[2]), "v"(wa[3]), "v"(v[0]), "v"(v[1]), "v"(v[2]),
            "v"(v[3])
            : "memory");
      } else {
        for (int e = tid; e < FP_BM * 16; e += 256) {
          const int m = e & 63, c = e >> 6;
          d2v v;
          v[0] = 0.0;
          v[1] = 0.0;
          if (c < VC && e == tid) { v[0] = vcv.x; v[1] = vcv.y; }  // tid < 64 VC holds column c
          asm volatile("ds_write_b128 %0, %1\n\ts_waitcnt lgkmcnt(0)"
                       ::"v"(lds_off(&sm.s2.t[m][c])), "v"(v) : "memory");
        }
      }
      lds_barrier();  // T of phase ph complete
      if (ph + 1 < NPH) wait_vmcnt<8>();  // this wavefront's copies of phase ph done
      else wait_vmcnt<0>();
      const int nks = ph < NCT ? 4 : 1;  // the vector-ALU phase holds at most 3 columns
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int pp = wid + 4 * u;
        if (pp < npb) {  // wave-uniform
          const int r = lane & 15, j = lane & 15;
          const int trow = min(pp * R + r, FP_BM - 1);  // rows r >= R are not stored
          // the phase's operands of this pair in one read block (T at g = 4 ks + l / 16:
          // 64 bytes apart; R_p swizzled by j)
          d2v a[4], bv[4];
          unsigned rb[4];
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
            rb[ks] = lds_off(&sm.s2.rt[ph & 1][pp][j * 16 + ((4 * ks + (lane >> 4)) ^ (j & 7))]);
          lds_read_4x2(a, bv, lds_off(&sm.s2.t[trow][lane >> 4]), rb);
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
            if (ks < nks) {
              q1[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][0], bv[ks][0], q1[u], 0, 0, 0);
              q2[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][1], bv[ks][1], q2[u], 0, 0, 0);
              q3[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks][0] + a[ks][1],
                                                           bv[ks][0] + bv[ks][1], q3[u], 0, 0, 0);
            }
        }
      }
    }
    // add the blocks into the outputs: entry (r, j) of pair p; resonant rows
    // r = (v, v'), columns j = (c, c'); coupling rows r = (c, v'), j = (v, c')
    const int nvnc = nv * nc;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int pp = wid + 4 * u;
      if (pp >= npb) continue;
      const int p = perm[s0 + (m0 / R) + pp];
      const int ik = pair_row(p, nk);
      const int jk = ik + (int)(p - ((int64_t)ik * nk - (int64_t)ik * (ik - 1) / 2));
      const int jj = lane & 15;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = (lane >> 4) + 4 * i;
        if (rr >= R || jj >= N2) continue;
        int v, c, v2, c2;
        if (!ra) {
          v = rr / nv; v2 = rr % nv; c = jj / nc; c2 = jj % nc;
        } else {
          c = rr / nv; v2 = rr % nv; v = jj / nc; c2 = jj % nc;
        }
        const int64_t row = (int64_t)ik * nvnc + v * nc + c;
        const int64_t col = (int64_t)jk * nvnc + v2 * nc + c2;
        const double2 val = make_double2(coef * (q1[u][i] - q2[u][i]),
                                         coef * (q3[u][i] - q1[u][i] - q2[u][i]));
        double2* d0 = out0 + row + col * ld;
        const double2 o = *d0;
        *d0 = make_double2(o.x + val.x, o.y + val.y);
        if (out1) {
          double2* d1 = out1 + row + col * ld;
          if (!ra) {
            *d1 = val;  // the resonant term writes A-B first
          } else {
            const double2 o1 = *d1;
            *d1 = make_double2(o1.x - val.x, o1.y - val.y);
          }
        }
      }
    }
  }
}

template <int NCT, int VC>
void launch_fp2(const double2* left, int R, int ng, int nk, const double2* W,
                const int32_t* perm, const int32_t* cls, int nq, double2* Tout,
                const int32_t* info, hipStream_t s) {
  const int spc = (int)cdiv((int64_t)nk * R, FP_BM);  // a class holds at most nk pairs
  BSE_LAUNCH((k_first_product2<NCT, VC, false>), dim3((unsigned)((int64_t)nq * spc)), dim3(256),
             0, s, left, R, ng, W, perm, cls, nq, spc, Tout, info, (const double2*)nullptr, 0,
             nk, 0, 0, 0, 0.0, (double2*)nullptr, (double2*)nullptr, (int64_t)0,
             (const int32_t*)nullptr);
}

// Tiles of ppt pairs of each class, listed class by class: map[b] = q |
// t << 13 for tile t of class q, -1 from the last tile to cap (one block of
// 1024 threads; at most cdiv(P, ppt) + nq tiles)
__global__ __launch_bounds__(1024) void k_tile_map(const int32_t* __restrict__ cls, int nq,
                                                   int ppt, int32_t* __restrict__ map, int cap) {
  __shared__ int32_t wtot[16];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int per = cdiv(nq, 1024), q0 = min(nq, tid * per), q1 = min(nq, q0 + per);
  int tot = 0;
  for (int q = q0; q < q1; ++q) tot += cdiv(cls[q + 1] - cls[q], ppt);
  int incl = tot;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wtot[wid] = incl;
  __syncthreads();
  int run = incl - tot, all = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wid) run += wtot[w];
    all += wtot[w];
  }
  for (int q = q0; q < q1; ++q) {
    const int nt = cdiv(cls[q + 1] - cls[q], ppt);
    for (int t = 0; t < nt; ++t) map[run + t] = q | (t << 13);
    run += nt;
  }
  for (int b = all + tid; b < cap; b += 1024) map[b] = -1;
}

template <int NCT, int VC>
void launch_df(int prec, const double2* left, const double2* right, int R, int N2, int ng, int nk,
               int nv, int nc, const double2* W, const int32_t* perm, const int32_t* cls, int nq,
               int ra, double coef, double2* out0, double2* out1, int64_t ld, int32_t* tmap,
               const int32_t* info, hipStream_t s) {
  const int ppt = FP_BM / R;
  const int spc = cdiv(nk, ppt);  // a class holds at most nk pairs
  const int64_t P = (int64_t)nk * (nk + 1) / 2;
  const int cap = (int)(cdiv(P, ppt) + nq);
  BSE_LAUNCH(k_tile_map, dim3(1), dim3(1024), 0, s, cls, nq, ppt, tmap, cap);
  if (prec == BSE_PREC_FP32)
    BSE_LAUNCH((k_first_product2<NCT, VC, true, BSE_PREC_FP32>), dim3((unsigned)cap), dim3(256),
               0, s, left, R, ng, W, perm, cls, nq, spc, (double2*)nullptr, info, right, N2, nk,
               nv, nc, ra, coef, out0, out1, ld, (const int32_t*)tmap);
  else
    BSE_LAUNCH((k_first_product2<NCT, VC, true>), dim3((unsigned)cap), dim3(256), 0, s, left, R,
               ng, W, perm, cls, nq, spc, (double2*)nullptr, info, right, N2, nk, nv, nc, ra,
               coef, out0, out1, ld, (const int32_t*)tmap);
}

}  // namespace

// Returns false when the shape is outside what the fused kernel handles
// (nothing is launched; the caller takes the two-pass path).
bool launch_direct_fused(int prec, int variant, const double2* left, const double2* right, int R,
                         int N2, int ng, int nk, int nv, int nc, const double2* W,
                         const int32_t* perm, const int32_t* cls, int nq, int ra, double coef,
                         double2* out0, double2* out1, int64_t ld, double2* Tout,
                         const int32_t* info, hipStream_t s) {
  if (ng > 128 || R < 1 || R > DBM || N2 < 1) return false;
  if (prec == BSE_PREC_FP32)
    dispatch<BSE_PREC_FP32>(variant, left, right, R, N2, ng, nk, nv, nc, W, perm, cls, nq, ra,
                            coef, out0, out1, ld, Tout, info, s);
  else if (prec == BSE_PREC_FP64)
    dispatch<BSE_PREC_FP64>(variant, left, right, R, N2, ng, nk, nv, nc, W, perm, cls, nq, ra,
                            coef, out0, out1, ld, Tout, info, s);
  else
    return false;
  return hipGetLastError() == hipSuccess;
}

// (N_G above 113 would need the eighth column tile, which spills registers)
bool first_product_fits(int ng, int R) { return ng >= 16 && ng <= 113 && R >= 1; }

// First product alone (FP64), written to Tout in class order (the shape must
// pass first_product_fits).  shape 0: operands through registers; 1: copied
// straight into LDS.  Returns false on a launch error.
bool launch_first_product(int shape, const double2* left, int R, int ng, int nk,
                          const double2* W, const int32_t* perm, const int32_t* cls, int nq,
                          double2* Tout, const int32_t* info, hipStream_t s) {
  if (!first_product_fits(ng, R)) return false;
  // columns past 16 NCT go to the vector ALU when there are at most 3 of them,
  // else the last tile is padded
  const int vc = ng % 16 <= 3 ? ng % 16 : 0;
  const int nct = vc || ng % 16 == 0 ? ng / 16 : ng / 16 + 1;
#define BSE_FP2(NCT, VC)                                                                \
  if (shape == 1) launch_fp2<NCT, VC>(left, R, ng, nk, W, perm, cls, nq, Tout, info, s); \
  else launch_fp<NCT, VC>(left, R, ng, nk, W, perm, cls, nq, Tout, info, s);
#define BSE_FP(NCT)                             \
  case NCT:                                     \
    if (vc == 0) { BSE_FP2(NCT, 0) }            \
    else if (vc == 1) { BSE_FP2(NCT, 1) }       \
    else if (vc == 2) { BSE_FP2(NCT, 2) }       \
    else { BSE_FP2(NCT, 3) }                    \
    break;
  switch (nct) {
    BSE_FP(1) BSE_FP(2) BSE_FP(3) BSE_FP(4) BSE_FP(5) BSE_FP(6) BSE_FP(7)
    default: return false;
  }
#undef BSE_FP
#undef BSE_FP2
  return hipGetLastError() == hipSuccess;
}

// One pass per direct term on the matrix cores (FP64, or the first product in
// FP32 for the precision form): the first product as
// in launch_first_product, the second per pair, the blocks added into the
// outputs.  tmap: cdiv(P, 64 / R) + nq ints of device scratch for the tile
// list.  Returns false when the shape is not handled (nothing launched):
// N_G outside 16..113, R outside 9..16 or N2 above 16.
bool launch_direct_onepass(int prec, const double2* left, const double2* right, int R, int N2,
                           int ng, int nk, int nv, int nc, const double2* W, const int32_t* perm,
                           const int32_t* cls, int nq, int ra, double coef, double2* out0,
                           double2* out1, int64_t ld, int32_t* tmap, const int32_t* info,
                           hipStream_t s) {
  if (!first_product_fits(ng, R) || R < 9 || R > 16 || N2 < 1 || N2 > 16) return false;
  if (prec != BSE_PREC_FP64 && prec != BSE_PREC_FP32) return false;
  const int vc = ng % 16 <= 3 ? ng % 16 : 0;
  const int nct = vc || ng % 16 == 0 ? ng / 16 : ng / 16 + 1;
#define BSE_DF2(NCT, VC) \
  launch_df<NCT, VC>(prec, left, right, R, N2, ng, nk, nv, nc, W, perm, cls, nq, ra, coef, out0, out1, ld, tmap, info, s);
#define BSE_DF(NCT)                             \
  case NCT:                                     \
    if (vc == 0) { BSE_DF2(NCT, 0) }            \
    else if (vc == 1) { BSE_DF2(NCT, 1) }       \
    else if (vc == 2) { BSE_DF2(NCT, 2) }       \
    else { BSE_DF2(NCT, 3) }                    \
    break;
  switch (nct) {
    BSE_DF(1) BSE_DF(2) BSE_DF(3) BSE_DF(4) BSE_DF(5) BSE_DF(6) BSE_DF(7)
    default: return false;
  }
#undef BSE_DF
#undef BSE_DF2
  return hipGetLastError() == hipSuccess;
}
