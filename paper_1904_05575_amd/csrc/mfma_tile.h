// Block-level complex FP64 tile product on MFMA, shared by the GEMM kernels.
//
// A workgroup of WM x WN waves computes a BM x BN complex tile
//   acc(m, n) = sum_k a(m, k) b(k, n)
// staging BM x 16 and 16 x BN slices of the operands in LDS.  The caller
// supplies loaders that return one (already conjugated / scaled / masked)
// complex element; `a_mfast` / `b_nfast` pick the thread-to-element order
// that keeps the global reads coalesced for the operand's layout.
//
// v_mfma_f64_16x16x4_f64 lane layout: A operand lane l -> (m = l%16, k = l/16),
// B operand lane l -> (k = l/16, n = l%16), accumulator register r of lane l
// -> (m = l/16 + 4*r, n = l%16).
//
// G3 = false: four real products per complex one (re = ar br - ai bi,
// im = ar bi + ai br).  G3 = true: three (Gauss's product: P1 = ar br,
// P2 = ai bi, P3 = (ar + ai)(br + bi); re = P1 - P2, im = P3 - P1 - P2),
// a quarter fewer matrix-core operations for one more accumulator per tile.
#pragma once
#include "common.h"

template <int BM, int BN, int WM, int WN, bool G3 = false>
struct ZTile {
  static constexpr int BK = 16;
  static constexpr int PAD = 2;
  static constexpr int NT = WM * WN * 64;
  static constexpr int TI = BM / WM / 16;
  static constexpr int TJ = BN / WN / 16;
  static_assert(TI >= 1 && TJ >= 1, "tile too small for the wave grid");

  struct Smem {
    double a_re[BK][BM + PAD], a_im[BK][BM + PAD];
    double b_re[BK][BN + PAD], b_im[BK][BN + PAD];
  };

  d4 cr[TI][TJ], ci[TI][TJ];  // G3: P1 and P2
  d4 c3[G3 ? TI : 1][G3 ? TJ : 1];  // G3: P3
  int wm0, wn0, lane;

  BSE_DEV void init() {
    lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    wm0 = (wid % WM) * (BM / WM);
    wn0 = (wid / WM) * (BN / WN);
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        cr[i][j] = d4{0, 0, 0, 0};
        ci[i][j] = d4{0, 0, 0, 0};
        if constexpr (G3) c3[i][j] = d4{0, 0, 0, 0};
      }
  }

  // acc (+)= a b for one 16 x 16 x 4 slice of tile (i, j)
  BSE_DEV void mac(int i, int j, double ar, double ai, double nai, double br, double bi) {
    if constexpr (G3) {
      cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cr[i][j], 0, 0, 0);
      ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, ci[i][j], 0, 0, 0);
      c3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, br + bi, c3[i][j], 0, 0, 0);
    } else {
      cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cr[i][j], 0, 0, 0);
      cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, bi, cr[i][j], 0, 0, 0);
      ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, ci[i][j], 0, 0, 0);
      ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, ci[i][j], 0, 0, 0);
    }
  }

  // loadA(mm, k) / loadB(k, nn): element of the operand at tile-local row mm
  // (column nn) and absolute k; must return 0 outside the operand.
  template <class LA, class LB>
  BSE_DEV void run(Smem& s, int k_lo, int k_hi, bool a_mfast, bool b_nfast, LA loadA, LB loadB) {
    const int tid = threadIdx.x;
    for (int k0 = k_lo; k0 < k_hi; k0 += BK) {
      for (int e = tid; e < BM * BK; e += NT) {
        int mm, kk;
        if (a_mfast) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
        const int k = k0 + kk;
        double2 v = (k < k_hi) ? loadA(mm, k) : make_double2(0.0, 0.0);
        s.a_re[kk][mm] = v.x;
        s.a_im[kk][mm] = v.y;
      }
      for (int e = tid; e < BN * BK; e += NT) {
        int nn, kk;
        if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
        const int k = k0 + kk;
        double2 v = (k < k_hi) ? loadB(k, nn) : make_double2(0.0, 0.0);
        s.b_re[kk][nn] = v.x;
        s.b_im[kk][nn] = v.y;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        double ar[TI], ai[TI], nai[TI], br[TJ], bi[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i) {
          ar[i] = s.a_re[kr][wm0 + i * 16 + (lane & 15)];
          ai[i] = s.a_im[kr][wm0 + i * 16 + (lane & 15)];
          nai[i] = -ai[i];
        }
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          br[j] = s.b_re[kr][wn0 + j * 16 + (lane & 15)];
          bi[j] = s.b_im[kr][wn0 + j * 16 + (lane & 15)];
        }
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) mac(i, j, ar[i], ai[i], nai[i], br[j], bi[j]);
      }
      __syncthreads();
    }
  }

  // Main loop with register prefetch: while one K slice is multiplied from
  // LDS, the next one is in flight in registers; two LDS buffers, one barrier
  // per slice.  addrA(mm, k, ok) / addrB(k, nn, ok) return the address of an
  // element for any index (clamped inside the operand) and set ok when the
  // element exists, so that every load is issued without a condition;
  // fixA(v, k) / fixB(v, k) apply conjugation or scaling to an existing one.
  struct Smem2 {
    Smem buf[2];
  };
  template <class AA, class AB, class FA, class FB>
  BSE_DEV void run_pf(Smem2& s, int k_lo, int k_hi, bool a_mfast, bool b_nfast, AA addrA,
                      AB addrB, FA fixA, FB fixB) {
    constexpr int NA = BM * BK / NT, NB = BN * BK / NT;
    static_assert(NA * NT == BM * BK && NB * NT == BN * BK, "slice not divisible");
    const int tid = threadIdx.x;
    double2 ra[NA], rb[NB];
    bool oa[NA], ob[NB];
    auto a_at = [&](int e, int& mm, int& kk) {
      if (a_mfast) { mm = e % BM; kk = e / BM; } else { kk = e % BK; mm = e / BK; }
    };
    auto b_at = [&](int e, int& kk, int& nn) {
      if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
    };
    auto fetch = [&](int k0) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        int mm, kk;
        a_at(tid + NT * q, mm, kk);
        bool ok;
        const double2* p = addrA(mm, k0 + kk, ok);
        ra[q] = *p;
        oa[q] = ok && k0 + kk < k_hi;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        int kk, nn;
        b_at(tid + NT * q, kk, nn);
        bool ok;
        const double2* p = addrB(k0 + kk, nn, ok);
        rb[q] = *p;
        ob[q] = ok && k0 + kk < k_hi;
      }
    };
    auto put = [&](Smem& sm, int k0) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        int mm, kk;
        a_at(tid + NT * q, mm, kk);
        const double2 v = oa[q] ? fixA(ra[q], k0 + kk) : make_double2(0.0, 0.0);
        sm.a_re[kk][mm] = v.x;
        sm.a_im[kk][mm] = v.y;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        int kk, nn;
        b_at(tid + NT * q, kk, nn);
        const double2 v = ob[q] ? fixB(rb[q], k0 + kk) : make_double2(0.0, 0.0);
        sm.b_re[kk][nn] = v.x;
        sm.b_im[kk][nn] = v.y;
      }
    };
    if (k_lo >= k_hi) return;
    fetch(k_lo);
    int buf = 0;
    for (int k0 = k_lo; k0 < k_hi; k0 += BK) {
      put(s.buf[buf], k0);
      __syncthreads();
      if (k0 + BK < k_hi) fetch(k0 + BK);
      slice(s.buf[buf]);
      buf ^= 1;
    }
  }

  // acc += the BK-deep slice staged in sm
  BSE_DEV void slice(const Smem& sm) {
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      double ar[TI], ai[TI], nai[TI], br[TJ], bi[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        ar[i] = sm.a_re[kr][wm0 + i * 16 + (lane & 15)];
        ai[i] = sm.a_im[kr][wm0 + i * 16 + (lane & 15)];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        br[j] = sm.b_re[kr][wn0 + j * 16 + (lane & 15)];
        bi[j] = sm.b_im[kr][wn0 + j * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) mac(i, j, ar[i], ai[i], nai[i], br[j], bi[j]);
    }
  }

  // store(m_local, n_local, value) for every accumulator element.
  template <class ST>
  BSE_DEV void store(ST st) {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
        {
          double2 v;
          if constexpr (G3)
            v = make_double2(cr[i][j][r] - ci[i][j][r], c3[i][j][r] - cr[i][j][r] - ci[i][j][r]);
          else
            v = make_double2(cr[i][j][r], ci[i][j][r]);
          st(wm0 + i * 16 + (lane >> 4) + 4 * r, wn0 + j * 16 + (lane & 15), v);
        }
  }
};
