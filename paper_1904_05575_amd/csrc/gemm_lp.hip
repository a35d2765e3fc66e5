// Reduced-precision complex GEMMs of the kernel assembly (the precision form
// of the direct and exchange terms): FP32 operands, or operands split into
// three BF16 terms, on the matrix cores with FP32 accumulation inside a
// K-chunk and FP64 accumulation across chunks.
//
// Complex products use the real view of interleaved data (see stage1.hip):
//   A (M x 2K) = A as doubles,  B' (2K x 2N): row 2k = B[k], row 2k+1 = i B[k].
// BF16 split of x: x32 = fl32(x) (round to nearest even), hi = bf16(x32),
// mid = bf16(x32 - hi), lo = bf16(x32 - hi - mid); the differences are exact
// in FP32.  With 6 products (hi*hi, hi*mid, mid*hi, hi*lo, lo*hi, mid*mid)
// the dropped terms are O(2^-24) relative; with 3 products (the first three)
// O(2^-16).
#include "bse_internal.h"
#include "common.h"
#include "timing.h"

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int LBM = 64;   // rows per block (4 waves x 16)
constexpr int KC = 16;    // complex k per chunk (32 real)
constexpr int KR = 2 * KC;

BSE_DEV unsigned short bf16_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
BSE_DEV float bf16_to_f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// One precision-dependent tile: 64 rows x BN2 real columns.
template <int PREC, int BN2>
struct LpSmem;

template <int BN2>
struct alignas(16) LpSmem<BSE_PREC_FP32, BN2> {
  float a[KR][LBM + 4];
  float b[KR][BN2 + 4];
};

template <int BN2>
struct alignas(16) LpSmem<BSE_PREC_BF16X3, BN2> {
  // k-contiguous so that a lane reads its 8 consecutive k in one 16-byte load
  unsigned short a[3][LBM][KR + 8];
  unsigned short b[3][BN2][KR + 8];
};

// Stage the real-view tiles of one chunk.  ga(mm, kc) / gb(kc, nn) return the
// complex operand elements (zero outside).
template <int PREC, int BN2, class GA, class GB>
BSE_DEV void lp_stage(LpSmem<PREC, BN2>& s, int kc0, GA ga, GB gb) {
  const int tid = threadIdx.x;
  constexpr int BNC = BN2 / 2;
  for (int e = tid; e < LBM * KC; e += 256) {
    const int mm = e / KC, kk = e % KC;
    const double2 v = ga(mm, kc0 + kk);
    const float xr = (float)v.x, xi = (float)v.y;
    if constexpr (PREC == BSE_PREC_FP32) {
      s.a[2 * kk][mm] = xr;
      s.a[2 * kk + 1][mm] = xi;
    } else {
      const float x2[2] = {xr, xi};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const unsigned short h = bf16_rne(x2[t]);
        const float r1 = x2[t] - bf16_to_f(h);
        const unsigned short m = bf16_rne(r1);
        const unsigned short l = bf16_rne(r1 - bf16_to_f(m));
        s.a[0][mm][2 * kk + t] = h;
        s.a[1][mm][2 * kk + t] = m;
        s.a[2][mm][2 * kk + t] = l;
      }
    }
  }
  for (int e = tid; e < KC * BNC; e += 256) {
    const int kk = e / BNC, nc = e % BNC;
    const double2 v = gb(kc0 + kk, nc);
    const float br = (float)v.x, bi = (float)v.y;
    // rows 2kk: (br, bi) at columns (2nc, 2nc+1); rows 2kk+1: (-bi, br)
    const float vals[4] = {br, bi, -bi, br};
    const int rk[4] = {2 * kk, 2 * kk, 2 * kk + 1, 2 * kk + 1};
    const int cn[4] = {2 * nc, 2 * nc + 1, 2 * nc, 2 * nc + 1};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if constexpr (PREC == BSE_PREC_FP32) {
        s.b[rk[t]][cn[t]] = vals[t];
      } else {
        const unsigned short h = bf16_rne(vals[t]);
        const float r1 = vals[t] - bf16_to_f(h);
        const unsigned short m = bf16_rne(r1);
        const unsigned short l = bf16_rne(r1 - bf16_to_f(m));
        s.b[0][cn[t]][rk[t]] = h;
        s.b[1][cn[t]][rk[t]] = m;
        s.b[2][cn[t]][rk[t]] = l;
      }
    }
  }
}

BSE_DEV bf8 ld_bf8(const unsigned short* p) {
  const uint4 u = *(const uint4*)p;
  return __builtin_bit_cast(bf8, u);
}

// Multiply the staged chunk into the FP32 accumulators of this wave
// (16 rows x NT column tiles).
template <int PREC, int BN2>
BSE_DEV void lp_mma(LpSmem<PREC, BN2>& s, f4 (&acc)[BN2 / 16], int nterms) {
  constexpr int NT = BN2 / 16;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int row = wid * 16 + (lane & 15);
  if constexpr (PREC == BSE_PREC_FP32) {
#pragma unroll
    for (int ks = 0; ks < KR / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      const float a = s.a[kr][row];
#pragma unroll
      for (int j = 0; j < NT; ++j)
        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, s.b[kr][j * 16 + (lane & 15)], acc[j], 0,
                                                      0, 0);
    }
  } else {
    const int k8 = (lane >> 4) * 8;
    const bf8 ah = ld_bf8(&s.a[0][row][k8]);
    const bf8 am = ld_bf8(&s.a[1][row][k8]);
    const bf8 al = ld_bf8(&s.a[2][row][k8]);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      const int col = j * 16 + (lane & 15);
      const bf8 bh = ld_bf8(&s.b[0][col][k8]);
      const bf8 bm = ld_bf8(&s.b[1][col][k8]);
      f4 c = acc[j];
      if (nterms >= 6) {
        const bf8 bl = ld_bf8(&s.b[2][col][k8]);
        // small terms first so that they are not absorbed by the large one
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
      }
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
      acc[j] = c;
    }
  }
}

// Full K loop: FP32 accumulation per chunk, FP64 across chunks.  The FP64
// result for (row 4*(lane/16)+r of the wave's 16, column tile j) is in acc64.
template <int PREC, int BN2, class GA, class GB>
BSE_DEV void lp_gemm(LpSmem<PREC, BN2>& s, int K, int nterms, GA ga, GB gb,
                     double (&acc64)[BN2 / 16][4]) {
  constexpr int NT = BN2 / 16;
#pragma unroll
  for (int j = 0; j < NT; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[j][r] = 0.0;
  for (int kc0 = 0; kc0 < K; kc0 += KC) {
    lp_stage<PREC, BN2>(s, kc0, ga, gb);
    __syncthreads();
    f4 acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    lp_mma<PREC, BN2>(s, acc, nterms);
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[j][r] += (double)acc[j][r];
    __syncthreads();
  }
}

// output element (row m_local, real column n2_local) held by acc64[j][r]
BSE_DEV int lp_row(int r) { return (threadIdx.x >> 6) * 16 + 4 * ((threadIdx.x & 63) >> 4) + r; }
BSE_DEV int lp_col(int j) { return j * 16 + (threadIdx.x & 15); }

// ---------------------------------------------------------------- stage 1
// Real view of W(q) (see stage1.hip), split once per build for the matrix
// cores: B'(k, n) = row 2g: W[g] as doubles, row 2g+1: i W[g] as doubles.
//   BF16: planes hi, mid, lo of B', layout [q][plane][n < n2p][k < k2p] (k contiguous,
//         eight k per lane of the 16x16x32 operand)
//   FP32: layout [q][k < k2p][n < n2p]
// zero outside 2 ng.
template <int PREC>
__global__ __launch_bounds__(256) void k_split_w(const double2* __restrict__ W, int ng, int n2p,
                                                 int k2p, void* __restrict__ Wsp) {
  const int q = blockIdx.y;
  const double2* __restrict__ Wq = W + (int64_t)q * ng * ng;
  const int64_t per = (int64_t)n2p * k2p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < per;
       e += (int64_t)gridDim.x * blockDim.x) {
    int k, n;
    if constexpr (PREC == BSE_PREC_FP32) { k = (int)(e / n2p); n = (int)(e % n2p); }
    else { n = (int)(e / k2p); k = (int)(e % k2p); }
    float v = 0.f;
    if (k < 2 * ng && n < 2 * ng) {
      const double2 w = Wq[(int64_t)(k >> 1) * ng + (n >> 1)];
      const double d = (k & 1) ? ((n & 1) ? w.x : -w.y) : ((n & 1) ? w.y : w.x);
      v = (float)d;
    }
    if constexpr (PREC == BSE_PREC_FP32) {
      ((float*)Wsp)[(int64_t)q * per + e] = v;
    } else {
      unsigned short* o = (unsigned short*)Wsp + (int64_t)q * 3 * per;
      const unsigned short h = bf16_rne(v);
      const float r1 = v - bf16_to_f(h);
      const unsigned short m = bf16_rne(r1);
      const unsigned short l = bf16_rne(r1 - bf16_to_f(m));
      o[e] = h;
      o[per + e] = m;
      o[2 * per + e] = l;
    }
  }
}

// T[pos*R + sub, G'] = sum_G conj(L[p][sub][G]) W[q][G][G'] in the precision
// form: 64 rows x up to S1L_NMAX real columns per block of 8 wavefronts (4 row
// groups x 2 column halves of 8 tiles); wider W(q) (n2p > S1L_NMAX) take
// several column blocks (blockIdx.y), each splitting its rows of A again.  Each wavefront loads and splits its own A
// fragments (eight consecutive real k per lane); the block stages the split
// W(q) through two LDS buffers, one 32-deep slice ahead in registers.  FP32
// accumulation inside a slice (16 complex k), FP64 across slices.
constexpr int S1L_BM = 64, S1L_KS = 32, S1L_NMAX = 256;
template <int PREC>
struct S1LSmem;
template <>
struct alignas(16) S1LSmem<BSE_PREC_BF16X3> {
  unsigned short b[2][3][S1L_NMAX][S1L_KS + 8];
};
template <>
struct alignas(16) S1LSmem<BSE_PREC_FP32> {
  float b[2][S1L_KS][S1L_NMAX + 4];
};

template <int PREC>
__global__ __launch_bounds__(512) void k_stage1_lp(const double2* __restrict__ Left, int R,
                                                   int ng, const void* __restrict__ Wsp,
                                                   int n2p, int k2p,
                                                   const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ cls,
                                                   int tiles_per_class, int nterms,
                                                   double2* __restrict__ T,
                                                   const int32_t* info) {
  constexpr int NTW = 8;  // column tiles per wavefront
  __shared__ S1LSmem<PREC> sm;
  if (failed(info)) return;
  const int q = blockIdx.x / tiles_per_class, mt = blockIdx.x % tiles_per_class;
  const int s0 = cls[q], rows = (cls[q + 1] - s0) * R;
  const int m0 = mt * S1L_BM;
  if (m0 >= rows) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int rg = wid & 3, hf = wid >> 2, g = lane >> 4, l16 = lane & 15;
  const int col0 = blockIdx.y * S1L_NMAX;  // first real column of this block
  const int ntiles = min(S1L_NMAX, n2p - col0) / 16;
  const int64_t per = (int64_t)n2p * k2p;
  const int nslices = k2p / S1L_KS;

  // this lane's A row (clamped inside the class; masked at the store)
  const int mrow = m0 + rg * 16 + l16;
  const bool row_ok = mrow < rows;
  const double2* arow;
  {
    const int m = row_ok ? mrow : m0;
    const int64_t p = perm[s0 + m / R];
    arow = Left + (p * R + m % R) * ng;
  }
  // slices ahead in registers: complex G = k0/2 + 4g .. +3 of A, 16-byte units of B
  auto load_a = [&](double2 (&an)[4], int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int t = 0; t < 4; ++t) an[t] = arow[min(k0 / 2 + 4 * g + t, ng - 1)];
  };
  // W(q) slice in 16-byte units over the whole LDS buffer (S1L_NMAX columns), so
  // that every thread moves the same number of units without a condition;
  // columns past n2p repeat column n2p-1 and are never read
  constexpr int UNITS = (PREC == BSE_PREC_FP32) ? S1L_KS * S1L_NMAX / 4 : 3 * S1L_NMAX * S1L_KS / 8;
  constexpr int UPT = UNITS / 512;
  static_assert(UPT * 512 == UNITS, "slice units");
  auto load_b = [&](u32x4 (&bn)[UPT], int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const int e = tid + 512 * u;
      if constexpr (PREC == BSE_PREC_FP32) {
        const int kk = e / (S1L_NMAX / 4), c4 = min(col0 / 4 + e % (S1L_NMAX / 4), n2p / 4 - 1);
        const int64_t off = (int64_t)q * per + (int64_t)(k0 + kk) * n2p + 4 * c4;  // floats
        bn[u] = *(const u32x4*)((const float*)Wsp + off);
      } else {
        const int seg = e & 3, row = e >> 2;  // row = plane * S1L_NMAX + n
        const int plane = row / S1L_NMAX, nn = min(col0 + row % S1L_NMAX, n2p - 1);
        const int64_t off =
            (int64_t)q * 3 * per + (int64_t)plane * per + (int64_t)nn * k2p + k0 + 8 * seg;
        bn[u] = *(const u32x4*)((const unsigned short*)Wsp + off);
      }
    }
  };
  auto store_b = [&](const u32x4 (&bn)[UPT], int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < UPT; ++u) {
      const int e = tid + 512 * u;
      if constexpr (PREC == BSE_PREC_FP32) {
        const int kk = e / (S1L_NMAX / 4), c4 = e % (S1L_NMAX / 4);
        *(u32x4*)&sm.b[buf][kk][4 * c4] = bn[u];
      } else {
        const int seg = e & 3, row = e >> 2;
        *(u32x4*)&sm.b[buf][row / S1L_NMAX][row % S1L_NMAX][8 * seg] = bn[u];
      }
    }
  };

  double acc64[NTW][4];
#pragma unroll
  for (int j = 0; j < NTW; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[j][r] = 0.0;

  // one slice: stage its W part, split its A part, start the loads of the slice
  // two ahead into the register set just freed, multiply
  auto slice = [&](int sl, double2 (&ac)[4], u32x4 (&bc)[UPT]) __attribute__((always_inline)) {
    const int buf = sl & 1, k0 = sl * S1L_KS;
    store_b(bc, buf);
    float ak[8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bool ok = row_ok && (k0 / 2 + 4 * g + t) < ng;
      ak[2 * t] = ok ? (float)ac[t].x : 0.f;
      ak[2 * t + 1] = ok ? (float)(-ac[t].y) : 0.f;
    }
    __syncthreads();
    {  // unconditional (clamped to the last slice) so that waits stay counted
      const int kn = min(k0 + 2 * S1L_KS, k2p - S1L_KS);
      load_a(ac, kn);
      load_b(bc, kn);
    }
    f4 acc[NTW];
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
    if constexpr (PREC == BSE_PREC_FP32) {
      const float* brow = &sm.b[buf][8 * g][16 * hf * NTW + l16];
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        if (hf * NTW + j < ntiles) {
          f4 c = acc[j];
#pragma unroll
          for (int t = 0; t < 8; ++t)
            c = __builtin_amdgcn_mfma_f32_16x16x4f32(ak[t], brow[t * (S1L_NMAX + 4) + 16 * j], c, 0,
                                                     0, 0);
          acc[j] = c;
        }
      }
    } else {
      unsigned short hs[8], ms[8], ls[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        hs[t] = bf16_rne(ak[t]);
        const float r1 = ak[t] - bf16_to_f(hs[t]);
        ms[t] = bf16_rne(r1);
        ls[t] = bf16_rne(r1 - bf16_to_f(ms[t]));
      }
      const bf8 ah = __builtin_bit_cast(bf8, hs), am = __builtin_bit_cast(bf8, ms),
                al = __builtin_bit_cast(bf8, ls);
#pragma unroll
      for (int j = 0; j < NTW; ++j) {
        const int tj = hf * NTW + j;
        if (tj < ntiles) {
          const int col = 16 * tj + l16;
          const bf8 bh = ld_bf8(&sm.b[buf][0][col][8 * g]);
          const bf8 bm = ld_bf8(&sm.b[buf][1][col][8 * g]);
          f4 c = acc[j];
          if (nterms >= 6) {
            const bf8 bl = ld_bf8(&sm.b[buf][2][col][8 * g]);
            // small terms first so that they are not absorbed by the large one
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bm, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
          }
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bh, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bm, c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
          acc[j] = c;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[j][r] += (double)acc[j][r];
  };
  double2 a0[4], a1[4];
  u32x4 bs0[UPT], bs1[UPT];
  load_a(a0, 0);
  load_b(bs0, 0);
  load_a(a1, min(S1L_KS, k2p - S1L_KS));
  load_b(bs1, min(S1L_KS, k2p - S1L_KS));
  for (int sl = 0; sl < nslices; sl += 2) {
    slice(sl, a0, bs0);
    if (sl + 1 < nslices) slice(sl + 1, a1, bs1);
  }
  double* Td = (double*)T;
#pragma unroll
  for (int j = 0; j < NTW; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + rg * 16 + 4 * g + r, n2 = col0 + 16 * (hf * NTW + j) + l16;
      if (hf * NTW + j < ntiles && m < rows && n2 < 2 * ng) Td[((int64_t)s0 * R + m) * (2 * ng) + n2] = acc64[j][r];
    }
}

// ---------------------------------------------------------------- exchange
// C (column-major, ld; upper tiles) = alpha * conj(Mcv) diag(vbar) Mcv^T
template <int PREC, int BN2>
__global__ __launch_bounds__(256) void k_exchange_lp(const double2* __restrict__ Mcv, int n, int ng,
                                                     const double* __restrict__ vbar, double alpha,
                                                     int nterms, double2* __restrict__ C,
                                                     int64_t ld, const int32_t* info) {
  __shared__ LpSmem<PREC, BN2> sm;
  if (failed(info)) return;
  const int m0 = blockIdx.x * LBM, n0c = blockIdx.y * (BN2 / 2);
  if (m0 > n0c + BN2 / 2 - 1) return;  // strictly below the diagonal
  auto ga = [&](int mm, int k) -> double2 {
    const int m = m0 + mm;
    if (m >= n || k >= ng) return make_double2(0.0, 0.0);
    const double2 v = Mcv[(int64_t)m * ng + k];
    const double s = vbar[k];
    return make_double2(v.x * s, -v.y * s);
  };
  auto gb = [&](int k, int nc) -> double2 {
    const int c = n0c + nc;
    if (k >= ng || c >= n) return make_double2(0.0, 0.0);
    return Mcv[(int64_t)c * ng + k];
  };
  double acc64[BN2 / 16][4];
  lp_gemm<PREC, BN2>(sm, ng, nterms, ga, gb, acc64);
  // each lane owns (re, im) pairs on adjacent lanes: gather them via a shuffle
#pragma unroll
  for (int j = 0; j < BN2 / 16; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double mine = acc64[j][r];
      const double other = __shfl_xor(mine, 1, 64);
      const int m = m0 + lp_row(r), n2 = 2 * n0c + lp_col(j);
      if ((n2 & 1) == 0) {
        const int c = n2 >> 1;
        if (m < n && c < n && m <= c) C[(int64_t)m + (int64_t)c * ld] = make_double2(alpha * mine, alpha * other);
      }
    }
}

}  // namespace

int lp_n2p(int ng) { return (2 * ng + 15) / 16 * 16; }
int lp_k2p(int ng) { return (2 * ng + S1L_KS - 1) / S1L_KS * S1L_KS; }

size_t split_w_bytes(int nq, int ng) {
  return (size_t)nq * 3 * lp_n2p(ng) * lp_k2p(ng) * 2;  // the larger of the two layouts
}

bool launch_split_w(int prec, const double2* W, int nq, int ng, void* Wsp, hipStream_t s) {
  const int n2p = lp_n2p(ng), k2p = lp_k2p(ng);
  dim3 grid((unsigned)std::min(64, cdiv((int64_t)n2p * k2p, 256)), (unsigned)nq);
  if (prec == BSE_PREC_FP32)
    BSE_LAUNCH((k_split_w<BSE_PREC_FP32>), grid, dim3(256), 0, s, W, ng, n2p, k2p, Wsp);
  else
    BSE_LAUNCH((k_split_w<BSE_PREC_BF16X3>), grid, dim3(256), 0, s, W, ng, n2p, k2p, Wsp);
  return hipGetLastError() == hipSuccess;
}

bool launch_stage1_lp(int prec, int nterms, const double2* left, int R, int ng, const void* Wsp,
                      const int32_t* perm, const int32_t* cls, int nq, int nk, double2* T,
                      const int32_t* info, hipStream_t s) {
  const int n2p = lp_n2p(ng), k2p = lp_k2p(ng);
  const int tiles = cdiv((int64_t)nk * R, S1L_BM);
  dim3 grid((unsigned)(nq * tiles), (unsigned)cdiv(n2p, S1L_NMAX));
  if (prec == BSE_PREC_FP32)
    BSE_LAUNCH((k_stage1_lp<BSE_PREC_FP32>), grid, dim3(512), 0, s, left, R, ng, Wsp, n2p, k2p,
               perm, cls, tiles, nterms, T, info);
  else
    BSE_LAUNCH((k_stage1_lp<BSE_PREC_BF16X3>), grid, dim3(512), 0, s, left, R, ng, Wsp, n2p, k2p,
               perm, cls, tiles, nterms, T, info);
  return hipGetLastError() == hipSuccess;
}

bool launch_exchange_lp(int prec, int nterms, const double2* Mcv, int n, int ng,
                        const double* vbar, double alpha, double2* C, int64_t ld,
                        const int32_t* info, hipStream_t s) {
  dim3 grid((unsigned)cdiv(n, LBM), (unsigned)cdiv(n, 32));
  if (prec == BSE_PREC_FP32)
    BSE_LAUNCH((k_exchange_lp<BSE_PREC_FP32, 64>), grid, dim3(256), 0, s, Mcv, n, ng, vbar, alpha,
               nterms, C, ld, info);
  else
    BSE_LAUNCH((k_exchange_lp<BSE_PREC_BF16X3, 64>), grid, dim3(256), 0, s, Mcv, n, ng, vbar,
               alpha, nterms, C, ld, info);
  return hipGetLastError() == hipSuccess;
}
