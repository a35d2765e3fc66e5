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
template <int PREC, int BN2>
__global__ __launch_bounds__(256) void k_stage1_lp(const double2* __restrict__ Left, int R, int ng,
                                                   const double2* __restrict__ W,
                                                   const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ cls,
                                                   int tiles_per_class, int nterms,
                                                   double2* __restrict__ T, const int32_t* info) {
  __shared__ LpSmem<PREC, BN2> sm;
  if (failed(info)) return;
  const int q = blockIdx.x / tiles_per_class, mt = blockIdx.x % tiles_per_class;
  const int s0 = cls[q], rows = (cls[q + 1] - s0) * R;
  const int m0 = mt * LBM;
  if (m0 >= rows) return;
  const int n0c = blockIdx.y * (BN2 / 2);
  const double2* __restrict__ Wq = W + (int64_t)q * ng * ng;
  auto ga = [&](int mm, int k) -> double2 {
    const int m = m0 + mm;
    if (m >= rows || k >= ng) return make_double2(0.0, 0.0);
    const int64_t p = perm[s0 + m / R];
    const double2 v = Left[(p * R + m % R) * ng + k];
    return make_double2(v.x, -v.y);
  };
  auto gb = [&](int k, int nc) -> double2 {
    const int n = n0c + nc;
    if (k >= ng || n >= ng) return make_double2(0.0, 0.0);
    return Wq[(int64_t)k * ng + n];
  };
  double acc64[BN2 / 16][4];
  lp_gemm<PREC, BN2>(sm, ng, nterms, ga, gb, acc64);
  double* Td = (double*)T;
#pragma unroll
  for (int j = 0; j < BN2 / 16; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + lp_row(r), n2 = 2 * n0c + lp_col(j);
      if (m < rows && n2 < 2 * ng) Td[((int64_t)s0 * R + m) * (2 * ng) + n2] = acc64[j][r];
    }
}

// ---------------------------------------------------------------- batched stage 2
// blk[b] (M x N) = T[b] (M x K) x Right[perm[b]]^T, Right[p] stored (N x K)
template <int PREC, int BN2>
__global__ __launch_bounds__(256) void k_batched_lp(const double2* __restrict__ A, int M, int K,
                                                    const double2* __restrict__ Bm, int N,
                                                    const int32_t* __restrict__ bidx, int nterms,
                                                    double2* __restrict__ C, int b_off,
                                                    const int32_t* info) {
  __shared__ LpSmem<PREC, BN2> sm;
  if (failed(info)) return;
  const int b = blockIdx.z + b_off;
  const int m0 = blockIdx.x * LBM, n0c = blockIdx.y * (BN2 / 2);
  const double2* __restrict__ Ab = A + (int64_t)b * M * K;
  const double2* __restrict__ Bb = Bm + (int64_t)bidx[b] * N * K;
  auto ga = [&](int mm, int k) -> double2 {
    const int m = m0 + mm;
    if (m >= M || k >= K) return make_double2(0.0, 0.0);
    return Ab[(int64_t)m * K + k];
  };
  auto gb = [&](int k, int nc) -> double2 {
    const int n = n0c + nc;
    if (k >= K || n >= N) return make_double2(0.0, 0.0);
    return Bb[(int64_t)n * K + k];
  };
  double acc64[BN2 / 16][4];
  lp_gemm<PREC, BN2>(sm, K, nterms, ga, gb, acc64);
  double* Cd = (double*)(C + (int64_t)b * M * N);
#pragma unroll
  for (int j = 0; j < BN2 / 16; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + lp_row(r), n2 = 2 * n0c + lp_col(j);
      if (m < M && n2 < 2 * N) Cd[(int64_t)m * (2 * N) + n2] = acc64[j][r];
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

bool launch_stage1_lp(int prec, int nterms, const double2* left, int R, int ng, const double2* W,
                      const int32_t* perm, const int32_t* cls, int nq, int nk, double2* T,
                      const int32_t* info, hipStream_t s) {
  const int tiles = cdiv((int64_t)nk * R, LBM);
  dim3 grid((unsigned)(nq * tiles), (unsigned)cdiv(ng, 32));
  if (prec == BSE_PREC_FP32)
    BSE_LAUNCH((k_stage1_lp<BSE_PREC_FP32, 64>), grid, dim3(256), 0, s, left, R, ng, W, perm, cls,
               tiles, nterms, T, info);
  else
    BSE_LAUNCH((k_stage1_lp<BSE_PREC_BF16X3, 64>), grid, dim3(256), 0, s, left, R, ng, W, perm,
               cls, tiles, nterms, T, info);
  return hipGetLastError() == hipSuccess;
}

bool launch_batched_lp(int prec, int nterms, const double2* A, int M, int K, const double2* B,
                       int N, const int32_t* bidx, int batch, double2* C, const int32_t* info,
                       hipStream_t s) {
  for (int b0 = 0; b0 < batch; b0 += 65535) {
    const int nb = std::min(65535, batch - b0);
    dim3 grid((unsigned)cdiv(M, LBM), (unsigned)cdiv(N, 32), (unsigned)nb);
    if (prec == BSE_PREC_FP32)
      BSE_LAUNCH((k_batched_lp<BSE_PREC_FP32, 64>), grid, dim3(256), 0, s, A, M, K, B, N, bidx,
                 nterms, C, b0, info);
    else
      BSE_LAUNCH((k_batched_lp<BSE_PREC_BF16X3, 64>), grid, dim3(256), 0, s, A, M, K, B, N, bidx,
                 nterms, C, b0, info);
  }
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
