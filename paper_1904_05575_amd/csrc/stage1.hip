// Stage 1 of the direct terms (paper Sec. 4.2, eqs. wrrm and wrabar), grouped
// by momentum-transfer class q:
//   T[pos*R + sub, G'] = sum_G conj(L[p][sub][G]) W[q][G][G'],   p = perm[pos]
//
// The complex product is computed as one real GEMM on the FP64 matrix cores
// by viewing interleaved complex arrays as real ones:
//   A  (rows x 2K)  = conj(L) read as doubles (re, -im, re, -im, ...)
//   B' (2K x 2N)    row 2k   = W[k] as doubles   (re0, im0, re1, im1, ...)
//                   row 2k+1 = i W[k] as doubles (-im0, re0, -im1, re1, ...)
//   C  (rows x 2N)  = T read as doubles
// so that C[m][2n] = Re T and C[m][2n+1] = Im T.  Padding then follows 2*NG
// (226 -> 240 for NG = 113) instead of NG (113 -> 128) in both K and N.
#include "bse_internal.h"
#include "common.h"
#include "timing.h"

namespace {

constexpr int BM = 64;    // pair rows per block (4 row groups of 16)
constexpr int BK = 16;    // real k per LDS stage (8 complex k, 4 MFMA k-steps)
constexpr int NTHR = 512; // 8 waves: 4 row groups x 2 halves of the columns
constexpr int APAD = 4;

template <int BN2>
struct S1Smem {
  double a[2][BK][BM + APAD];
  double b[2][BK][BN2 + 4];
};

template <int BN2>
__global__ __launch_bounds__(NTHR, (BN2 == 240 || BN2 == 192) ? 4 : 2) void k_stage1_real(const double2* __restrict__ Left, int R,
                                                      int ng, const double2* __restrict__ W,
                                                      const int32_t* __restrict__ perm,
                                                      const int32_t* __restrict__ cls,
                                                      int tiles_per_class,
                                                      double2* __restrict__ T,
                                                      const int32_t* info) {
  constexpr int NT = BN2 / 16;
  constexpr int NTH = (NT + 1) / 2;  // column tiles per wave
  constexpr int BPER = (BK / 2 * BN2 + NTHR - 1) / NTHR;
  __shared__ S1Smem<BN2> sm;
  if (failed(info)) return;
  const int q = blockIdx.x / tiles_per_class, mt = blockIdx.x % tiles_per_class;
  const int s0 = cls[q], rows = (cls[q + 1] - s0) * R;
  const int m0 = mt * BM;
  if (m0 >= rows) return;
  const int K2 = 2 * ng, N2 = 2 * ng;
  const double* __restrict__ Wq = (const double*)(W + (int64_t)q * ng * ng);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int mg = wid & 3, nh = wid >> 2;
  const int jt0 = nh * NTH;

  // A staging: thread -> (row, one complex k); rows past the class are
  // clamped to a valid row and zeroed when stored
  const int arow = tid >> 3, akc = tid & 7;
  const bool arow_ok = (m0 + arow) < rows;
  const double2* arow_ptr;
  {
    const int m = arow_ok ? (m0 + arow) : m0;
    const int64_t p = perm[s0 + m / R];
    arow_ptr = Left + (p * R + m % R) * ng;
  }
  // one chunk's loads in registers; two sets, so that the loads of chunk
  // ch + 2 are in flight while chunk ch is multiplied
  struct Regs {
    double2 ra;
    double rb[BPER];
  };

  auto load_chunk = [&](Regs& g_, int k0) {
    const int kc = (k0 >> 1) + akc;  // complex k
    g_.ra = arow_ptr[kc < ng ? kc : ng - 1];
#pragma unroll
    for (int u = 0; u < BPER; ++u) {
      const int e = tid + u * NTHR;
      const int wr = e / BN2, nn = e % BN2;
      int g = (k0 >> 1) + wr;
      g = g < ng ? g : ng - 1;
      const int nc = nn < N2 ? nn : N2 - 1;
      g_.rb[u] = Wq[(int64_t)g * N2 + nc];
    }
  };
  auto store_chunk = [&](int buf, const Regs& g_, int k0) {
    const double2 ra = g_.ra;
    const double* rb = g_.rb;
    const int kc = (k0 >> 1) + akc;
    const bool okA = arow_ok && kc < ng;
    sm.a[buf][2 * akc][arow] = okA ? ra.x : 0.0;
    sm.a[buf][2 * akc + 1][arow] = okA ? -ra.y : 0.0;  // conj
#pragma unroll
    for (int u = 0; u < BPER; ++u) {
      const int e = tid + u * NTHR;
      const int wr = e / BN2, nn = e % BN2;
      const double partner = __shfl_xor(rb[u], 1, 64);
      if (e < BK / 2 * BN2) {
        const bool ok = ((k0 >> 1) + wr) < ng && nn < N2;
        sm.b[buf][2 * wr][nn] = ok ? rb[u] : 0.0;
        // row of i W[g]: (re, im) -> (-im, re)
        sm.b[buf][2 * wr + 1][nn] = ok ? ((nn & 1) ? partner : -partner) : 0.0;
      }
    }
  };

  d4 acc[NTH];
#pragma unroll
  for (int j = 0; j < NTH; ++j) acc[j] = d4{0, 0, 0, 0};

  const int nchunks = (K2 + BK - 1) / BK;
  Regs R0, R1;
  load_chunk(R0, 0);
  store_chunk(0, R0, 0);
  if (nchunks > 1) load_chunk(R1, BK);
  if (nchunks > 2) load_chunk(R0, 2 * BK);
  __syncthreads();
  // step ch: multiply chunk ch (LDS buffer ch & 1), store chunk ch + 1 from
  // `next` into the other buffer, then reuse `next` for chunk ch + 3
  auto step = [&](int ch, Regs& next) {
    const int buf = ch & 1;
    const int k0 = ch * BK;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      if (k0 + ks * 4 < K2) {
        const int kr = ks * 4 + (lane >> 4);
        const double a = sm.a[buf][kr][mg * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < NTH; ++j) {
          if (jt0 + j < NT) {
            const double b = sm.b[buf][kr][(jt0 + j) * 16 + (lane & 15)];
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
          }
        }
      }
    }
    if (ch + 1 < nchunks) store_chunk(buf ^ 1, next, (ch + 1) * BK);
    __syncthreads();
    if (ch + 3 < nchunks) load_chunk(next, (ch + 3) * BK);
  };
  for (int ch = 0; ch < nchunks; ch += 2) {
    step(ch, R1);                           // R1 holds chunk ch + 1
    if (ch + 1 < nchunks) step(ch + 1, R0);  // R0 holds chunk ch + 2
  }

  double* Td = (double*)T;
#pragma unroll
  for (int j = 0; j < NTH; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + mg * 16 + (lane >> 4) + 4 * r;
      const int nn = (jt0 + j) * 16 + (lane & 15);
      if (jt0 + j < NT && m < rows && nn < N2) Td[((int64_t)s0 * R + m) * N2 + nn] = acc[j][r];
    }
}

template <int BN2>
void launch(const double2* left, int R, int ng, const double2* W, const int32_t* perm,
            const int32_t* cls, int nq, int nk, double2* T, const int32_t* info, hipStream_t s) {
  const int tiles = cdiv((int64_t)nk * R, BM);  // a class holds at most nk pairs
  BSE_LAUNCH(k_stage1_real<BN2>, dim3((unsigned)(nq * tiles)), dim3(NTHR), 0, s, left, R, ng, W,
             perm, cls, tiles, T, info);
}

}  // namespace

// Returns false when NG is larger than the kernel's widest tile.
bool launch_stage1(const double2* left, int R, int ng, const double2* W, const int32_t* perm,
                   const int32_t* cls, int nq, int nk, double2* T, const int32_t* info,
                   hipStream_t s) {
  const int n2 = 2 * ng;
  if (n2 <= 64) launch<64>(left, R, ng, W, perm, cls, nq, nk, T, info, s);
  else if (n2 <= 128) launch<128>(left, R, ng, W, perm, cls, nq, nk, T, info, s);
  else if (n2 <= 192) launch<192>(left, R, ng, W, perm, cls, nq, nk, T, info, s);
  else if (n2 <= 240) launch<240>(left, R, ng, W, perm, cls, nq, nk, T, info, s);
  else if (n2 <= 288) launch<288>(left, R, ng, W, perm, cls, nq, nk, T, info, s);
  else return false;
  return true;
}
