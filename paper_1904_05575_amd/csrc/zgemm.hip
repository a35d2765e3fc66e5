// Strided / batched complex FP64 GEMM on MFMA (see zgemm.h).
#include <algorithm>
#include <vector>

#include "bse_internal.h"
#include "common.h"
#include "mfma_tile.h"
#include "timing.h"
#include "zgemm.h"

namespace {

// One output tile (bx, by) of batch entry b.
template <int BM, int BN, int WM, int WN, bool G3>
BSE_DEV void zgemm_tile(const ZgemmParams& p, int bx, int by, int b) {
  using T = ZTile<BM, BN, WM, WN, G3>;
  __shared__ typename T::Smem2 sm;
  if (failed(p.info)) return;
  const int m0 = bx * BM, n0 = by * BN;
  if (p.c_uplo == 1 && m0 > n0 + BN - 1) return;
  if (p.c_uplo == 2 && n0 > m0 + BM - 1) return;
  const int64_t bb = p.b_batch_idx ? (int64_t)p.b_batch_idx[b] : (int64_t)b;
  const double2* __restrict__ A = p.A + b * p.a_bs;
  const double2* __restrict__ B = p.B + bb * p.b_bs;
  const double* __restrict__ ks = p.kscale ? p.kscale + b * p.ks_bs : nullptr;

  int k_lo = 0, k_hi = p.K;
  if (p.a_tri == 1) k_lo = max(k_lo, m0);
  if (p.a_tri == 2) k_hi = min(k_hi, m0 + BM);
  if (p.b_tri == 1) k_hi = min(k_hi, n0 + BN);
  if (p.b_tri == 2) k_lo = max(k_lo, n0);

  const double asgn = p.conjA ? -1.0 : 1.0, bsgn = p.conjB ? -1.0 : 1.0;
  const int mlast = p.M - 1, nlast = p.N - 1, klast = p.K - 1;
  auto addrA = [&](int mm, int k, bool& ok) -> const double2* {
    const int m = m0 + mm;
    ok = m < p.M && k < p.K;
    if (p.a_tri == 1) ok = ok && (k >= m);
    if (p.a_tri == 2) ok = ok && (k <= m);
    return A + (int64_t)min(m, mlast) * p.a_rs + (int64_t)min(k, klast) * p.a_cs;
  };
  auto addrB = [&](int k, int nn, bool& ok) -> const double2* {
    const int n = n0 + nn;
    ok = n < p.N && k < p.K;
    if (p.b_tri == 1) ok = ok && (k <= n);
    if (p.b_tri == 2) ok = ok && (k >= n);
    return B + (int64_t)min(k, klast) * p.b_rs + (int64_t)min(n, nlast) * p.b_cs;
  };
  auto fixA = [&](double2 v, int k) -> double2 {
    v.y *= asgn;
    if (ks) {
      const double s = ks[k];
      v.x *= s;
      v.y *= s;
    }
    return v;
  };
  auto fixB = [&](double2 v, int) -> double2 {
    v.y *= bsgn;
    return v;
  };
  T t;
  t.init();
  t.run_pf(sm, k_lo, k_hi, p.a_rs == 1, p.b_cs == 1, addrA, addrB, fixA, fixB);

  double2* C = p.C + b * p.c_bs;
  t.store([&](int mm, int nn, double2 acc) {
    const int m = m0 + mm, n = n0 + nn;
    if (m >= p.M || n >= p.N) return;
    if (p.c_uplo == 1 && m > n) return;
    if (p.c_uplo == 2 && m < n) return;
    double2 v = cmul(p.alpha, acc);
    if (p.ndiv) v = cscale(v, 1.0 / p.ndiv[n]);
    double2* dst = C + (int64_t)m * p.c_rs + (int64_t)n * p.c_cs;
    if (p.beta != 0.0) {
      const double2 o = *dst;
      v.x += p.beta * o.x;
      v.y += p.beta * o.y;
    }
    *dst = v;
  });
}

template <int BM, int BN, int WM, int WN, bool G3>
__global__ __launch_bounds__(WM* WN * 64) void zgemm_kernel(ZgemmParams p, int b_off) {
  zgemm_tile<BM, BN, WM, WN, G3>(p, blockIdx.x, blockIdx.y, blockIdx.z + b_off);
}

// Square products that store one triangle (c_uplo 1 or 2, M = N, square
// tiles) run on the triangle's tiles only: tile t of the nt (nt + 1) / 2 is
// (I, J), I >= J, in row order of the lower triangle, i.e. (bx, by) = (I, J)
// for the lower triangle and (J, I) for the upper one.
BSE_DEV void tri_tile(int64_t t, int uplo, int& bx, int& by) {
  int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  if ((int64_t)(I + 1) * (I + 2) / 2 <= t) ++I;
  if ((int64_t)I * (I + 1) / 2 > t) --I;
  const int J = (int)(t - (int64_t)I * (I + 1) / 2);
  bx = uplo == 2 ? I : J;
  by = uplo == 2 ? J : I;
}

template <int BM, int BN, int WM, int WN, bool G3>
__global__ __launch_bounds__(WM* WN * 64) void zgemm_tri_kernel(ZgemmParams p, int b_off) {
  int bx, by;
  tri_tile((int64_t)blockIdx.x, p.c_uplo, bx, by);
  zgemm_tile<BM, BN, WM, WN, G3>(p, bx, by, blockIdx.z + b_off);
}

// Products of different shapes and operands (blockIdx.z = item), the rest of
// the parameters shared; the items travel by value so that every operand load
// is a global load.
template <int BM, int BN, int WM, int WN, bool G3>
__global__ __launch_bounds__(WM* WN * 64) void zgemm_group_kernel(ZgemmParams base, ZgemmGroup g) {
  int i = 0;  // the item that owns this block (uniform scan of the ranges)
  while (i + 1 < ZGEMM_GROUP_MAX && (int)blockIdx.x >= g.first[i + 1]) ++i;
  const ZgemmItem& q = g.it[i];
  const int64_t t = (int64_t)blockIdx.x - g.first[i];  // the item's tile
  int bx, by;
  if (base.c_uplo != 0 && q.M == q.N && BM == BN) {
    tri_tile(t, base.c_uplo, bx, by);
  } else {
    const int gm = cdiv(q.M, BM);
    bx = (int)(t % gm);
    by = (int)(t / gm);
  }
  if (bx * BM >= q.M || by * BN >= q.N) return;
  ZgemmParams p = base;
  p.M = q.M;
  p.N = q.N;
  p.K = q.K;
  p.A = q.A;
  p.a_rs = q.a_rs;
  p.a_cs = q.a_cs;
  p.B = q.B;
  p.b_rs = q.b_rs;
  p.b_cs = q.b_cs;
  p.C = q.C;
  p.c_rs = q.c_rs;
  p.c_cs = q.c_cs;
  p.info = q.info;
  p.a_tri = q.a_tri;
  p.b_tri = q.b_tri;
  zgemm_tile<BM, BN, WM, WN, G3>(p, bx, by, 0);
}

template <int BM, int BN, int WM, int WN, bool G3>
hipError_t launch_group(const ZgemmParams& base, ZgemmGroup g, int count, hipStream_t s) {
  int64_t total = 0;  // compact grid: each item's tiles (its triangle's, when it stores one)
  for (int i = 0; i < ZGEMM_GROUP_MAX; ++i) {
    g.first[i] = (int32_t)total;
    if (i >= count) continue;
    const ZgemmItem& q = g.it[i];
    const int64_t gm = cdiv(q.M, BM), gn = cdiv(q.N, BN);
    total += (base.c_uplo != 0 && q.M == q.N && BM == BN) ? gm * (gm + 1) / 2 : gm * gn;
  }
  g.first[ZGEMM_GROUP_MAX] = (int32_t)total;
  if (total == 0) return hipSuccess;
  TimedLaunch tl(base.tag, s);
  if (tl.a)
    hipExtLaunchKernelGGL((zgemm_group_kernel<BM, BN, WM, WN, G3>), dim3((unsigned)total),
                          dim3(WM * WN * 64), 0, s, tl.a, tl.b, 0, base, g);
  else
    hipLaunchKernelGGL((zgemm_group_kernel<BM, BN, WM, WN, G3>), dim3((unsigned)total),
                       dim3(WM * WN * 64), 0, s, base, g);
  launch_check(base.tag);
  return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, bool G3>
hipError_t launch(const ZgemmParams& p, int batch, hipStream_t s) {
  TimedLaunch tl(p.tag, s);
  const bool tri = p.c_uplo != 0 && p.M == p.N && BM == BN;  // the triangle's tiles only
  const int64_t nt = cdiv(p.M, BM);
  // a timed product spans its first and last chunk of at most 65535 batch entries
  for (int b0 = 0; b0 < batch; b0 += 65535) {
    const int nb = batch - b0 < 65535 ? batch - b0 : 65535;
    const dim3 grid = tri ? dim3((unsigned)(nt * (nt + 1) / 2), 1, nb)
                          : dim3(cdiv(p.M, BM), cdiv(p.N, BN), nb);
    const bool first = b0 == 0, last = b0 + nb >= batch;
    if (tri && tl.a)
      hipExtLaunchKernelGGL((zgemm_tri_kernel<BM, BN, WM, WN, G3>), grid, dim3(WM * WN * 64), 0,
                            s, first ? tl.a : nullptr, last ? tl.b : nullptr, 0, p, b0);
    else if (tri)
      hipLaunchKernelGGL((zgemm_tri_kernel<BM, BN, WM, WN, G3>), grid, dim3(WM * WN * 64), 0, s,
                         p, b0);
    else if (tl.a)
      hipExtLaunchKernelGGL((zgemm_kernel<BM, BN, WM, WN, G3>), grid, dim3(WM * WN * 64), 0, s,
                            first ? tl.a : nullptr, last ? tl.b : nullptr, 0, p, b0);
    else
      hipLaunchKernelGGL((zgemm_kernel<BM, BN, WM, WN, G3>), grid, dim3(WM * WN * 64), 0, s, p, b0);
    launch_check(p.tag);
  }
  return hipGetLastError();
}

// Tile edge: the caller's choice, else from the shape.
int tile_edge(const ZgemmParams& p, int batch) {
  if (p.tile == 16 || p.tile == 32 || p.tile == 64) return p.tile;
  if (p.M <= 16 && p.N <= 16) return 16;
  if (p.M <= 32 || p.N <= 32 || (int64_t)cdiv(p.M, 64) * cdiv(p.N, 64) * batch < 512) return 32;
  return 64;
}

}  // namespace

// Gauss's three products take a third more accumulators; measured at N = 6144
// they pay on the 16- and 32-edge tiles (Householder and Cholesky updates,
// exchange) and lose on the 64-edge tile, whose four-product form is kept.
// Each item takes the tile edge and the products per complex one that zgemm()
// would take for it alone, so that its values are those of that call; items
// sharing both go into one launch.
hipError_t zgemm_group(const ZgemmParams& base, const ZgemmItem* items, int count,
                       hipStream_t s) {
  std::vector<int> key(count, -1);
  for (int i = 0; i < count; ++i) {
    if (items[i].M <= 0 || items[i].N <= 0) continue;
    ZgemmParams one = base;
    one.M = items[i].M;
    one.N = items[i].N;
    const int prods = base.products ? base.products
                                    : tune_choice(BSE_TUNE_GEMM_PRODUCTS,
                                                  std::max(one.M, one.N), 3);
    const int edge = tile_edge(one, 1);
    key[i] = edge * 8 + (edge == 64 ? 4 : prods);
  }
  std::vector<char> done(count, 0);
  for (int i = 0; i < count; ++i) {
    if (key[i] < 0 || done[i]) continue;
    ZgemmGroup g{};
    int ng = 0;
    for (int j = i; j < count && ng < ZGEMM_GROUP_MAX; ++j)
      if (!done[j] && key[j] == key[i]) {
        g.it[ng++] = items[j];
        done[j] = 1;
      }
    hipError_t e;
    switch (key[i]) {
      case 16 * 8 + 3:
        e = launch_group<16, 16, 1, 1, true>(base, g, ng, s);
        break;
      case 16 * 8 + 4:
        e = launch_group<16, 16, 1, 1, false>(base, g, ng, s);
        break;
      case 32 * 8 + 3:
        e = launch_group<32, 32, 2, 2, true>(base, g, ng, s);
        break;
      case 32 * 8 + 4:
        e = launch_group<32, 32, 2, 2, false>(base, g, ng, s);
        break;
      default:
        e = launch_group<64, 64, 2, 2, false>(base, g, ng, s);
    }
    if (e != hipSuccess) return e;  // items of this key past the first launch: later in the loop
  }
  return hipSuccess;
}

hipError_t zgemm(const ZgemmParams& p, int batch, hipStream_t s) {
  if (p.M <= 0 || p.N <= 0 || batch <= 0) return hipSuccess;
  const int prods = p.products ? p.products
                               : tune_choice(BSE_TUNE_GEMM_PRODUCTS, std::max(p.M, p.N), 3);
  switch (tile_edge(p, batch)) {
    case 16:
      return prods == 3 ? launch<16, 16, 1, 1, true>(p, batch, s)
                        : launch<16, 16, 1, 1, false>(p, batch, s);
    case 32:
      return prods == 3 ? launch<32, 32, 2, 2, true>(p, batch, s)
                        : launch<32, 32, 2, 2, false>(p, batch, s);
    default:
      return launch<64, 64, 2, 2, false>(p, batch, s);
  }
}
