// Plane-wave pair elements from orbitals (paper Sec. 4.1, for orbitals
// expanded in plane waves: the cell integral of the orbital product keeps the
// plane waves whose wave vectors cancel):
//   M_mn(k, k', G) = sum_K conj(C_m,k(K)) C_n,k'(K + G)
//   N_mn(k, k', G) = sum_K conj(C_m,k(K)) conj(C_n,k'(-K - G))
// over the orbitals' plane-wave sphere K (terms whose partner K + G or -K - G
// lies outside it are absent).  For every pair p = (ik <= ik') one block
// stages the two k-points' coefficients in LDS and forms every element the
// BSE inputs take: Mvv, Mcc (and Ncv, Nvc for the full BSE), and M_cv at
// k = k' on the diagonal pairs.  A thread owns one G of one band block of at
// most 4 x 4 and accumulates the block's outer products over K in registers;
// the partner positions come from a [K][G] table (G fastest, so that the
// lanes of a wavefront read it coalesced).
#include "bse_internal.h"
#include "common.h"
#include "timing.h"

namespace {

constexpr int PG_THREADS = 256;
constexpr int PG_MAXB = 4;       // bands of a block on either side
constexpr int PG_MAXKINDS = 24;

struct PgKind {
  double2* out;          // element (a, b, G) of pair p at out + p ps + a as + b bs + G
  int64_t ps, as, bs;
  int a0, na, b0, nb;    // band ranges (into the nv + nc bands of a k-point)
  int ia, ib;            // first local index of this block within the array's a / b
  int modified;          // N-type element
  int diag_only;         // only diagonal pairs, p taken as ik (M_cv)
};
struct PgKinds {
  PgKind k[PG_MAXKINDS];
  int n;
};

__global__ __launch_bounds__(PG_THREADS) void k_pair_elements(
    const double2* __restrict__ C, int nk, int nbt, int nkb, int ng,
    const int32_t* __restrict__ kpg, const int32_t* __restrict__ mkg, PgKinds kinds) {
  extern __shared__ double2 cs[];  // [2][nbt][nkb]: bands at k, bands at k'
  const int p = blockIdx.x;
  // pair p -> (ik, jk), p = ik nk - ik (ik - 1) / 2 + (jk - ik)
  int ik = 0;
  {
    int lo = 0, hi = nk - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      const int64_t start = (int64_t)mid * nk - (int64_t)mid * (mid - 1) / 2;
      if (start <= p) lo = mid; else hi = mid - 1;
    }
    ik = lo;
  }
  const int jk = ik + (int)(p - ((int64_t)ik * nk - (int64_t)ik * (ik - 1) / 2));
  const int per = nbt * nkb;
  for (int e = threadIdx.x; e < 2 * per; e += PG_THREADS) {
    const int side = e / per, r = e % per;
    cs[e] = C[(int64_t)(side ? jk : ik) * per + r];
  }
  __syncthreads();
  const double2* __restrict__ ca = cs;
  const double2* __restrict__ cb = cs + per;
  // work items: (kind, G)
  int nitems = 0;
  for (int t = 0; t < kinds.n; ++t)
    if (!kinds.k[t].diag_only || ik == jk) nitems += ng;
  for (int it = threadIdx.x; it < nitems; it += PG_THREADS) {
    int t = 0, rest = it;
    for (; t < kinds.n; ++t) {
      if (kinds.k[t].diag_only && ik != jk) continue;
      if (rest < ng) break;
      rest -= ng;
    }
    const PgKind kd = kinds.k[t];
    const int g = rest;
    const int32_t* __restrict__ tab = kd.modified ? mkg : kpg;
    double2 acc[PG_MAXB][PG_MAXB];
#pragma unroll
    for (int a = 0; a < PG_MAXB; ++a)
#pragma unroll
      for (int b = 0; b < PG_MAXB; ++b) acc[a][b] = make_double2(0.0, 0.0);
    for (int K = 0; K < nkb; ++K) {
      const int bp = tab[(int64_t)K * ng + g];
      if (bp < 0 || bp >= nkb) continue;  // outside the sphere
      double2 x[PG_MAXB], y[PG_MAXB];
#pragma unroll
      for (int a = 0; a < PG_MAXB; ++a) {
        const double2 v = ca[(kd.a0 + min(a, kd.na - 1)) * nkb + K];
        x[a] = make_double2(v.x, -v.y);  // conj(C_m,k(K))
      }
#pragma unroll
      for (int b = 0; b < PG_MAXB; ++b) {
        const double2 v = cb[(kd.b0 + min(b, kd.nb - 1)) * nkb + bp];
        y[b] = kd.modified ? make_double2(v.x, -v.y) : v;
      }
#pragma unroll
      for (int a = 0; a < PG_MAXB; ++a)
#pragma unroll
        for (int b = 0; b < PG_MAXB; ++b) {
          acc[a][b].x = fma(x[a].x, y[b].x, fma(-x[a].y, y[b].y, acc[a][b].x));
          acc[a][b].y = fma(x[a].x, y[b].y, fma(x[a].y, y[b].x, acc[a][b].y));
        }
    }
    const int64_t base = (int64_t)(kd.diag_only ? ik : p) * kd.ps + g;
#pragma unroll
    for (int a = 0; a < PG_MAXB; ++a)
#pragma unroll
      for (int b = 0; b < PG_MAXB; ++b)
        if (a < kd.na && b < kd.nb)
          kd.out[base + (int64_t)(kd.ia + a) * kd.as + (int64_t)(kd.ib + b) * kd.bs] = acc[a][b];
  }
}

// Blocks of at most PG_MAXB x PG_MAXB bands covering an (na_tot x nb_tot)
// array of elements, appended to the list.
bool add_blocks(PgKinds& ks, double2* out, int64_t ps, int64_t as, int64_t bs, int a0,
                int na_tot, int b0, int nb_tot, int modified, int diag_only) {
  for (int ia = 0; ia < na_tot; ia += PG_MAXB)
    for (int ib = 0; ib < nb_tot; ib += PG_MAXB) {
      if (ks.n >= PG_MAXKINDS) return false;
      PgKind& k = ks.k[ks.n++];
      k.out = out;
      k.ps = ps;
      k.as = as;
      k.bs = bs;
      k.a0 = a0 + ia;
      k.na = std::min(PG_MAXB, na_tot - ia);
      k.b0 = b0 + ib;
      k.nb = std::min(PG_MAXB, nb_tot - ib);
      k.ia = ia;
      k.ib = ib;
      k.modified = modified;
      k.diag_only = diag_only;
    }
  return true;
}

}  // namespace

extern "C" {

bse_status bse_pair_elements(const bse_orb_desc* d, const void* C, const int32_t* kpg,
                             const int32_t* mkg, void* Mcv, void* Mvv, void* Mcc, void* Ncv,
                             void* Nvc, hipStream_t stream) {
  launch_failure_reset();
  if (!d || d->nk <= 0 || d->nv <= 0 || d->nc <= 0 || d->ng <= 0 || d->nkb <= 0) return BSE_ERR_ARG;
  if (d->nk > 46340) return BSE_ERR_ARG;
  const bool full = d->coupling == BSE_FULL;
  if (d->coupling != BSE_FULL && d->coupling != BSE_TDA) return BSE_ERR_ARG;
  if (!C || !kpg || !Mcv || !Mvv || !Mcc) return BSE_ERR_ARG;
  if (full && (!mkg || !Ncv || !Nvc)) return BSE_ERR_ARG;
  const int nv = d->nv, nc = d->nc, ng = d->ng, nkb = d->nkb, nbt = nv + nc;
  const size_t lds = (size_t)2 * nbt * nkb * sizeof(double2);
  if (lds > 160 * 1024) return BSE_ERR_ARG;
  PgKinds ks{};
  const int64_t G = ng;
  bool ok = add_blocks(ks, (double2*)Mvv, (int64_t)nv * nv * G, nv * G, G, 0, nv, 0, nv, 0, 0) &&
            add_blocks(ks, (double2*)Mcc, (int64_t)nc * nc * G, nc * G, G, nv, nc, nv, nc, 0, 0) &&
            add_blocks(ks, (double2*)Mcv, (int64_t)nv * nc * G, nc * G, G, 0, nv, nv, nc, 0, 1);
  if (ok && full)
    ok = add_blocks(ks, (double2*)Ncv, (int64_t)nc * nv * G, nv * G, G, nv, nc, 0, nv, 1, 0) &&
         add_blocks(ks, (double2*)Nvc, (int64_t)nv * nc * G, nc * G, G, 0, nv, nv, nc, 1, 0);
  if (!ok) return BSE_ERR_ARG;  // too many band blocks for one launch
  const int64_t P = (int64_t)d->nk * (d->nk + 1) / 2;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_pair_elements,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return BSE_ERR_HIP;
  BSE_LAUNCH(k_pair_elements, dim3((unsigned)P), dim3(PG_THREADS), lds, stream,
             (const double2*)C, d->nk, nbt, nkb, ng, kpg, full ? mkg : kpg, ks);
  return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
}

}  // extern "C"
