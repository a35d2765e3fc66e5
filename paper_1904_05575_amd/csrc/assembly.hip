// Assembly of the BSE Hamiltonian blocks (paper Sec. 2.3 eqs. diagonalblock,
// couplingblock; Sec. 4.2 eqs. vrrofM, wrrm, wrabar).
//
//   exchange   V_aa'   = sum_G vbar_G M*_a(G) M_a'(G)           (one HERK-shaped GEMM)
//   direct     W^rr    = M*_vv W(k-k') M_cc  per k-pair          (two-stage contraction)
//   coupling   W^ra    = N*_cv W(-k-k') N_vc per k-pair
//   A+B = E + kappa (4 gx V - gc (W^rr + W^ra)),  A-B = E - kappa gc (W^rr - W^ra)
//   TDA: A = E + kappa (2 gx V - gc W^rr)
//
// Only k-pairs ik <= ik' are evaluated (the upper triangle); the lower
// triangle is the mirror and the diagonal is made real (Hermitian rule).
// The direct terms are contracted per momentum-transfer class so that every
// W(q) slice is read once per class instead of once per pair:
//   stage 1  T[pair rows, G'] = conj(M_left) x W(q)         grouped GEMM over classes
//   stage 2  blk[pair]        = T[pair] x M_right[pair]^T    batched GEMM over pairs
// followed by a scatter of the (nv nc)^2 block of every pair into A+B / A-B.
// In FP64 with stored pair elements (N_G <= 128) both stages of a term run in
// one fused pass instead (direct.hip), which adds its blocks into the outputs.
#include "bse_internal.h"
#include "common.h"
#include "mfma_tile.h"
#include "timing.h"
#include "zgemm.h"

namespace {

// ---------------------------------------------------------------- class sort
// perm[pos] lists the pairs grouped by class q = qm[ik][ik']; cls[q] is the
// first position of class q; inv[p] the position of pair p.  Block 0 sorts by
// qm0, block 1 (if qm1 is given) by qm1.  Wavefronts take rows ik, lanes ik'.
__global__ __launch_bounds__(1024) void k_class_sort(const int32_t* __restrict__ qm0,
                                                     const int32_t* __restrict__ qm1, int nk,
                                                     int nq, int32_t* perm0, int32_t* cls0,
                                                     int32_t* inv0, int32_t* perm1, int32_t* cls1,
                                                     int32_t* inv1, int32_t* info) {
  extern __shared__ int32_t sh[];
  __shared__ int32_t wtot[16];
  const int32_t* __restrict__ qm = blockIdx.x == 0 ? qm0 : qm1;
  int32_t* perm = blockIdx.x == 0 ? perm0 : perm1;
  int32_t* cls = blockIdx.x == 0 ? cls0 : cls1;
  int32_t* inv = blockIdx.x == 0 ? inv0 : inv1;
  int32_t* hist = sh;
  int32_t* cur = sh + nq;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wid = tid >> 6, nw = nt >> 6;
  for (int q = tid; q < nq; q += nt) hist[q] = 0;
  __syncthreads();
  for (int ik = wid; ik < nk; ik += nw)
    for (int jk = ik + lane; jk < nk; jk += 64) {
      const int q = qm[(int64_t)ik * nk + jk];
      if (q < 0 || q >= nq) {
        set_info(info, BSE_INFO_BAD_QMAP);
        continue;
      }
      atomicAdd(&hist[q], 1);
    }
  __syncthreads();
  // exclusive scan of hist: chunk totals per thread, scanned within each
  // wavefront by shuffles, then over the wavefront totals
  const int per = cdiv(nq, nt), q0 = min(nq, tid * per), q1 = min(nq, q0 + per);
  int tot = 0;
  for (int q = q0; q < q1; ++q) tot += hist[q];
  int incl = tot;
  for (int off = 1; off < 64; off <<= 1) {
    const int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane == 63) wtot[wid] = incl;
  __syncthreads();
  int run = incl - tot, all = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wid) run += wtot[w];
    all += wtot[w];
  }
  for (int q = q0; q < q1; ++q) {
    // a class holds at most nk pairs on a mesh (the stage-1 grid relies on it)
    if (hist[q] > nk) set_info(info, BSE_INFO_BAD_QMAP);
    cls[q] = run;
    cur[q] = run;
    run += hist[q];
  }
  if (tid == 0) cls[nq] = all;
  __syncthreads();
  for (int ik = wid; ik < nk; ik += nw) {
    const int prow = (int)((int64_t)ik * nk - (int64_t)ik * (ik - 1) / 2);
    for (int jk = ik + lane; jk < nk; jk += 64) {
      const int q = qm[(int64_t)ik * nk + jk];
      if (q < 0 || q >= nq) continue;
      const int p = prow + (jk - ik);
      const int pos = atomicAdd(&cur[q], 1);
      perm[pos] = p;
      inv[p] = pos;
    }
  }
}

// ---------------------------------------------------------------- stage 1
// T[(pos*R + sub), G'] = sum_G conj(Left[p][sub][G]) W[q][G][G'],  p = perm[pos]
constexpr int S1_BM = 64, S1_BN = 64;

__global__ __launch_bounds__(256) void k_stage1(const double2* __restrict__ Left, int R, int ng,
                                                const double2* __restrict__ W,
                                                const int32_t* __restrict__ perm,
                                                const int32_t* __restrict__ cls, int tiles_per_class,
                                                double2* __restrict__ T, const int32_t* info) {
  using Tile = ZTile<S1_BM, S1_BN, 2, 2>;
  __shared__ Tile::Smem sm;
  if (failed(info)) return;
  const int q = blockIdx.x / tiles_per_class, mt = blockIdx.x % tiles_per_class;
  const int s0 = cls[q], rows = (cls[q + 1] - s0) * R;
  const int m0 = mt * S1_BM;
  if (m0 >= rows) return;
  const int n0 = blockIdx.y * S1_BN;
  const double2* __restrict__ Wq = W + (int64_t)q * ng * ng;
  auto loadA = [&](int mm, int k) -> double2 {
    const int m = m0 + mm;
    if (m >= rows) return make_double2(0.0, 0.0);
    const int s = s0 + m / R, sub = m % R;
    const int64_t p = perm[s];
    const double2 v = Left[(p * R + sub) * ng + k];
    return make_double2(v.x, -v.y);
  };
  auto loadB = [&](int k, int nn) -> double2 {
    const int n = n0 + nn;
    if (n >= ng) return make_double2(0.0, 0.0);
    return Wq[(int64_t)k * ng + n];
  };
  Tile t;
  t.init();
  t.run(sm, 0, ng, false, true, loadA, loadB);
  t.store([&](int mm, int nn, double2 v) {
    const int m = m0 + mm, n = n0 + nn;
    if (m < rows && n < ng) T[((int64_t)s0 * R + m) * ng + n] = v;
  });
}

// ---------------------------------------------------------------- stage 2, drawn M_cc
// blk[pos][r][u u'] = sum_G' T[pos][r][G'] M[p][u][u'][G'] (p = perm[pos]) for
// pair elements given by an envelope and a key instead of an array: each
// M[p][u][u'][G'] is drawn where it is used, from the Philox4x32-10 block at
// counter (p, u, u', G') (Salmon, Moraes, Dror, Shaw, SC'11: ten rounds of two
// 32x32 -> 64-bit products, key bumped by the Weyl increments), turned into a
// complex normal by Box-Muller and scaled by env[G'].  One thread per
// (pair, u u'); the pair's rows of T, scaled by the envelope, sit in LDS and
// are read as broadcasts.  The draws dominate (a log, a square root and a
// sine/cosine pair per element), so the kernel is bound by the vector ALU.
constexpr uint32_t PH_M0 = 0xD2511F53u, PH_M1 = 0xCD9E8D57u;  // round multipliers
constexpr uint32_t PH_W0 = 0x9E3779B9u, PH_W1 = 0xBB67AE85u;  // key increments
constexpr int S2D_THREADS = 256;
constexpr int S2D_LDS = 4096;  // R x ng values of one pair held in LDS

BSE_DEV double2 drawn_normal(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                             uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(PH_M0, c0), lo0 = PH_M0 * c0;
    const uint32_t hi1 = __umulhi(PH_M1, c2), lo1 = PH_M1 * c2;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += PH_W0;
    k1 += PH_W1;
  }
  // uniforms from the top 53 bits of (w1:w0) and (w3:w2): u1 in (0, 1], u2 in [0, 1)
  const uint64_t b1 = ((uint64_t)c1 << 32 | c0) >> 11;
  const uint64_t b2 = ((uint64_t)c3 << 32 | c2) >> 11;
  const double u1 = ((double)b1 + 1.0) * 0x1p-53;
  const double u2 = (double)b2 * 0x1p-53;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos((2.0 * M_PI) * u2, &sn, &cs);
  constexpr double SQRT2 = 1.4142135623730951;
  return make_double2((rad * cs) / SQRT2, (rad * sn) / SQRT2);
}

template <int RM>
__global__ __launch_bounds__(S2D_THREADS) void k_stage2_drawn(
    const double2* __restrict__ T, int R, int ng, int nc, const double* __restrict__ env,
    uint64_t key, const int32_t* __restrict__ perm, double2* __restrict__ blk,
    const int32_t* info) {
  __shared__ double2 ts[S2D_LDS];
  if (failed(info)) return;
  const int pos = blockIdx.x;
  const uint32_t p = (uint32_t)perm[pos];
  const int n2 = nc * nc;
  const double2* __restrict__ Tp = T + (int64_t)pos * R * ng;
  for (int e = threadIdx.x; e < R * ng; e += S2D_THREADS) ts[e] = cscale(Tp[e], env[e % ng]);
  __syncthreads();
  const int cc = blockIdx.y * S2D_THREADS + threadIdx.x;
  if (cc >= n2) return;
  const uint32_t u = (uint32_t)(cc / nc), u2 = (uint32_t)(cc % nc);
  const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
  double2 acc[RM];
#pragma unroll
  for (int r = 0; r < RM; ++r) acc[r] = make_double2(0.0, 0.0);
  for (int g = 0; g < ng; ++g) {
    const double2 z = drawn_normal(p, u, u2, (uint32_t)g, k0, k1);
#pragma unroll
    for (int r = 0; r < RM; ++r)
      if (r < R) acc[r] = cadd(acc[r], cmul(ts[r * ng + g], z));
  }
  double2* __restrict__ out = blk + (int64_t)pos * R * n2;
#pragma unroll
  for (int r = 0; r < RM; ++r)
    if (r < R) out[(int64_t)r * n2 + cc] = acc[r];
}

// ---------------------------------------------------------------- combine
// Scatter the per-pair blocks into the output matrices (column-major, ld).
//   rr block: blk_rr[pos][(v*nv + v')][(c*nc + c')]
//   ra block: blk_ra[pos][(c*nv + v')][(v*nc + c')]
__global__ __launch_bounds__(256) void k_combine(int npairs, int nk, int nv, int nc, int64_t ld,
                                                 const int32_t* __restrict__ inv_rr,
                                                 const double2* __restrict__ blk_rr,
                                                 const int32_t* __restrict__ inv_ra,
                                                 const double2* __restrict__ blk_ra, double c0r,
                                                 double c0a, double c1r, double c1a,
                                                 double2* __restrict__ out0,
                                                 double2* __restrict__ out1, const int32_t* info) {
  if (failed(info)) return;
  const int nvnc = nv * nc, nb = nvnc * nvnc;
  const int64_t total = (int64_t)npairs * nb;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(g / nb), e = (int)(g % nb);
    const int a = e % nvnc, bcol = e / nvnc;
    const int v = a / nc, c = a % nc, v2 = bcol / nc, c2 = bcol % nc;
    // pair p -> (ik, jk): invert p = ik*nk - ik(ik-1)/2 + (jk - ik)
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
    const double2 rr =
        blk_rr[((int64_t)inv_rr[p] * nv * nv + (v * nv + v2)) * (nc * nc) + (c * nc + c2)];
    double2 ra = make_double2(0.0, 0.0);
    if (blk_ra) ra = blk_ra[((int64_t)inv_ra[p] * nc * nv + (c * nv + v2)) * (nv * nc) + (v * nc + c2)];
    const int64_t row = (int64_t)ik * nvnc + a, col = (int64_t)jk * nvnc + bcol;
    double2* d0 = out0 + row + col * ld;
    double2 o = *d0;
    o.x += c0r * rr.x + c0a * ra.x;
    o.y += c0r * rr.y + c0a * ra.y;
    *d0 = o;
    if (out1) out1[row + col * ld] = make_double2(c1r * rr.x + c1a * ra.x, c1r * rr.y + c1a * ra.y);
  }
}

// ---------------------------------------------------------------- finalize
// Hermitian rule: lower = conj(upper), diagonal = E + Re(diagonal).
constexpr int FT = 32;
__global__ __launch_bounds__(256) void k_finalize(double2* __restrict__ M, int64_t n, int64_t ld,
                                                  const double* __restrict__ eps_v,
                                                  const double* __restrict__ eps_c, int nv, int nc,
                                                  double scissor, int32_t* info) {
  __shared__ double2 tile[FT][FT + 1];
  if (failed(info)) return;
  const int bi = blockIdx.x, bj = blockIdx.y;  // tile row / column
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  if (bi > bj) {
    // read upper tile (rows bj*FT.., cols bi*FT..), write its conjugate transpose
    for (int r = ty; r < FT; r += 8) {
      const int64_t row = (int64_t)bj * FT + tx, col = (int64_t)bi * FT + r;
      if (row < n && col < n) tile[r][tx] = M[row + col * ld];
    }
    __syncthreads();
    for (int r = ty; r < FT; r += 8) {
      const int64_t row = (int64_t)bi * FT + tx, col = (int64_t)bj * FT + r;
      if (row < n && col < n) {
        const double2 u = tile[tx][r];
        M[row + col * ld] = make_double2(u.x, -u.y);
      }
    }
  } else {
    for (int r = ty; r < FT; r += 8) {
      const int64_t row = (int64_t)bi * FT + tx, col = (int64_t)bi * FT + r;
      if (row < n && col < n) tile[r][tx] = M[row + col * ld];
    }
    __syncthreads();
    for (int r = ty; r < FT; r += 8) {
      const int64_t row = (int64_t)bi * FT + tx, col = (int64_t)bi * FT + r;
      if (row >= n || col >= n) continue;
      if (row > col) {
        const double2 u = tile[tx][r];  // element (col, row)
        M[row + col * ld] = make_double2(u.x, -u.y);
      } else if (row == col) {
        const int nvnc = nv * nc;
        const int ik = (int)(row / nvnc), a = (int)(row % nvnc);
        const double e = eps_c[(int64_t)ik * nc + a % nc] - eps_v[(int64_t)ik * nv + a / nc] + scissor;
        const double d = e + tile[r][tx].x;
        if (!isfinite(d)) set_info(info, BSE_INFO_NONFINITE);
        M[row + col * ld] = make_double2(d, 0.0);
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- host side
size_t build_workspace_fp64(const bse_desc* d) {
  const int64_t P = (int64_t)d->nk * (d->nk + 1) / 2;
  WsLayout L;
  L.add(P * 4);        // perm_rr
  L.add((kMaxQ + 1) * 4);  // cls_rr
  L.add(P * 4);        // inv_rr
  L.add(P * 4);        // perm_ra
  L.add((kMaxQ + 1) * 4);  // cls_ra
  L.add(P * 4);        // inv_ra
  const int64_t R1 = (int64_t)d->nv * d->nv, N1 = (int64_t)d->nc * d->nc, R2 = (int64_t)d->nc * d->nv;
  const bool full = d->coupling == BSE_FULL;
  L.add(P * R1 * d->ng * 16);                    // T_rr
  L.add(full ? P * R2 * d->ng * 16 : 0);         // T_ra
  L.add(P * R1 * N1 * 16);                       // blk_rr
  L.add(full ? P * R2 * R2 * 16 : 0);            // blk_ra
  // W split for the precision form: the q-mesh and, for the coupling block on
  // a generically shifted k-mesh, the second q-set of -k-k'
  L.add((int64_t)split_w_bytes(full ? 2 * d->nk : d->nk, d->ng));
  return L.total;
}

bse_status build_fp64(const bse_desc* d, const bse_inputs* in, void* out0, void* out1, void* ws,
                      int32_t* info, hipStream_t s) {
  const int nk = d->nk, nv = d->nv, nc = d->nc, ng = d->ng, nq = in->nq;
  const int64_t n = (int64_t)nk * nv * nc, ld = d->ld;
  const int64_t P = (int64_t)nk * (nk + 1) / 2;
  const bool full = d->coupling == BSE_FULL;
  double gx, gc;
  bse_gamma(d->type, &gx, &gc);
  const double kap = d->kappa;
  // drawn M_cc: the pair's rows of T must fit in LDS (checked before any launch)
  if (!in->Mcc && ((int64_t)nv * nv > 16 || (int64_t)nv * nv * ng > S2D_LDS)) return BSE_ERR_ARG;

  WsLayout L(ws);
  int32_t* perm_rr = (int32_t*)L.add(P * 4);
  int32_t* cls_rr = (int32_t*)L.add((kMaxQ + 1) * 4);
  int32_t* inv_rr = (int32_t*)L.add(P * 4);
  int32_t* perm_ra = (int32_t*)L.add(P * 4);
  int32_t* cls_ra = (int32_t*)L.add((kMaxQ + 1) * 4);
  int32_t* inv_ra = (int32_t*)L.add(P * 4);
  const int64_t R1 = (int64_t)nv * nv, N1 = (int64_t)nc * nc, R2 = (int64_t)nc * nv;
  double2* T_rr = (double2*)L.add(P * R1 * ng * 16);
  double2* T_ra = (double2*)L.add(full ? P * R2 * ng * 16 : 0);
  double2* blk_rr = (double2*)L.add(P * R1 * N1 * 16);
  double2* blk_ra = (double2*)L.add(full ? P * R2 * R2 * 16 : 0);
  void* Wsp = L.add((int64_t)split_w_bytes(full ? 2 * nk : nk, ng));
  (void)cls_ra;

  // class sorts
  BSE_LAUNCH(k_class_sort, dim3(full ? 2 : 1), dim3(1024), 2 * nq * sizeof(int32_t), s,
             in->qmap, full ? in->qramap : nullptr, nk, nq, perm_rr, cls_rr, inv_rr, perm_ra,
             cls_ra, inv_ra, info);

  const int prec = d->prec;
  const int nterms = d->split_terms == 0 ? 6 : d->split_terms;
  // default 9: one pass per term with both products on the matrix cores
  // (measured at N = 6144: 6.8 ms for both terms, against 5.3 + 2.4 + 0.3 ms
  // for the unpadded first product writing T, the batched second product and
  // the scatter (7), 5.8 + 2.4 + 0.3 ms with N_G padded to 128 (4), and 10.8 ms
  // fused with a vector-ALU second product waiting on memory (1)); shapes the
  // one pass does not take run as 7, and those (N_G > 113, FP32) as 4
  int dvar = tune_choice(BSE_TUNE_DIRECT, n, 9);
  const bool shape_ok = (prec == BSE_PREC_FP64 || prec == BSE_PREC_FP32) && in->Mcc &&
                        ng <= 128 && R1 <= 64 && (!full || R2 <= 64);
  if (dvar == 9 && !((prec == BSE_PREC_FP64 || prec == BSE_PREC_FP32) &&
                     first_product_fits(ng, (int)R1) && R1 >= 9 && R1 <= 16 && N1 <= 16 &&
                     (!full || (R2 >= 9 && R2 <= 16))))
    dvar = 7;
  const bool use_fused = shape_ok && ((dvar >= 1 && dvar <= 3) || dvar == 9);
  const bool use_g3_t = shape_ok && dvar >= 4 && dvar <= 8;  // Gauss first product, then two passes
  // the precision form splits W once per build (the two-pass products read
  // it); its buffer holds nk slices
  if (prec != BSE_PREC_FP64 && !use_fused && !use_g3_t) {
    if (nq > (full ? 2 * nk : nk)) return BSE_ERR_ARG;
    if (!launch_split_w(prec, (const double2*)in->W, nq, ng, Wsp, s)) return BSE_ERR_HIP;
  }
  // exchange: out0 (upper) = alpha * conj(Mcv) diag(vbar) Mcv^T
  const double ex_alpha = (full ? 4.0 : 2.0) * gx * kap;
  if (prec != BSE_PREC_FP64) {
    if (!launch_exchange_lp(prec, nterms, (const double2*)in->Mcv, (int)n, ng, in->vbar, ex_alpha,
                            (double2*)out0, ld, info, s))
      return BSE_ERR_HIP;
  } else {
    ZgemmParams g;
    g.M = (int)n;
    g.N = (int)n;
    g.K = ng;
    g.A = (const double2*)in->Mcv;
    g.a_rs = ng;
    g.a_cs = 1;
    g.conjA = 1;
    g.kscale = in->vbar;
    g.B = (const double2*)in->Mcv;
    g.b_rs = 1;
    g.b_cs = ng;
    g.C = (double2*)out0;
    g.c_rs = 1;
    g.c_cs = ld;
    g.alpha = make_double2(ex_alpha, 0.0);
    g.beta = 0.0;
    g.c_uplo = 1;
    g.info = info;
    g.tag = "zgemm_exchange";
    g.tile = tune_choice(BSE_TUNE_GEMM_EXCHANGE, n, 0);
    if (zgemm(g, 1, s) != hipSuccess) return BSE_ERR_HIP;
  }

  // direct terms, stage 1 (grouped by class) and stage 2 (batched by pair)
  auto direct = [&](const void* left, int R, const void* right, int N2, const int32_t* perm,
                    const int32_t* cls, double2* T, double2* blk) -> bool {
    if (use_g3_t && dvar >= 7 && prec == BSE_PREC_FP64 && first_product_fits(ng, R)) {
      if (!launch_first_product(dvar - 7, (const double2*)left, R, ng, nk, (const double2*)in->W,
                                perm, cls, nq, T, info, s))
        return false;
    } else if (use_g3_t) {
      if (!launch_direct_fused(prec, dvar >= 7 ? 1 : dvar - 3, (const double2*)left,
                               (const double2*)right, R, N2, ng, nk, nv, nc,
                               (const double2*)in->W, perm, cls, nq, 0, 0.0, nullptr, nullptr, 0,
                               T, info, s))
        return false;
    } else if (prec != BSE_PREC_FP64) {
      // stage 1 in the precision form; stage 2 (R x ng x N2 per pair, memory-bound)
      // runs in FP64 below
      if (!launch_stage1_lp(prec, nterms, (const double2*)left, R, ng, Wsp, perm, cls, nq, nk, T,
                            info, s))
        return false;
    } else if (!launch_stage1((const double2*)left, R, ng, (const double2*)in->W, perm, cls, nq,
                              nk, T, info, s)) {
      const int tiles = cdiv((int64_t)nk * R, S1_BM);  // a class holds at most nk pairs
      dim3 grid((unsigned)(nq * tiles), (unsigned)cdiv(ng, S1_BN));
      BSE_LAUNCH(k_stage1, grid, dim3(256), 0, s, (const double2*)left, R, ng,
                 (const double2*)in->W, perm, cls, tiles, T, info);
    }
    if (!right) {  // M_cc drawn in place (resonant term only)
      const dim3 grid((unsigned)P, (unsigned)cdiv(N2, S2D_THREADS));
      if (R <= 4)
        BSE_LAUNCH(k_stage2_drawn<4>, grid, dim3(S2D_THREADS), 0, s, T, R, ng, nc, in->mcc_env,
                   in->mcc_key, perm, blk, info);
      else
        BSE_LAUNCH(k_stage2_drawn<16>, grid, dim3(S2D_THREADS), 0, s, T, R, ng, nc, in->mcc_env,
                   in->mcc_key, perm, blk, info);
      return hipGetLastError() == hipSuccess;
    }
    ZgemmParams g;
    g.M = R;
    g.N = N2;
    g.K = ng;
    g.A = T;
    g.a_rs = ng;
    g.a_cs = 1;
    g.a_bs = (int64_t)R * ng;
    g.B = (const double2*)right;
    g.b_rs = 1;
    g.b_cs = ng;
    g.b_bs = (int64_t)N2 * ng;
    g.b_batch_idx = perm;
    g.C = blk;
    g.c_rs = N2;
    g.c_cs = 1;
    g.c_bs = (int64_t)R * N2;
    g.info = info;
    g.tag = "zgemm_direct_stage2";
    g.tile = tune_choice(BSE_TUNE_GEMM_STAGE2, n, 0);
    return zgemm(g, (int)P, s) == hipSuccess;
  };
  const double c = -gc * kap;
  // FP64 and FP32 with stored pair elements: one fused pass per term (T stays
  // on chip), each adding its blocks into the outputs (A+B += c rr,
  // A-B = c rr; then A+B += c ra, A-B -= c ra), unless the tuning table asks
  // for two passes
  if (use_fused) {
    // one pass per term: on the matrix cores for both products (9, FP64, when
    // the shape allows), else the vector-ALU second product (1-3)
    // (the tile lists of the one pass go where T would be: no T is written)
    auto term = [&](const void* left, const void* right, int R, int N2, const int32_t* perm,
                    const int32_t* cls, int ra, double2* o1, void* tmap) -> bool {
      if (dvar == 9)
        return launch_direct_onepass(prec, (const double2*)left, (const double2*)right, R, N2, ng, nk,
                                     nv, nc, (const double2*)in->W, perm, cls, nq, ra, c,
                                     (double2*)out0, o1, ld, (int32_t*)tmap, info, s);
      return launch_direct_fused(prec, dvar, (const double2*)left,
                                 (const double2*)right, R, N2, ng, nk, nv, nc,
                                 (const double2*)in->W, perm, cls, nq, ra, c, (double2*)out0, o1,
                                 ld, nullptr, info, s);
    };
    bool ok = term(in->Mvv, in->Mcc, (int)R1, (int)N1, perm_rr, cls_rr, 0,
                   full ? (double2*)out1 : nullptr, T_rr);
    if (ok && full)
      ok = term(in->Ncv, in->Nvc, (int)R2, (int)R2, perm_ra, cls_ra, 1, (double2*)out1, T_ra);
    if (!ok) return BSE_ERR_HIP;
    const int nt = cdiv(n, FT);
    BSE_LAUNCH(k_finalize, dim3(nt, nt), dim3(256), 0, s, (double2*)out0, n, ld, in->eps_v,
               in->eps_c, nv, nc, d->scissor, info);
    if (full)
      BSE_LAUNCH(k_finalize, dim3(nt, nt), dim3(256), 0, s, (double2*)out1, n, ld, in->eps_v,
                 in->eps_c, nv, nc, d->scissor, info);
    return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
  }
  if (!direct(in->Mvv, (int)R1, in->Mcc, (int)N1, perm_rr, cls_rr, T_rr, blk_rr)) return BSE_ERR_HIP;
  if (full && !direct(in->Ncv, (int)R2, in->Nvc, (int)R2, perm_ra, cls_ra, T_ra, blk_ra))
    return BSE_ERR_HIP;

  // scatter: A+B += -gc kappa (rr + ra), A-B = -gc kappa (rr - ra); TDA: A += -gc kappa rr
  {
    const int64_t total = P * (int64_t)(nv * nc) * (nv * nc);
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
    BSE_LAUNCH(k_combine, dim3(blocks), dim3(256), 0, s, (int)P, nk, nv, nc, ld, inv_rr,
                       blk_rr, full ? inv_ra : nullptr, full ? blk_ra : nullptr, c, c, c, -c,
                       (double2*)out0, full ? (double2*)out1 : nullptr, info);
  }
  // Hermitian rule + transition energies on the diagonal
  {
    const int nt = cdiv(n, FT);
    BSE_LAUNCH(k_finalize, dim3(nt, nt), dim3(256), 0, s, (double2*)out0, n, ld, in->eps_v,
                       in->eps_c, nv, nc, d->scissor, info);
    if (full)
      BSE_LAUNCH(k_finalize, dim3(nt, nt), dim3(256), 0, s, (double2*)out1, n, ld,
                         in->eps_v, in->eps_c, nv, nc, d->scissor, info);
  }
  return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
}
