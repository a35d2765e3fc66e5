// FP64 eigensolver of the BSE (paper Sec. 4.3).
//
// Full problem (squared form): with A-B = U^H U (Cholesky),
//   S = U (A+B) U^H  has the spectrum E^2 of (A-B)^1/2 (A+B) (A-B)^1/2,
//   S Z = E^2 Z,  X+Y = U^H Z E^-1/2.
// TDA: A X = E X.
// The Hermitian matrix (S or A) is reduced to a real symmetric tridiagonal
// T = Q^H S Q by Householder reflectors (blocked, lower), T is solved by
// multisection on Sturm counts and twisted factorisations, and the eigenvectors are
// back-transformed with the reflectors in compact-WY form.  When only the
// spectrum is wanted the back-transform is replaced by projecting the probe:
//   t_l = E_l^-1/2 z_l^T (Q^H U p)      (full),   t_l = z_l^T (Q^H p)   (TDA).
#include <math.h>

#include "bse_internal.h"
#include "common.h"
#include "solve_internal.h"
#include "timing.h"
#include "zgemm.h"

namespace {

constexpr int CH_NB = 32;   // Cholesky panel width

BSE_DEV double2 ld_acq(const double2* p) {
  double2 v;
  v.x = __hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v.y = __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

__global__ void k_copy_c(const double2* __restrict__ src, double2* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// dst[:, j] = src[:, j] for the n x n complex matrices (column-major, lds / ldd)
__global__ __launch_bounds__(256) void k_copy_mat(const double2* __restrict__ src, int64_t lds,
                                                  double2* __restrict__ dst, int64_t ldd,
                                                  int64_t n) {
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
      dst[i + j * ldd] = src[i + j * lds];
}

// dst[:, j] = src[:, j] * e[j] (n x n, column-major)
__global__ __launch_bounds__(256) void k_copy_scale_cols(const double2* __restrict__ src,
                                                         int64_t lds, double2* __restrict__ dst,
                                                         int64_t ldd, int64_t n,
                                                         const double* __restrict__ e,
                                                         const int32_t* info) {
  if (failed(info)) return;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    const double f = e[j];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * 256)
      dst[i + j * ldd] = cscale(src[i + j * lds], f);
  }
}

// X := U_b^-1 X for one nb x nb diagonal block U_b (nb <= 32) of an upper
// triangular U with a real diagonal, over the nb rows of X: one thread per
// column of X, backward substitution in registers, U_b in LDS.
__global__ __launch_bounds__(256) void k_trsm_diag(const double2* __restrict__ U, int64_t ld,
                                                   int nb, double2* __restrict__ X, int64_t ldx,
                                                   int64_t ncols, const int32_t* info) {
  __shared__ double2 u[32][33];
  if (failed(info)) return;
  const double2 zero = make_double2(0.0, 0.0);
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int r = e % 32, c = e / 32;
    u[r][c] = (r < nb && c < nb && r <= c) ? U[r + (int64_t)c * ld] : zero;
  }
  __syncthreads();
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= ncols) return;
  double2* xc = X + col * ldx;
  double2 x[32];
#pragma unroll
  for (int r = 0; r < 32; ++r) x[r] = r < nb ? xc[r] : zero;
#pragma unroll
  for (int r = 31; r >= 0; --r) {
    double2 t = x[r];
#pragma unroll
    for (int k = r + 1; k < 32; ++k) t = csub(t, cmul(u[r][k], x[k]));  // u = 0 past nb
    x[r] = r < nb ? cscale(t, 1.0 / u[r][r].x) : zero;
  }
#pragma unroll
  for (int r = 0; r < 32; ++r)
    if (r < nb) xc[r] = x[r];
}

__global__ void k_zero_ints(int32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// y = U p for the upper triangle U (column-major, ld) in two passes: block
// (row tile I, column chunk J) writes part[J][rows of I] = sum over the chunk's
// columns j >= i of U[i][j] p[j] (coalesced down the columns); then k_trmv_sum
// adds the chunks (in order) of every row.
constexpr int TRMV_ROWS = 256, TRMV_COLS = 256;
__global__ __launch_bounds__(TRMV_ROWS) void k_trmv_part(const double2* __restrict__ U,
                                                         int64_t ld, int n,
                                                         const double2* __restrict__ p,
                                                         double2* __restrict__ part,
                                                         const int32_t* info) {
  if (failed(info)) return;
  const int i0 = blockIdx.x * TRMV_ROWS, j0 = blockIdx.y * TRMV_COLS;
  if (j0 + TRMV_COLS <= i0) return;  // the chunk lies below the diagonal
  const int i = i0 + threadIdx.x;
  const int ic = min(i, n - 1), jend = min(j0 + TRMV_COLS, n);
  double2 acc = make_double2(0.0, 0.0);
  constexpr int UB = 8;  // columns whose loads go out together
  for (int j = max(j0, i0); j < jend; j += UB) {
    double2 uu[UB], pp[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int jj = min(j + u, jend - 1);
      uu[u] = U[ic + (int64_t)jj * ld];
      pp[u] = p[jj];
    }
#pragma unroll
    for (int u = 0; u < UB; ++u)
      if (j + u < jend && j + u >= i) acc = cadd(acc, cmul(uu[u], pp[u]));
  }
  if (i < n) part[(int64_t)blockIdx.y * n + i] = acc;
}

__global__ __launch_bounds__(256) void k_trmv_sum(const double2* __restrict__ part, int n,
                                                  double2* __restrict__ y, const int32_t* info) {
  if (failed(info)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int nch = cdiv(n, TRMV_COLS);
  double2 acc = make_double2(0.0, 0.0);
  for (int c = (i / TRMV_ROWS) * TRMV_ROWS / TRMV_COLS; c < nch; ++c)
    acc = cadd(acc, part[(int64_t)c * n + i]);
  y[i] = acc;
}
}  // namespace
namespace {

// ------------------------------------------------------------------ Cholesky
// One panel of the blocked Cholesky A - B = U^H U (Sec. 4.3): every block
// factors the jb x jb diagonal block A11 = U11^H U11 (right-looking; each
// thread keeps four fixed elements in registers and only the pivot row goes
// through LDS, one barrier per column), then solves U11^H X = A12 for its own
// PCOLS columns of the panel row by forward substitution (one column per
// thread, in registers; the updates of one step are independent).  Block 0
// stores U11 into u11 (panel j0 / CH_NB holds CH_NB x CH_NB entries), not into
// A: the other blocks may still be reading A11 when block 0 is done.
// k_potrf_store moves every U11 into A once the factorisation is complete.
constexpr int PCOLS = 256;
constexpr int PEL = CH_NB * CH_NB / PCOLS;  // diagonal-block elements per thread
BSE_DEV void potrf_panel_dev(double2* __restrict__ A, int64_t ld, int64_t n, int j0, int jb,
                             double2* __restrict__ u11, int32_t* info, int bx) {
  __shared__ double2 u[CH_NB][CH_NB + 1];  // rows of U11 as they are finished
  __shared__ double dsh[CH_NB];
  if (failed(info)) return;
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)j0 + jb + (int64_t)bx * PCOLS;
  const bool solve = jb == CH_NB && c0 + tid < n;
  // this thread's column of A12 (rows j0 .. j0 + jb - 1)
  double2 x[CH_NB];
#pragma unroll
  for (int r = 0; r < CH_NB; ++r)
    x[r] = solve ? A[(int64_t)(j0 + r) + (c0 + tid) * ld] : make_double2(0.0, 0.0);
  // elements e = tid + PCOLS q of the diagonal block: row e % 32, column e / 32
  double2 ae[PEL];
  int er[PEL], ec[PEL];
#pragma unroll
  for (int q = 0; q < PEL; ++q) {
    const int e = tid + PCOLS * q;
    er[q] = e % CH_NB;
    ec[q] = e / CH_NB;
    const bool in = er[q] < jb && ec[q] < jb && er[q] <= ec[q];
    ae[q] = in ? A[(int64_t)(j0 + er[q]) + (int64_t)(j0 + ec[q]) * ld] : make_double2(0.0, 0.0);
  }
  for (int j = 0; j < jb; ++j) {
    // the owners of row j publish it (column >= j), then every thread updates
#pragma unroll
    for (int q = 0; q < PEL; ++q)
      if (er[q] == j && ec[q] >= j && ec[q] < jb) u[j][ec[q]] = ae[q];
    __syncthreads();
    const double d = u[j][j].x;  // the same value in every thread: uniform exit
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0 && bx == 0) set_info(info, j0 + j + 1);
      return;
    }
    const double rd = 1.0 / d;
#pragma unroll
    for (int q = 0; q < PEL; ++q)
      if (er[q] > j && ec[q] >= er[q] && ec[q] < jb)
        ae[q] = csub(ae[q], cscale(cmulc(u[j][er[q]], u[j][ec[q]]), rd));
    if (tid == 0) dsh[j] = sqrt(d);
  }
  __syncthreads();
  // u holds the unscaled rows: U[j][c] = u[j][c] / sqrt(u[j][j])
  for (int e = tid; e < CH_NB * CH_NB; e += PCOLS) {
    const int r = e % CH_NB, c = e / CH_NB;
    if (r < jb && c < jb && r <= c)
      u[r][c] = (r == c) ? make_double2(dsh[r], 0.0) : cscale(u[r][c], 1.0 / dsh[r]);
  }
  __syncthreads();
  if (bx == 0) {
    double2* dst = u11 + (int64_t)(j0 / CH_NB) * CH_NB * CH_NB;
    for (int e = tid; e < jb * jb; e += PCOLS) {
      const int r = e % jb, c = e / jb;
      if (r <= c) dst[r + c * CH_NB] = u[r][c];
    }
  }
  if (jb != CH_NB) return;  // the last panel has no panel row
  // U11^H X = A12, right-looking: x[k] /= U[k][k]; x[r] -= conj(U[k][r]) x[k], r > k
#pragma unroll
  for (int k = 0; k < CH_NB; ++k) {
    x[k] = cscale(x[k], 1.0 / u[k][k].x);
#pragma unroll
    for (int r = k + 1; r < CH_NB; ++r) x[r] = csub(x[r], cmulc(u[k][r], x[k]));
  }
  if (solve)
#pragma unroll
    for (int r = 0; r < CH_NB; ++r) A[(int64_t)(j0 + r) + (c0 + tid) * ld] = x[r];
}

__global__ __launch_bounds__(PCOLS) void k_potrf_panel(double2* __restrict__ A, int64_t ld,
                                                       int64_t n, int j0, int jb,
                                                       double2* __restrict__ u11,
                                                       int32_t* info) {
  potrf_panel_dev(A, ld, n, j0, jb, u11, info, (int)blockIdx.x);
}

// The panel at column j0 of every problem of a group whose order exceeds j0
// (blockIdx.y = problem; the problems travel by value, so that every load is a
// global load).
struct PotrfGroup {
  CholItem it[CHOL_GROUP_MAX];
};
__global__ __launch_bounds__(PCOLS) void k_potrf_panel_b(PotrfGroup g, int j0) {
  const CholItem& q = g.it[blockIdx.y];
  if (j0 >= q.n) return;
  const int jb = (int)min<int64_t>(CH_NB, q.n - j0);
  const int64_t rest = q.n - j0 - jb;
  if ((int64_t)blockIdx.x >= (rest > 0 ? (rest + PCOLS - 1) / PCOLS : 1)) return;
  potrf_panel_dev(q.A, q.ld, q.n, j0, jb, q.u11, q.info, (int)blockIdx.x);
}

// U11 of every panel (staged by k_potrf_panel) into the upper triangle of A.
__global__ __launch_bounds__(256) void k_potrf_store(double2* __restrict__ A, int64_t ld,
                                                     int64_t n,
                                                     const double2* __restrict__ u11,
                                                     const int32_t* info) {
  if (failed(info)) return;
  const int64_t j0 = (int64_t)blockIdx.x * CH_NB;
  const int jb = (int)std::min<int64_t>(CH_NB, n - j0);
  const double2* src = u11 + (int64_t)blockIdx.x * CH_NB * CH_NB;
  for (int e = threadIdx.x; e < jb * jb; e += 256) {
    const int r = e % jb, c = e / jb;
    if (r <= c) A[(j0 + r) + (j0 + c) * ld] = src[r + c * CH_NB];
  }
}

// Mirror one triangle onto the other: from_lower ? upper = conj(lower) :
// lower = conj(upper); the diagonal is made real.
__global__ __launch_bounds__(256) void k_hermitize(double2* __restrict__ M, int64_t n, int64_t ld,
                                                   int from_lower, const int32_t* info) {
  __shared__ double2 tile[32][33];
  if (failed(info)) return;
  const int bi = blockIdx.x, bj = blockIdx.y;  // destination tile (row, column)
  const bool dst_upper = from_lower;
  if (dst_upper ? (bi > bj) : (bi < bj)) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // source tile is the transpose position
  for (int r = ty; r < 32; r += 8) {
    const int64_t row = (int64_t)bj * 32 + tx, col = (int64_t)bi * 32 + r;
    if (row < n && col < n) tile[r][tx] = M[row + col * ld];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t row = (int64_t)bi * 32 + tx, col = (int64_t)bj * 32 + r;
    if (row >= n || col >= n) continue;
    const bool write = dst_upper ? (row < col) : (row > col);
    if (write) {
      const double2 u = tile[tx][r];
      M[row + col * ld] = make_double2(u.x, -u.y);
    } else if (row == col) {
      M[row + col * ld] = make_double2(M[row + col * ld].x, 0.0);
    }
  }
}

// ------------------------------------------------------------------ tridiagonal eigensolver
// T (diagonal d, off-diagonal e) is solved through the copy (T - c I) sigma:
// shifted by the centre c of its Gershgorin interval, so that the rounding of
// every later step is relative to the spread of the spectrum, not to its
// distance from zero (core-level spectra sit far from zero), and scaled by a
// power of two sigma that brings its Gershgorin norm into [1/2, 1).  The
// leading and trailing principal minors of the copy minus x I then grow by at
// most a factor 3 per row and are carried as plain numbers, renormalised by a
// power of two every MR rows (exact, ratios unchanged): no division sits on
// their recurrence.  Eigenvalues are kept as lambda - c (unscaled) until the
// output, so that the eigenvector kernels see them without the rounding of c.
//
// stat: [0] gl, [1] gu  Gershgorin bounds of the shifted, scaled T, widened by
//                       the rounding of the counts
//       [2] pivmin      the underflow threshold (bisection tolerance)
//       [3] tnorm       Gershgorin norm of T - c I (unscaled; at least eps
//                       times that of T)
//       [4] sigma       the scale
//       [5] c           the shift
constexpr int MR = 8;                  // rows between renormalisations of the minors
constexpr double E2_FLOOR = 0x1p-600;  // floor of e^2 in the minor recurrences
constexpr int BS_G = 16384;            // points of the shared Sturm-count grid
constexpr int BS_L = 8;                // probe points per eigenvalue and round
constexpr int EV_NLDS = 6400;          // largest order whose shared rows (3 doubles) fit in LDS
constexpr int EV_JUNK = 64;            // spare columns of the pivot arrays
constexpr int STAT_N = 8;              // doubles of stat

__global__ __launch_bounds__(1024) void k_tri_prep(const double* __restrict__ d,
                                                   const double* __restrict__ e, int n,
                                                   double* __restrict__ ds, double* __restrict__ es,
                                                   double* __restrict__ e2s, double* stat,
                                                   const int32_t* info) {
  __shared__ double slo[16], shi[16];
  if (failed(info)) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  // Gershgorin interval of T - shift I, every thread gets it
  auto gersh = [&](double shift, double& glo, double& ghi) {
    double lo = INFINITY, hi = -INFINITY;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      const double em = (k > 0) ? fabs(e[k - 1]) : 0.0, ep = (k < n - 1) ? fabs(e[k]) : 0.0;
      const double dk = d[k] - shift;
      lo = fmin(lo, dk - em - ep);
      hi = fmax(hi, dk + em + ep);
    }
    for (int off = 32; off >= 1; off >>= 1) {
      lo = fmin(lo, __shfl_xor(lo, off, 64));
      hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    __syncthreads();  // earlier readers of slo, shi are done
    if (lane == 0) {
      slo[w] = lo;
      shi[w] = hi;
    }
    __syncthreads();
    glo = slo[0];
    ghi = shi[0];
    for (int i = 1; i < nw; ++i) {
      glo = fmin(glo, slo[i]);
      ghi = fmax(ghi, shi[i]);
    }
  };
  double lo0, hi0;
  gersh(0.0, lo0, hi0);
  const double c = (lo0 > -INFINITY && hi0 < INFINITY) ? 0.5 * (lo0 + hi0) : 0.0;
  double lo, hi;
  gersh(c, lo, hi);
  const double eps = 2.220446049250313e-16;
  const double tnorm = fmax(fmax(fabs(lo), fabs(hi)), eps * fmax(fabs(lo0), fabs(hi0)));
  const double sigma =
      (tnorm > 0.0 && tnorm < INFINITY) ? ldexp(1.0, -__builtin_amdgcn_frexp_exp(tnorm)) : 1.0;
  if (threadIdx.x == 0) {
    const double pivmin = 2.2250738585072014e-308;  // e^2 <= 1 after scaling
    const double tn = tnorm * sigma;
    stat[0] = lo * sigma - 2.0 * eps * tn * n - 2.0 * pivmin;
    stat[1] = hi * sigma + 2.0 * eps * tn * n + 2.0 * pivmin;
    stat[2] = pivmin;
    stat[3] = tnorm;
    stat[4] = sigma;
    stat[5] = c;
  }
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    ds[k] = (d[k] - c) * sigma;
    const double v = (k < n - 1) ? e[k] * sigma : 0.0;  // es, e2s carry a zero at n-1
    es[k] = v;
    e2s[k] = (k < n - 1) ? fmax(v * v, E2_FLOOR) : 0.0;
  }
}

// 1/q to full double precision: hardware reciprocal refined by two Newton steps.
BSE_DEV double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(fma(-q, r, 1.0), r, r);
  r = fma(fma(-q, r, 1.0), r, r);
  return r;
}

BSE_DEV uint32_t hi_word(double v) { return (uint32_t)((uint64_t)__double_as_longlong(v) >> 32); }

// Brings the larger of two consecutive minors to [1/2, 1) by a power of two.
BSE_DEV void renorm(double& a, double& b) {
  const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(a), fabs(b)));
  a = __builtin_amdgcn_ldexp(a, -ex);
  b = __builtin_amdgcn_ldexp(b, -ex);
}

// Number of eigenvalues of the scaled T below x: the sign changes along the
// leading principal minors p_{-1} = 1, p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2}
// of T - x I, i.e. the negative pivots of its LDL^T factorisation (Sturm).  Each
// computed ratio p_i / p_{i-1} is the pivot recurrence of T with relative
// perturbations of a few ulps in d_i - x and e_{i-1}^2.  Sign bits are packed
// 32 rows to a word (newest in bit 0) and the changes counted per word.
BSE_DEV int count_below(const double* __restrict__ ds, const double* __restrict__ e2s, int n,
                        double x) {
  double p2 = 1.0, p1 = ds[0] - x;
  uint32_t prev = hi_word(p1) >> 31;
  int cnt = (int)prev;
  int i = 1;
  for (; i + 32 <= n; i += 32) {
    uint32_t w = 0;
#pragma unroll
    for (int u = 0; u < 32; ++u) {
      const double pn = fma(ds[i + u] - x, p1, -(e2s[i + u - 1] * p2));
      p2 = p1;
      p1 = pn;
      w = __builtin_amdgcn_alignbit(w, hi_word(pn), 31);
      if (u % MR == MR - 1) renorm(p1, p2);
    }
    cnt += __popc(w ^ ((w >> 1) | (prev << 31)));
    prev = w & 1u;
  }
  for (int u = 0; i < n; ++i, ++u) {
    const double pn = fma(ds[i] - x, p1, -(e2s[i - 1] * p2));
    p2 = p1;
    p1 = pn;
    const uint32_t sg = hi_word(pn) >> 31;
    cnt += (int)(sg ^ prev);
    prev = sg;
    if (u % MR == MR - 1) renorm(p1, p2);
  }
  return cnt;
}

// Point g of the shared grid; g = -1 and g = BS_G are the ends gl and gu.
BSE_DEV double grid_x(double gl, double gu, int g) {
  if (g < 0) return gl;
  if (g >= BS_G) return gu;
  return gl + (gu - gl) * ((double)(g + 1) / (double)(BS_G + 1));
}

// Sturm counts on BS_G interior points of the Gershgorin interval, one per lane.
__global__ __launch_bounds__(64) void k_sturm_grid(const double* __restrict__ ds,
                                                   const double* __restrict__ e2s, int n,
                                                   const double* __restrict__ stat,
                                                   int32_t* __restrict__ counts,
                                                   const int32_t* info) {
  if (failed(info)) return;
  const int g = blockIdx.x * 64 + threadIdx.x;
  if (g >= BS_G) return;
  counts[g] = count_below(ds, e2s, n, grid_x(stat[0], stat[1], g));
}

BSE_DEV double probe_x(double lo, double width, int q) {
  return lo + width * ((double)q / (double)(BS_L + 1));
}

// Eigenvalue k (ascending) by multisection.  Its starting bracket is the grid
// cell where the shared counts pass k; then BS_L lanes probe BS_L interior
// points per round (eight eigenvalues per wavefront) and the bracket shrinks to
// the sub-interval where the count passes k, until it is below
// max(2 eps |lambda|, eps tnorm).  Results are unscaled.
__global__ __launch_bounds__(256) void k_bisect(const double* __restrict__ ds,
                                                const double* __restrict__ e2s, int n,
                                                const double* __restrict__ stat,
                                                const int32_t* __restrict__ counts,
                                                double* __restrict__ w, const int32_t* info) {
  if (failed(info)) return;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wv * (64 / BS_L) >= n) return;  // the whole wavefront is past the end
  const int lane = threadIdx.x & 63, grp = lane / BS_L, s = lane % BS_L;
  const int k = wv * (64 / BS_L) + grp;
  const double gl = stat[0], gu = stat[1], pivmin = stat[2], sigma = stat[4];
  const double tn = stat[3] * sigma;
  const double eps = 2.220446049250313e-16;
  int a = 0, b = BS_G;  // first grid point whose count exceeds k (counts[BS_G] = n)
  while (a < b) {
    const int m = (a + b) >> 1;
    if (counts[m] > k) b = m;
    else a = m + 1;
  }
  double lo = grid_x(gl, gu, a - 1), hi = grid_x(gl, gu, a);
  bool done = k >= n;
  for (int it = 0; it < 96; ++it) {
    const double width = hi - lo;
    const double tol = fmax(2.0 * eps * fmax(fabs(lo), fabs(hi)), eps * tn) + 4.0 * pivmin;
    done = done || !(width > tol);
    if (__ballot(!done) == 0ull) break;
    const int c = count_below(ds, e2s, n, probe_x(lo, width, s + 1));
    const uint32_t gb = (uint32_t)(__ballot(c > k) >> (BS_L * grp)) & ((1u << BS_L) - 1u);
    if (!done) {
      double nlo = lo, nhi = hi;
      if (gb == 0u) {
        nlo = probe_x(lo, width, BS_L);
      } else {
        const int f = __ffs(gb) - 1;
        nhi = probe_x(lo, width, f + 1);
        if (f > 0) nlo = probe_x(lo, width, f);
      }
      if (nlo == lo && nhi == hi) done = true;
      lo = nlo;
      hi = nhi;
    }
  }
  if (k < n && s == 0) w[k] = 0.5 * (lo + hi) / sigma;
}

// Independent brackets can leave two nearly equal eigenvalues out of order by
// an ulp: a running maximum restores the ascending order.
__global__ __launch_bounds__(1024) void k_monotone(double* __restrict__ w, int n,
                                                   const int32_t* info) {
  __shared__ double sm[1024];
  if (failed(info)) return;
  const int t = threadIdx.x, per = cdiv(n, 1024);
  const int a = min(n, t * per), b = min(n, a + per);
  double m = -INFINITY;
  for (int i = a; i < b; ++i) m = fmax(m, w[i]);
  sm[t] = m;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const double v = (t >= off) ? sm[t - off] : -INFINITY;
    __syncthreads();
    sm[t] = fmax(sm[t], v);
    __syncthreads();
  }
  double run = (t > 0) ? sm[t - 1] : -INFINITY;
  for (int i = a; i < b; ++i) {
    run = fmax(run, w[i]);
    if (w[i] != run) w[i] = run;
  }
}

BSE_DEV double hash_uniform(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return 2.0 * ((double)h / 4294967296.0) - 1.0;
}

// A zero the compiler cannot see through: added to a pointer it makes the
// accesses per-lane (vector) loads, so that rows that are the same for every
// lane are prefetched into registers like the per-lane ones.
BSE_DEV int lane_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}

// Runs body(t, u, v) for t = 0 .. count-1 with v (a small struct of doubles)
// filled by fetch(t, v) one block of TB steps ahead (two buffers; u = t mod TB,
// a compile-time index after unrolling; a fetch past the end repeats the last
// step).  Whole blocks run without bounds tests, the last one or two with them.
template <int TB, typename V, typename Fetch, typename Body>
BSE_DEV void stream(int count, Fetch&& fetch, Body&& body) {
  if (count <= 0) return;
  V b0[TB], b1[TB];
  auto fill = [&](V(&buf)[TB], int blk) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < TB; ++u) fetch(min(blk * TB + u, count - 1), buf[u]);
  };
  auto run = [&](V(&buf)[TB], int blk, bool guarded) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int t = blk * TB + u;
      if (guarded && t >= count) break;
      body(t, u, buf[u]);
    }
  };
  const int nfull = count / TB, nblk = cdiv(count, TB);
  fill(b0, 0);
  int blk = 0;
  for (; blk + 2 <= nfull; blk += 2) {
    fill(b1, blk + 1);
    run(b0, blk, false);
    fill(b0, blk + 2);
    run(b1, blk + 1, false);
  }
  if (blk < nblk) {
    fill(b1, blk + 1);
    run(b0, blk, true);
    if (blk + 1 < nblk) run(b1, blk + 1, true);
  }
}

// Runs blockf(t0, buf, nvalid) over blocks of TB steps: the steps t0 .. t0+TB-1,
// of which the first nvalid exist (the rest repeat the last one).  buf holds
// the lanes' own values of those steps, filled by fetch(t, v) NB-1 blocks
// ahead in a ring of NB buffers (indices fixed at compile time), so that
// several blocks of loads are in flight while one is used.  The block
// function can run its recurrence first and the independent per-step work
// afterwards, without branches.
template <int TB, int NB, typename V, typename Fetch, typename Block>
BSE_DEV void stream_blocks(int count, Fetch&& fetch, Block&& blockf) {
  if (count <= 0) return;
  V buf[NB][TB];
  auto fill = [&](V(&b)[TB], int blk) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < TB; ++u) fetch(min(blk * TB + u, count - 1), b[u]);
  };
  const int nblk = cdiv(count, TB);
#pragma unroll
  for (int i = 0; i < NB - 1; ++i) fill(buf[i], i);
  for (int blk = 0; blk < nblk; blk += NB) {
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      if (blk + s >= nblk) break;
      fill(buf[(s + NB - 1) % NB], blk + s + NB - 1);
      blockf((blk + s) * TB, buf[s], min(TB, count - (blk + s) * TB));
    }
  }
}

struct EvV2 {
  double a, b;
};
constexpr int EV_TB = 8;   // steps per block of the vector sweeps
constexpr int EV_NB = 6;   // blocks of the lanes' own rows in flight (one value per step)
constexpr int EV_NB2 = 4;  // the same with two values per step

// Eigenvectors of T, one lane per eigenvalue; Z, Dp and Dm are [row i][eigenvalue j].
//
// Isolated eigenvalues (blocks 0 .. nb-1): the twisted factorisation of
// T - lambda I.  The top-down pivots D+_i = p_i / p_{i-1} (leading minors) and
// the bottom-up pivots D-_i = q_i / q_{i+1} (trailing minors) give
// gamma_i = D+_i + D-_i - (d_i - lambda); with r = argmin |gamma_i| the vector
// z_r = 1, z_i = -(e_i / D+_i) z_{i+1} (i < r), z_{i+1} = -(e_i / D-_{i+1}) z_i
// (i >= r) solves (T - lambda I) z = gamma_r e_r, i.e. one step of inverse
// iteration from the unit vector that the factorisation marks as largest.  Z
// keeps z unnormalised; zs[j] = +-1 / |z| makes it unit length with its
// largest component positive.
//
// Eigenvalues of a cluster (neighbours closer than ortol_rel ||T - c I||, an
// absolute gap: the angle between a computed vector and the true one is about
// eps ||T - c I|| / gap; blocks nb .. 2nb-1): two
// solves of (T - lambda I) x = b through the top-down LDL^T factorisation
// (pivots kept at least eps tnorm in magnitude) from a pseudo-random start,
// the second from the normalised first; k_cluster_orth then orthonormalises
// the cluster.
//
// With yproj (the probe carried through the reduction), isolated lanes also
// form t_j = z^T yproj on the fly, and store_z = 0 skips their Z stores (only
// t is needed for the spectrum); cluster members always store Z.
__global__ __launch_bounds__(64) void k_eigvec(const double* __restrict__ ds,
                                               const double* __restrict__ es, int n,
                                               const double* __restrict__ w,
                                               const double* __restrict__ stat, double ortol_rel,
                                               double* __restrict__ Z, double* __restrict__ Dp,
                                               double* __restrict__ Dm, double* __restrict__ zs,
                                               const double2* __restrict__ yproj, int store_z,
                                               double2* __restrict__ tproj, int32_t* info) {
  __shared__ double ush[3][EV_NLDS];
  if (failed(info)) return;
  const int nb = cdiv(n, 64);
  const bool cl_role = (int)blockIdx.x >= nb;
  const int j = ((int)blockIdx.x - (cl_role ? nb : 0)) * 64 + (int)threadIdx.x;
  const bool valid = j < n;
  auto close = [&](int a) {  // eigenvalues a and a+1
    return w[a + 1] - w[a] <= ortol_rel * stat[3];
  };
  const bool member = valid && ((j > 0 && close(j - 1)) || (j + 1 < n && close(j)));
  const bool act = valid && (member == cl_role);
  if (__ballot(act) == 0ull) return;
  const int64_t N = n;
  const double sigma = stat[4];
  const double lam = w[valid ? j : n - 1] * sigma;
  // Pivots of the factorisations of T - lambda I: a pivot below eps ||T|| in
  // magnitude is replaced by -eps ||T|| inside the recurrence (the minor
  // becomes -eps ||T|| times the previous one), a perturbation of T of that
  // size.  The recurrences use the exact e^2: the floor that keeps the Sturm
  // counts of a split matrix going would here put a spurious coupling next to
  // an exactly zero pivot.
  const double tiny = 2.220446049250313e-16 * stat[3] * sigma;
  auto guard = [&](double v) { return fabs(v) >= tiny ? v : -tiny; };
  auto minor_next = [&](double a, double e2, double m1, double m2) __attribute__((always_inline)) {
    const double mn = fma(a, m1, -(e2 * m2));
    return fabs(mn) >= tiny * fabs(m1) ? mn : -tiny * m1;
  };

  // Dp and Dm have EV_JUNK spare columns after the n eigenvalues: lanes without
  // work store there, so that the sweeps carry no branches around their stores.
  const int64_t LDD = N + EV_JUNK;
  const int col = act ? j : n + (int)threadIdx.x;
  // Rows shared by the lanes are staged in LDS when they fit (d, e^2 for the
  // pivot sweeps; then e and the probe), so that only the lanes' own pivot rows
  // are prefetched, 16 ahead; otherwise they are read as vector loads.
  const bool use_lds = n <= EV_NLDS;
  auto stage = [&](const double* a0, const double* a1, const double2* y2)
      __attribute__((always_inline)) {
    __syncthreads();  // earlier readers are done (one wavefront per block)
    constexpr int SU = 8;
    for (int i0 = 0; i0 < n; i0 += 64 * SU) {
      double t0[SU], t1[SU], t2[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = min(i0 + 64 * u + (int)threadIdx.x, n - 1);
        t0[u] = a0[i];
        t1[u] = a1 ? a1[i] : (y2 ? y2[i].x : 0.0);
        t2[u] = y2 ? y2[i].y : 0.0;
      }
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int i = i0 + 64 * u + (int)threadIdx.x;
        if (i < n) {
          ush[0][i] = t0[u];
          ush[1][i] = t1[u];
          ush[2][i] = t2[u];
        }
      }
    }
    __syncthreads();
  };
  if (use_lds) stage(ds, es, nullptr);

  // top-down pivots D+ (both roles)
  auto sweep_down = [&](auto dk, auto ek) __attribute__((always_inline)) {
    double p2 = 1.0, p1 = minor_next(dk(0) - lam, 0.0, 1.0, 0.0);
    Dp[col] = guard(p1);
    int i = 1;
    for (; i + MR <= n; i += MR) {
#pragma unroll
      for (int u = 0; u < MR; ++u) {
        const double e = ek(i + u - 1);
        const double pn = minor_next(dk(i + u) - lam, e * e, p1, p2);
        Dp[(int64_t)(i + u) * LDD + col] = guard(pn * recip(p1));
        p2 = p1;
        p1 = pn;
      }
      renorm(p1, p2);
    }
    for (; i < n; ++i) {
      const double e = ek(i - 1);
      const double pn = minor_next(dk(i) - lam, e * e, p1, p2);
      Dp[(int64_t)i * LDD + col] = guard(pn * recip(p1));
      p2 = p1;
      p1 = pn;
    }
  };
  if (use_lds)
    sweep_down([&](int i) { return ush[0][i]; }, [&](int i) { return ush[1][i]; });
  else
    sweep_down([&](int i) { return ds[i]; }, [&](int i) { return es[i]; });

  const int zl = lane_zero();
  const double* dsv = ds + zl;  // rows shared by the lanes, read as vector loads
  const double* esv = es + zl;
  const double* Dpc = Dp + col;
  const double* Dmc = Dm + col;
  const double* Zc = Z + (valid ? j : 0);

  const int ldd = n + EV_JUNK;  // element offsets fit in int for the orders handled here
  const int junk = n + (int)threadIdx.x;  // row 0 of this lane's spare column
  if (!cl_role) {
    // Ud, Ue: d and e of row k; Uyr, Uyi: the probe of row k.
    auto iso = [&](auto Ud, auto Ue2) __attribute__((always_inline)) {
      // bottom-up pivots D- and the twist index (row n-1 first, then n-2 .. 0):
      // per block the minors' recurrence, then the ratios, stores and argmin
      double q2 = 1.0, q1 = minor_next(Ud(n - 1) - lam, 0.0, 1.0, 0.0);
      Dm[(n - 1) * ldd + col] = guard(q1);
      double best = fabs(Dpc[(n - 1) * ldd]);
      int r = n - 1;
      stream_blocks<EV_TB, EV_NB, double>(
          n - 1, [&](int t, double& v) __attribute__((always_inline)) { v = Dpc[(n - 2 - t) * ldd]; },
          [&](int t0, const double(&dp)[EV_TB], int nv) __attribute__((always_inline)) {
            // qs: the minors as computed (numerators of their own ratios);
            // qd: the same after a renormalisation (denominators of the next)
            double qs[EV_TB], qd[EV_TB], as[EV_TB], e2k[EV_TB];
#pragma unroll
            for (int u = 0; u < EV_TB; ++u) {
              const int k = max(n - 2 - (t0 + u), 0);
              as[u] = Ud(k) - lam;
              const double e = Ue2(k);
              e2k[u] = e * e;
            }
            const double qlast = q1;
#pragma unroll
            for (int u = 0; u < EV_TB; ++u) {
              const double qn = minor_next(as[u], e2k[u], q1, q2);
              q2 = q1;
              q1 = qn;
              qs[u] = qn;
              if (u % MR == MR - 1) renorm(q1, q2);
              qd[u] = q1;
            }
#pragma unroll
            for (int u = 0; u < EV_TB; ++u) {
              const double qp = (u == 0) ? qlast : qd[u - 1];
              const double dm = guard(qs[u] * recip(qp));
              const double g = dp[u] + dm - as[u];
              const bool ok = u < nv;
              const int k = n - 2 - (t0 + u);
              Dm[ok ? k * ldd + col : junk] = dm;
              const bool nb = ok && fabs(g) < best;
              best = nb ? fabs(g) : best;
              r = nb ? k : r;
            }
          });
      return r;
    };
    auto vec = [&](int r, auto Ue, auto Uyr, auto Uyi) __attribute__((always_inline)) {
      // z below r (descending), then above r (ascending): per block the ratios
      // first, then the product chain, then the sums
      double nrm = 1.0, big = 1.0;
      bool neg = false;
      double z = 1.0;
      double2 tacc = make_double2(0.0, 0.0);
      const bool st = act && store_z;
      // below: step t is row k = n-2-t (D+_k, e_k); above: row k + 1 from
      // row k = t (D-_{k+1}, e_k); the probe is taken at the row written
      auto half = [&](int t0, const double(&dv)[EV_TB], int nv, bool below)
          __attribute__((always_inline)) {
        double zz[EV_TB], ls[EV_TB], yr[EV_TB], yi[EV_TB];
        bool on[EV_TB];
#pragma unroll
        for (int u = 0; u < EV_TB; ++u) {
          const int k = below ? max(n - 2 - (t0 + u), 0) : min(t0 + u, n - 2);
          const int kw = below ? k : k + 1;
          ls[u] = Ue(k) * recip(dv[u]);
          yr[u] = Uyr(kw);
          yi[u] = Uyi(kw);
        }
#pragma unroll
        for (int u = 0; u < EV_TB; ++u) {
          const int k = below ? n - 2 - (t0 + u) : t0 + u;
          on[u] = (u < nv) && (below ? k < r : k >= r);
          z = on[u] ? -ls[u] * z : z;
          zz[u] = z;
        }
#pragma unroll
        for (int u = 0; u < EV_TB; ++u) {
          const double zon = on[u] ? zz[u] : 0.0;
          nrm = fma(zon, zon, nrm);
          tacc.x = fma(zon, yr[u], tacc.x);
          tacc.y = fma(zon, yi[u], tacc.y);
          const double az = fabs(zon);
          const bool nbig = az > big;
          big = nbig ? az : big;
          neg = nbig ? (zz[u] < 0.0) : neg;
        }
        if (st) {
#pragma unroll
          for (int u = 0; u < EV_TB; ++u) {
            const int kw = below ? n - 2 - (t0 + u) : t0 + u + 1;
            if (on[u]) Z[(int64_t)kw * N + j] = zz[u];
          }
        }
      };
      stream_blocks<EV_TB, EV_NB, double>(
          n - 1, [&](int t, double& v) __attribute__((always_inline)) { v = Dpc[(n - 2 - t) * ldd]; },
          [&](int t0, const double(&dv)[EV_TB], int nv) __attribute__((always_inline)) {
            half(t0, dv, nv, true);
          });
      if (st) Z[(int64_t)r * N + j] = 1.0;
      if (yproj) tacc = cadd(tacc, yproj[r]);
      z = 1.0;
      stream_blocks<EV_TB, EV_NB, double>(
          n - 1, [&](int t, double& v) __attribute__((always_inline)) { v = Dmc[(t + 1) * ldd]; },
          [&](int t0, const double(&dv)[EV_TB], int nv) __attribute__((always_inline)) {
            half(t0, dv, nv, false);
          });
      if (act) {
        zs[j] = (neg ? -1.0 : 1.0) / sqrt(nrm);
        if (yproj) tproj[j] = tacc;
      }
    };
    const double* yv = (const double*)(yproj ? yproj : (const double2*)ds) + zl;  // re at 2k
    const int yld = yproj ? 2 : 0;
    if (use_lds) {
      auto L0 = [&](int k) { return ush[0][k]; };
      auto L1 = [&](int k) { return ush[1][k]; };
      auto L2 = [&](int k) { return ush[2][k]; };
      const int r = iso(L0, L1);
      stage(es, nullptr, yproj);
      vec(r, L0, L1, L2);
    } else {
      const int r = iso([&](int k) { return dsv[k]; }, [&](int k) { return esv[k]; });
      vec(r, [&](int k) { return esv[k]; }, [&](int k) { return yv[k * yld]; },
          [&](int k) { return yv[k * yld + 1]; });
    }
    return;
  }

  // cluster members: inverse iteration through L D+ L^T (e_{n-1} is stored as 0)
  auto piv = [&](double v) { return fabs(v) >= tiny ? v : (v >= 0.0 ? tiny : -tiny); };
  auto inv = [&](auto Ue) __attribute__((always_inline)) {
    double scale = 1.0;
    for (int it = 0; it < 2; ++it) {
      double lprev = 0.0, yprev = 0.0;
      stream_blocks<EV_TB, EV_NB2, EvV2>(
          n,
          [&](int i, EvV2& v) __attribute__((always_inline)) {
            v.a = Dpc[i * ldd];
            v.b = Zc[(int64_t)i * N];
          },
          [&](int t0, const EvV2(&v)[EV_TB], int nv) __attribute__((always_inline)) {
            double ys[EV_TB], ls[EV_TB];
#pragma unroll
            for (int u = 0; u < EV_TB; ++u) ls[u] = Ue(min(t0 + u, n - 1)) * recip(piv(v[u].a));
#pragma unroll
            for (int u = 0; u < EV_TB; ++u) {
              const double b =
                  (it == 0) ? hash_uniform((uint32_t)(t0 + u), (uint32_t)j) : v[u].b * scale;
              ys[u] = fma(-lprev, yprev, b);
              lprev = ls[u];
              yprev = ys[u];
            }
#pragma unroll
            for (int u = 0; u < EV_TB; ++u)
              if (act && u < nv) Z[(int64_t)(t0 + u) * N + j] = ys[u];
          });
      double xprev = 0.0, big = 0.0;
      stream_blocks<EV_TB, EV_NB2, EvV2>(
          n,
          [&](int t, EvV2& v) __attribute__((always_inline)) {
            const int i = n - 1 - t;
            v.a = Dpc[i * ldd];
            v.b = Zc[(int64_t)i * N];
          },
          [&](int t0, const EvV2(&v)[EV_TB], int nv) __attribute__((always_inline)) {
            double xs[EV_TB], rp[EV_TB], el[EV_TB];
#pragma unroll
            for (int u = 0; u < EV_TB; ++u) {
              rp[u] = recip(piv(v[u].a));
              el[u] = Ue(max(n - 1 - (t0 + u), 0));
            }
#pragma unroll
            for (int u = 0; u < EV_TB; ++u) {
              xs[u] = fma(-(el[u] * rp[u]), xprev, v[u].b * rp[u]);
              xprev = xs[u];
            }
#pragma unroll
            for (int u = 0; u < EV_TB; ++u) {
              if (u < nv) big = fmax(big, fabs(xs[u]));
              if (act && u < nv) Z[(int64_t)(n - 1 - (t0 + u)) * N + j] = xs[u];
            }
          });
      if (act && (!(big > 0.0) || !(big < INFINITY))) set_info(info, BSE_INFO_NO_CONVERGE);
      scale = 1.0 / big;
    }
  };
  if (use_lds) {
    stage(es, nullptr, nullptr);
    inv([&](int k) { return ush[0][k]; });
  } else {
    inv([&](int k) { return esv[k]; });
  }
  if (act) zs[j] = 1.0;
}

// Largest |v| with its value (ties: lower index).
struct ArgMax {
  double a, v;
  int i;
};
BSE_DEV ArgMax argmax_merge(ArgMax x, ArgMax y) {
  if (y.a > x.a || (y.a == x.a && y.i < x.i)) return y;
  return x;
}

// Orthonormalises each cluster (one block per cluster, led by its first
// eigenvalue): modified Gram-Schmidt, two passes, over the members in order,
// then unit length with the largest component positive.
__global__ __launch_bounds__(256) void k_cluster_orth(const double* __restrict__ w, int n,
                                                      const double* __restrict__ stat,
                                                      double ortol_rel, double* __restrict__ Z,
                                                      const double2* __restrict__ yproj,
                                                      double2* __restrict__ tproj,
                                                      int32_t* info) {
  __shared__ double sh[4];
  __shared__ double sa[4], sv[4];
  __shared__ int si[4];
  if (failed(info)) return;
  const int k = blockIdx.x;
  auto close = [&](int a) {
    return w[a + 1] - w[a] <= ortol_rel * stat[3];
  };
  if (k + 1 >= n || !close(k) || (k > 0 && close(k - 1))) return;
  int kend = k + 1;
  while (kend + 1 < n && close(kend)) ++kend;
  const int64_t N = n;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int j = k; j <= kend; ++j) {
    for (int pass = 0; pass < 2; ++pass) {
      for (int jp = k; jp < j; ++jp) {
        double dot = 0.0;
        for (int i = tid; i < n; i += 256) dot += Z[(int64_t)i * N + jp] * Z[(int64_t)i * N + j];
        dot = block_sum(dot, sh);
        for (int i = tid; i < n; i += 256) Z[(int64_t)i * N + j] -= dot * Z[(int64_t)i * N + jp];
      }
    }
    double nrm = 0.0;
    ArgMax m{-1.0, 0.0, 0};
    for (int i = tid; i < n; i += 256) {
      const double v = Z[(int64_t)i * N + j];
      nrm += v * v;
      m = argmax_merge(m, ArgMax{fabs(v), v, i});
    }
    nrm = block_sum(nrm, sh);
    for (int off = 32; off >= 1; off >>= 1) {
      ArgMax o{__shfl_xor(m.a, off, 64), __shfl_xor(m.v, off, 64), __shfl_xor(m.i, off, 64)};
      m = argmax_merge(m, o);
    }
    __syncthreads();
    if (lane == 0) {
      sa[wv] = m.a;
      sv[wv] = m.v;
      si[wv] = m.i;
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) m = argmax_merge(m, ArgMax{sa[q], sv[q], si[q]});
    if (!(nrm > 0.0) || !(nrm < INFINITY)) {
      if (tid == 0) set_info(info, BSE_INFO_NO_CONVERGE);
      return;
    }
    const double s = (m.v < 0.0 ? -1.0 : 1.0) / sqrt(nrm);
    double tx = 0.0, ty = 0.0;
    for (int i = tid; i < n; i += 256) {
      const double v = Z[(int64_t)i * N + j] * s;
      Z[(int64_t)i * N + j] = v;
      if (yproj) {
        tx = fma(v, yproj[i].x, tx);
        ty = fma(v, yproj[i].y, ty);
      }
    }
    if (yproj) {
      tx = block_sum(tx, sh);
      ty = block_sum(ty, sh);
      if (tid == 0) tproj[j] = make_double2(tx, ty);
    }
  }
}

// E = sqrt(mu) (full) and the column scale of Z (E^-1/2), or E = mu (TDA); the
// column scale also carries the normalisation zs of the tridiagonal eigenvectors.
// With tproj (z^T of the projected probe, unnormalised), osc = |tproj|^2 scale^2.
__global__ void k_eigvals(const double* __restrict__ mu, const double* __restrict__ stat,
                          const double* __restrict__ zs, int n, int full,
                          double* __restrict__ E, double* __restrict__ colscale,
                          const double2* __restrict__ tproj, double* __restrict__ osc,
                          int32_t* info) {
  if (failed(info)) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double m = mu[k] + stat[5];  // mu holds lambda - c
  if (full) {
    if (!(m > 0.0)) {
      set_info(info, BSE_INFO_NOT_PD_PLUS);
      return;
    }
    const double ek = sqrt(m);
    E[k] = ek;
    colscale[k] = zs[k] / sqrt(ek);
  } else {
    E[k] = m;
    colscale[k] = zs[k];
  }
  if (tproj) osc[k] = cabs2(tproj[k]) * colscale[k] * colscale[k];
}

// Z (complex, column-major, ldz)[i, j] = Ztri[i][j] * scale[j]
__global__ __launch_bounds__(256) void k_ztri_to_complex(const double* __restrict__ Zt, int n,
                                                         const double* __restrict__ scale,
                                                         double2* __restrict__ Z, int64_t ldz,
                                                         const int32_t* info) {
  __shared__ double tile[32][33];
  if (failed(info)) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    tile[r][tx] = (i < n && j < n) ? Zt[i * n + j] * scale[j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t j = j0 + r, i = i0 + tx;
    if (i < n && j < n) Z[i + j * ldz] = make_double2(tile[tx][r], 0.0);
  }
}

// ------------------------------------------------------------------ reflector blocks
// T factor (I - V T V^H = H_j0 ... H_j0+jb-1) of every panel; one block per panel.
// Vcol(r, a) = M[r, j0+a] for r >= j0+a+1 (the unit entry is stored), else 0.
__global__ __launch_bounds__(256) void k_larft(const double2* __restrict__ M, int64_t ld, int n,
                                               const double2* __restrict__ tau,
                                               double2* __restrict__ Tall,
                                               const int32_t* info) {
  __shared__ double2 vs[64][TRD_NB + 1];
  __shared__ double2 G[TRD_NB][TRD_NB + 1];
  __shared__ double2 T[TRD_NB][TRD_NB + 1];
  if (failed(info)) return;
  const int pnl = blockIdx.x;
  const int j0 = pnl * TRD_NB;
  const int jb = min(TRD_NB, n - 1 - j0);
  if (jb <= 0) return;
  const int tid = threadIdx.x;
  double2 acc[4];
  for (int q = 0; q < 4; ++q) acc[q] = make_double2(0.0, 0.0);
  for (int r0 = j0 + 1; r0 < n; r0 += 64) {
    for (int e = tid; e < 64 * TRD_NB; e += 256) {
      const int rr = e % 64, a = e / 64;
      const int r = r0 + rr;
      double2 v = make_double2(0.0, 0.0);
      if (a < jb && r < n && r >= j0 + a + 1) v = M[r + (int64_t)(j0 + a) * ld];
      vs[rr][a] = v;
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int pidx = tid + q * 256;  // (a, b) = (pidx % 32, pidx / 32)
      const int a = pidx % TRD_NB, b = pidx / TRD_NB;
      double2 s = acc[q];
      for (int rr = 0; rr < 64; ++rr) s = cadd(s, cmulc(vs[rr][a], vs[rr][b]));
      acc[q] = s;
    }
    __syncthreads();
  }
  for (int q = 0; q < 4; ++q) {
    const int pidx = tid + q * 256;
    G[pidx % TRD_NB][pidx / TRD_NB] = acc[q];
  }
  for (int e = tid; e < TRD_NB * TRD_NB; e += 256) T[e % TRD_NB][e / TRD_NB] = make_double2(0.0, 0.0);
  __syncthreads();
  // T[:i, i] = -tau_i T[:i, :i] G[:i, i];  T[i, i] = tau_i
  for (int i = 0; i < jb; ++i) {
    const double2 ti = tau[j0 + i];
    if (tid < i) {
      double2 s = make_double2(0.0, 0.0);
      for (int k = tid; k < i; ++k) s = cadd(s, cmul(T[tid][k], G[k][i]));
      T[tid][i] = make_double2(-(ti.x * s.x - ti.y * s.y), -(ti.x * s.y + ti.y * s.x));
    }
    if (tid == 0) T[i][i] = ti;
    __syncthreads();
  }
  double2* To = Tall + (int64_t)pnl * TRD_NB * TRD_NB;
  for (int e = tid; e < TRD_NB * TRD_NB; e += 256) To[e] = T[e % TRD_NB][e / TRD_NB];
}

}  // namespace

// ------------------------------------------------------------------ host side
namespace {
struct SolveWs {
  double2* Wk;    // n x n complex (T1 of the squared form, then Z)
  double* Ztri;   // n x n real, [row][eigenvalue]
  double* Dp;     // n x (n + EV_JUNK) top-down pivots, [row][eigenvalue]
  double* Dm;     // n x (n + EV_JUNK) bottom-up pivots, [row][eigenvalue]
  double2* VW;    // n x 2 TRD_NB panel [V | W]
  double2* WV;    // n x 2 TRD_NB panel [W | V]
  double2* W1;    // TRD_NB x n (back-transform); the Cholesky's U11 blocks before that
  double2* W2;    // TRD_NB x n
  double2* ybuf;  // n
  double2* yvec;  // n (probe projection)
  double2* tproj; // n (eigenvectors of T against the projected probe)
  double2* hs;    // small state
  double2* part;  // partial sums
  double2* Tall;  // T factors
  double2* tau;   // n
  double* dd;
  double* ee;
  double* ds;     // scaled T: diagonal, off-diagonal, squared off-diagonal
  double* es;
  double* e2s;
  double* mu;
  double* zs;     // eigenvector normalisation
  double* colscale;
  double* stat;
  int32_t* grid;  // shared Sturm counts
  int32_t* counters;
  size_t total;
};

SolveWs carve(const bse_desc* d, void* base) {
  const int64_t n = (int64_t)d->nk * d->nv * d->nc;
  const int64_t npnl = (n + TRD_NB - 1) / TRD_NB + 1;
  WsLayout L(base);
  SolveWs w;
  w.Wk = (double2*)L.add(n * n * 16);
  w.Ztri = (double*)L.add(n * n * 8);
  w.Dp = (double*)L.add(n * (n + EV_JUNK) * 8);
  w.Dm = (double*)L.add(n * (n + EV_JUNK) * 8);
  w.VW = (double2*)L.add(n * 2 * TRD_NB * 16);
  w.WV = (double2*)L.add(n * 2 * TRD_NB * 16);
  static_assert(CH_NB <= TRD_NB, "the U11 blocks fit in W1");
  w.W1 = (double2*)L.add((n + CH_NB) * TRD_NB * 16);
  w.W2 = (double2*)L.add(n * TRD_NB * 16);
  w.ybuf = (double2*)L.add(n * 16);
  w.yvec = (double2*)L.add(n * 16);
  w.tproj = (double2*)L.add(n * 16);
  w.hs = (double2*)L.add(HS_SIZE * 16);
  w.part = (double2*)L.add(trd_part_elems(n) * 16);
  w.Tall = (double2*)L.add(npnl * TRD_NB * TRD_NB * 16);
  w.tau = (double2*)L.add(n * 16);
  w.dd = (double*)L.add(n * 8);
  w.ee = (double*)L.add(n * 8);
  w.ds = (double*)L.add(n * 8);
  w.es = (double*)L.add(n * 8);
  w.e2s = (double*)L.add(n * 8);
  w.mu = (double*)L.add(n * 8);
  w.zs = (double*)L.add(n * 8);
  w.colscale = (double*)L.add(n * 8);
  w.stat = (double*)L.add(STAT_N * 8);
  w.grid = (int32_t*)L.add(BS_G * 4);
  w.counters = (int32_t*)L.add(64 * 4);
  w.total = L.total;
  return w;
}

// A12 := A12 - U01^H U01' on the upper triangle of the target (rows r0.., columns c0..), with
// U01 the k rows of U starting at row u0: one MFMA GEMM.
bool herk_update(double2* H1, int64_t ld, int64_t u0, int k, int64_t r0, int rows, int64_t c0,
                 int cols, int tile, const char* tag, int32_t* info, hipStream_t s) {
  ZgemmParams h;
  h.M = rows;
  h.N = cols;
  h.K = k;
  h.A = H1 + u0 + r0 * ld;  // (m, kk) = conj(U[u0 + kk][r0 + m])
  h.a_rs = ld;
  h.a_cs = 1;
  h.conjA = 1;
  h.B = H1 + u0 + c0 * ld;  // (kk, j) = U[u0 + kk][c0 + j]
  h.b_rs = 1;
  h.b_cs = ld;
  h.C = H1 + r0 + c0 * ld;
  h.c_rs = 1;
  h.c_cs = ld;
  h.alpha = make_double2(-1.0, 0.0);
  h.beta = 1.0;
  h.c_uplo = 1;
  h.info = info;
  h.tag = tag;
  h.tile = tile;
  return zgemm(h, 1, s) == hipSuccess;
}

// X := U^-1 X for the n x n upper triangular U (real diagonal; column-major,
// ld) and n x ncols X (ldx): blocks of TS_NB rows from the bottom, each solved
// in 32-row diagonal blocks (the rows above them within the block updated by a
// product of K <= 32), then the rows above the block updated by one product of
// K = TS_NB.
constexpr int TS_NB = 256;
bool trsm_upper(const double2* U, int64_t ld, int64_t n, double2* X, int64_t ldx, int64_t ncols,
                int32_t* info, hipStream_t s) {
  auto update = [&](int64_t r0, int64_t rows, int64_t c0, int64_t k, const char* tag) {
    ZgemmParams g;  // X[r0 : r0+rows] -= U[r0 : r0+rows, c0 : c0+k] X[c0 : c0+k]
    g.M = (int)rows;
    g.N = (int)ncols;
    g.K = (int)k;
    g.A = U + r0 + c0 * ld;
    g.a_rs = 1;
    g.a_cs = ld;
    g.B = X + c0;
    g.b_rs = 1;
    g.b_cs = ldx;
    g.C = X + r0;
    g.c_rs = 1;
    g.c_cs = ldx;
    g.alpha = make_double2(-1.0, 0.0);
    g.beta = 1.0;
    g.info = info;
    g.tag = tag;
    g.tile = tune_choice(BSE_TUNE_GEMM_VECTORS, n, 32);
    return zgemm(g, 1, s) == hipSuccess;
  };
  for (int64_t i0 = ((n - 1) / TS_NB) * TS_NB, i1 = n; i1 > 0; i1 = i0, i0 -= TS_NB) {
    for (int64_t s0 = i0 + ((i1 - 1 - i0) / 32) * 32, s1 = i1; s1 > i0; s1 = s0, s0 -= 32) {
      BSE_LAUNCH(k_trsm_diag, dim3((unsigned)cdiv(ncols, 256)), dim3(256), 0, s,
                 U + s0 + s0 * ld, ld, (int)(s1 - s0), X + s0, ldx, ncols, info);
      if (s0 > i0 && !update(i0, s0 - i0, s0, s1 - s0, "zgemm_trsm_in")) return false;
    }
    if (i0 > 0 && !update(0, i0, i0, i1 - i0, "zgemm_trsm")) return false;
  }
  return hipGetLastError() == hipSuccess;
}

// A - B = U^H U (upper).  Panels of CH_NB columns are factored in pairs: after
// the first panel of a pair only the second panel's rows are updated (K =
// CH_NB), and after the second the trailing matrix takes one update of
// K = 2 CH_NB, which halves the passes over it.
bool cholesky(double2* H1, int64_t n, int64_t ld, double2* u11, int32_t* info, hipStream_t s) {
  const int tile = tune_choice(BSE_TUNE_GEMM_POTRF, n, 0);
  for (int64_t j0 = 0; j0 < n; j0 += 2 * CH_NB) {
    const int jb = (int)std::min<int64_t>(CH_NB, n - j0);
    const int64_t j1 = j0 + jb, rest1 = n - j1;
    BSE_LAUNCH(k_potrf_panel, dim3((unsigned)std::max<int64_t>(1, cdiv(rest1, PCOLS))),
               dim3(PCOLS), 0, s, H1, ld, n, (int)j0, jb, u11, info);
    if (rest1 <= 0) break;
    const int jb2 = (int)std::min<int64_t>(CH_NB, rest1);
    const int64_t j2 = j1 + jb2, rest2 = n - j2;
    // rows j1 .. j2-1 (the next panel) over columns j1 .. n-1
    if (!herk_update(H1, ld, j0, jb, j1, jb2, j1, (int)rest1, tile, "zgemm_potrf_rows", info, s))
      return false;
    BSE_LAUNCH(k_potrf_panel, dim3((unsigned)std::max<int64_t>(1, cdiv(rest2, PCOLS))),
               dim3(PCOLS), 0, s, H1, ld, n, (int)j1, jb2, u11, info);
    if (rest2 <= 0) break;
    // trailing matrix: rows and columns j2 .. n-1, K = jb + jb2
    if (!herk_update(H1, ld, j0, jb + jb2, j2, (int)rest2, j2, (int)rest2, tile,
                     "zgemm_potrf_herk", info, s))
      return false;
  }
  BSE_LAUNCH(k_potrf_store, dim3((unsigned)cdiv(n, CH_NB)), dim3(256), 0, s, H1, ld, n, u11, info);
  return true;
}

ZgemmItem herk_item(const CholItem& q, int64_t u0, int k, int64_t r0, int rows, int64_t c0,
                    int cols) {
  ZgemmItem h;  // as herk_update: C(r0.., c0..) -= U(u0.., r0..)^H U(u0.., c0..)
  h.M = rows;
  h.N = cols;
  h.K = k;
  h.A = q.A + u0 + r0 * q.ld;
  h.a_rs = q.ld;
  h.a_cs = 1;
  h.B = q.A + u0 + c0 * q.ld;
  h.b_rs = 1;
  h.b_cs = q.ld;
  h.C = q.A + r0 + c0 * q.ld;
  h.c_rs = 1;
  h.c_cs = q.ld;
  h.info = q.info;
  return h;
}

}  // namespace

// cholesky() of several problems in step: one panel launch per panel serves
// every problem, and the updates after it run as one grouped GEMM (each item
// with the tile zgemm() would give it alone): every problem's values are those
// of cholesky() on its own.  Problems with the same tuned tile only (the
// caller groups them); at most CHOL_GROUP_MAX per call.
bool cholesky_batch(const CholItem* it, int np, hipStream_t s) {
  if (np <= 0) return true;
  if (np > CHOL_GROUP_MAX) return false;
  PotrfGroup g{};
  int64_t nmax = 0;
  for (int p = 0; p < np; ++p) {
    g.it[p] = it[p];
    nmax = std::max(nmax, it[p].n);
  }
  const int tile = tune_choice(BSE_TUNE_GEMM_POTRF, it[0].n, 0);
  ZgemmParams base;
  base.conjA = 1;
  base.alpha = make_double2(-1.0, 0.0);
  base.beta = 1.0;
  base.c_uplo = 1;
  base.tile = tile;
  std::vector<ZgemmItem> up;
  auto panel = [&](int64_t j0) {
    int gx = 0;
    for (int p = 0; p < np; ++p) {
      if (j0 >= it[p].n) continue;
      const int64_t rest = it[p].n - j0 - std::min<int64_t>(CH_NB, it[p].n - j0);
      gx = std::max(gx, rest > 0 ? cdiv(rest, PCOLS) : 1);
    }
    if (gx > 0)
      BSE_LAUNCH(k_potrf_panel_b, dim3((unsigned)gx, (unsigned)np), dim3(PCOLS), 0, s, g,
                 (int)j0);
  };
  for (int64_t j0 = 0; j0 < nmax; j0 += 2 * CH_NB) {
    panel(j0);
    const int64_t j1 = j0 + CH_NB;
    up.clear();
    for (int p = 0; p < np; ++p) {  // rows j1 .. j2-1 over columns j1 .. n-1
      const int64_t n = it[p].n, rest1 = n - j1;
      if (j0 >= n || rest1 <= 0) continue;
      const int jb2 = (int)std::min<int64_t>(CH_NB, rest1);
      up.push_back(herk_item(it[p], j0, CH_NB, j1, jb2, j1, (int)rest1));
    }
    base.tag = "zgemm_potrf_rows";
    if (!up.empty() && zgemm_group(base, up.data(), (int)up.size(), s) != hipSuccess) return false;
    panel(j1);
    up.clear();
    for (int p = 0; p < np; ++p) {  // trailing matrix: rows and columns j2 .. n-1
      const int64_t n = it[p].n, rest1 = n - j1;
      if (j0 >= n || rest1 <= 0) continue;
      const int64_t j2 = j1 + std::min<int64_t>(CH_NB, rest1), rest2 = n - j2;
      if (rest2 <= 0) continue;
      up.push_back(herk_item(it[p], j0, 2 * CH_NB, j2, (int)rest2, j2, (int)rest2));
    }
    base.tag = "zgemm_potrf_herk";
    if (!up.empty() && zgemm_group(base, up.data(), (int)up.size(), s) != hipSuccess) return false;
  }
  for (int p = 0; p < np; ++p)
    BSE_LAUNCH(k_potrf_store, dim3((unsigned)cdiv(it[p].n, CH_NB)), dim3(256), 0, s, it[p].A,
               it[p].ld, it[p].n, it[p].u11, it[p].info);
  return hipGetLastError() == hipSuccess;
}

namespace {

// Z := Q Z for the n x ncols complex matrix Z (column-major, ldz).
// Groups of QG consecutive panels at a time (Z := P_a0 P_a1 ... Z, P_p = I - V_p
// T_p V_p^H): with V = [V_a0 V_a1 ...] (columns J0.., rows J0+1..), W = V^H Z and
// the Gram blocks G = V^H V, the panels' coefficient rows are Y_b = T_b (W_b -
// sum_{c > b} G_bc Y_c), taken from the last panel back, and then Z -= V Y in one
// product: one launch of K = m rows (W and G side by side) and one product of
// K = 32 QG columns per group in place of QG of each with 32 (the panel products
// of a 32-wide V use a small part of the machine at these orders).
bool apply_q_grouped(const double2* M, int64_t n, int64_t ld, double2* Z, int64_t ldz,
                     int64_t ncols, int QG, SolveWs& w, int32_t* info, hipStream_t s) {
  const int GW = QG * TRD_NB;  // leading dimension of W, Y and G
  const int64_t npnl = (n - 1 + TRD_NB - 1) / TRD_NB;
  double2* W = (double2*)w.Dp;     // GW x ncols (pivot arrays: free after the eigenvectors)
  double2* Y = (double2*)w.Dm;     // GW x ncols
  double2* G = (double2*)w.Ztri;   // GW x GW (free once Z holds the eigenvectors)
  const int64_t ngrp = (npnl + QG - 1) / QG;
  for (int64_t g = ngrp - 1; g >= 0; --g) {
    const int64_t p0 = g * QG, J0 = p0 * TRD_NB, m = n - J0 - 1;
    const int k = (int)std::min<int64_t>(QG, npnl - p0);
    const int wg = (int)std::min<int64_t>(GW, n - 1 - J0);
    const double2* V = M + (J0 + 1) + J0 * ld;
    // W = V^H Z[J0+1:, :] and G = V^H V (only its blocks above the diagonal
    // are used) in one launch: the Gram's few tiles run beside W's
    ZgemmItem it[2];
    it[0].M = wg;
    it[0].N = (int)ncols;
    it[0].K = (int)m;
    it[0].A = V;
    it[0].a_rs = ld;
    it[0].a_cs = 1;
    it[0].a_tri = 1;
    it[0].B = Z + (J0 + 1);
    it[0].b_rs = 1;
    it[0].b_cs = ldz;
    it[0].C = W;
    it[0].c_rs = 1;
    it[0].c_cs = GW;
    it[0].info = info;
    it[1] = it[0];
    it[1].N = wg;
    it[1].B = V;
    it[1].b_cs = ld;
    it[1].b_tri = 2;
    it[1].C = G;
    ZgemmParams a;
    a.conjA = 1;
    a.products = tune_choice(BSE_TUNE_GEMM_PRODUCTS, std::max<int64_t>(wg, ncols), 3);
    a.tag = "zgemm_bt_vhz";
    a.tile = tune_choice(BSE_TUNE_GEMM_VECTORS, n, 32);
    if (zgemm_group(a, it, k > 1 ? 2 : 1, s) != hipSuccess) return false;
    for (int b = k - 1; b >= 0; --b) {
      const int64_t pnl = p0 + b;
      const int jb = (int)std::min<int64_t>(TRD_NB, n - 1 - pnl * TRD_NB);
      const int r0 = b * TRD_NB, rest = wg - r0 - jb;  // rows of the later panels in Y
      if (rest > 0) {
        ZgemmParams c;  // W_b -= G[b, later] Y[later]
        c.M = jb;
        c.N = (int)ncols;
        c.K = rest;
        c.A = G + r0 + (int64_t)(r0 + jb) * GW;
        c.a_rs = 1;
        c.a_cs = GW;
        c.B = Y + (r0 + jb);
        c.b_rs = 1;
        c.b_cs = GW;
        c.C = W + r0;
        c.c_rs = 1;
        c.c_cs = GW;
        c.alpha = make_double2(-1.0, 0.0);
        c.beta = 1.0;
        c.info = info;
        c.tag = "zgemm_bt_gw";
        if (zgemm(c, 1, s) != hipSuccess) return false;
      }
      ZgemmParams t;  // Y_b = T_b W_b
      t.M = jb;
      t.N = (int)ncols;
      t.K = jb;
      t.A = w.Tall + pnl * TRD_NB * TRD_NB;
      t.a_rs = 1;
      t.a_cs = TRD_NB;
      t.a_tri = 1;
      t.B = W + r0;
      t.b_rs = 1;
      t.b_cs = GW;
      t.C = Y + r0;
      t.c_rs = 1;
      t.c_cs = GW;
      t.info = info;
      t.tag = "zgemm_bt_tw";
      if (zgemm(t, 1, s) != hipSuccess) return false;
    }
    ZgemmParams u;  // Z[J0+1:, :] -= V Y
    u.M = (int)m;
    u.N = (int)ncols;
    u.K = wg;
    u.A = V;
    u.a_rs = 1;
    u.a_cs = ld;
    u.a_tri = 2;
    u.B = Y;
    u.b_rs = 1;
    u.b_cs = GW;
    u.C = Z + (J0 + 1);
    u.c_rs = 1;
    u.c_cs = ldz;
    u.alpha = make_double2(-1.0, 0.0);
    u.beta = 1.0;
    u.info = info;
    u.tag = "zgemm_bt_update";
    u.tile = tune_choice(BSE_TUNE_GEMM_VECTORS, n, 32);
    if (zgemm(u, 1, s) != hipSuccess) return false;
  }
  return true;
}

bool apply_q(const double2* M, int64_t n, int64_t ld, double2* Z, int64_t ldz, int64_t ncols,
             SolveWs& w, int32_t* info, hipStream_t s) {
  // groups of 8, else 4 panels, when the pivot arrays hold W and Y (32 QG rows
  // of Z's columns each) and Ztri holds G (measured at N = 6144 with vectors:
  // solve 358 ms panel by panel, 320 ms in groups of 4, 316 ms in groups of 8)
  for (int qg : {8, 4}) {
    const int64_t gw = (int64_t)qg * TRD_NB;
    if (gw * ncols * 16 <= n * (n + EV_JUNK) * 8 && gw * gw * 16 <= n * n * 8)
      return apply_q_grouped(M, n, ld, Z, ldz, ncols, qg, w, info, s);
  }
  const int64_t npnl = (n - 1 + TRD_NB - 1) / TRD_NB;
  double2* W1 = w.W1;  // jb x ncols
  double2* W2 = w.W2;  // jb x ncols
  for (int64_t pnl = npnl - 1; pnl >= 0; --pnl) {
    const int64_t j0 = pnl * TRD_NB;
    const int jb = (int)std::min<int64_t>(TRD_NB, n - 1 - j0);
    const int64_t m = n - j0 - 1;
    const double2* V = M + (j0 + 1) + j0 * ld;
    ZgemmParams a;  // W1 = V^H Z[j0+1:, :]
    a.M = jb;
    a.N = (int)ncols;
    a.K = (int)m;
    a.A = V;
    a.a_rs = ld;
    a.a_cs = 1;
    a.conjA = 1;
    a.a_tri = 1;
    a.B = Z + (j0 + 1);
    a.b_rs = 1;
    a.b_cs = ldz;
    a.C = W1;
    a.c_rs = 1;
    a.c_cs = jb;
    a.info = info;
    a.tag = "zgemm_bt_vhz";
    a.tile = tune_choice(BSE_TUNE_GEMM_VECTORS, n, 32);
    if (zgemm(a, 1, s) != hipSuccess) return false;
    ZgemmParams b;  // W2 = T W1
    b.M = jb;
    b.N = (int)ncols;
    b.K = jb;
    b.A = w.Tall + pnl * TRD_NB * TRD_NB;
    b.a_rs = 1;
    b.a_cs = TRD_NB;
    b.a_tri = 1;
    b.B = W1;
    b.b_rs = 1;
    b.b_cs = jb;
    b.C = W2;
    b.c_rs = 1;
    b.c_cs = jb;
    b.info = info;
    b.tag = "zgemm_bt_tw";
    if (zgemm(b, 1, s) != hipSuccess) return false;
    ZgemmParams c;  // Z[j0+1:, :] -= V W2
    c.M = (int)m;
    c.N = (int)ncols;
    c.K = jb;
    c.A = V;
    c.a_rs = 1;
    c.a_cs = ld;
    c.a_tri = 2;
    c.B = W2;
    c.b_rs = 1;
    c.b_cs = jb;
    c.C = Z + (j0 + 1);
    c.c_rs = 1;
    c.c_cs = ldz;
    c.alpha = make_double2(-1.0, 0.0);
    c.beta = 1.0;
    c.info = info;
    c.tag = "zgemm_bt_update";
    c.tile = tune_choice(BSE_TUNE_GEMM_VECTORS, n, 32);
    if (zgemm(c, 1, s) != hipSuccess) return false;
  }
  return true;
}
}  // namespace

size_t solve_workspace(const bse_desc* d) { return carve(d, nullptr).total; }

void launch_zero_ints(int32_t* p, int n, hipStream_t s) {
  BSE_LAUNCH(k_zero_ints, dim3(1), dim3(64), 0, s, p, n);
}

bse_status solve_run(const bse_desc* d, void* H0v, void* H1v, double* E, void* XpYv, void* XmYv,
                     int64_t ldx, const void* probev, double* osc, void* ws, int32_t* info,
                     hipStream_t s, int phase) {
  const int64_t n = (int64_t)d->nk * d->nv * d->nc, ld = d->ld;
  const bool full = d->coupling == BSE_FULL;
  double2* H0 = (double2*)H0v;
  double2* H1 = (double2*)H1v;
  double2* XpY = (double2*)XpYv;
  double2* XmY = XpY ? (double2*)XmYv : nullptr;
  const double2* probe = (const double2*)probev;
  SolveWs w = carve(d, ws);
  double2* Hm = H0;  // Hermitian matrix handed to the tridiagonalisation
  // spectrum-only: the probe is carried through the reduction, y = Q^H (U p)
  const bool project = (XpY == nullptr) && probe && osc;
  const dim3 cgrid((unsigned)std::min<int64_t>(cdiv(n, 256), 8),
                   (unsigned)std::min<int64_t>(n, 65535));
  if (phase & SOLVE_PRE1) {
    BSE_LAUNCH(k_zero_ints, dim3(1), dim3(64), 0, s, w.counters, 64);
  }
  if (full && (phase & SOLVE_CHOL) && !cholesky(H1, n, ld, w.W1, info, s)) return BSE_ERR_HIP;
  if (phase & SOLVE_PRE2) {
    if (full) {
      ZgemmParams a;  // T1 = (A+B) U^H
      a.M = (int)n;
      a.N = (int)n;
      a.K = (int)n;
      a.A = H0;
      a.a_rs = 1;
      a.a_cs = ld;
      a.B = H1;
      a.b_rs = ld;
      a.b_cs = 1;
      a.conjB = 1;
      a.b_tri = 2;
      a.C = w.Wk;
      a.c_rs = 1;
      a.c_cs = n;
      a.info = info;
      a.tag = "zgemm_sq_t1";
      a.tile = tune_choice(BSE_TUNE_GEMM_SQUARED, n, 0);
      if (zgemm(a, 1, s) != hipSuccess) return BSE_ERR_HIP;
      ZgemmParams b;  // S (lower) = U T1  -> H0
      b.M = (int)n;
      b.N = (int)n;
      b.K = (int)n;
      b.A = H1;
      b.a_rs = 1;
      b.a_cs = ld;
      b.a_tri = 1;
      b.B = w.Wk;
      b.b_rs = 1;
      b.b_cs = n;
      b.C = H0;
      b.c_rs = 1;
      b.c_cs = ld;
      b.c_uplo = 2;
      b.info = info;
      b.tag = "zgemm_sq_s";
      b.tile = tune_choice(BSE_TUNE_GEMM_SQUARED_S, n, tune_choice(BSE_TUNE_GEMM_SQUARED, n, 0));
      if (zgemm(b, 1, s) != hipSuccess) return BSE_ERR_HIP;
      const int nt = cdiv(n, 32);
      BSE_LAUNCH(k_hermitize, dim3(nt, nt), dim3(256), 0, s, H0, n, ld, 1, info);
    }

    if (project) {
      if (full) {
        // y = U p (the hemv partial-sum space is free until the sweep starts)
        const dim3 grid((unsigned)cdiv(n, TRMV_ROWS), (unsigned)cdiv(n, TRMV_COLS));
        BSE_LAUNCH(k_trmv_part, grid, dim3(TRMV_ROWS), 0, s, H1, ld, (int)n, probe, w.part, info);
        BSE_LAUNCH(k_trmv_sum, dim3(cdiv(n, 256)), dim3(256), 0, s, w.part, (int)n, w.yvec, info);
      } else {
        BSE_LAUNCH(k_copy_c, dim3(cdiv(n, 256)), dim3(256), 0, s, probe, w.yvec, n);
      }
    }
  }  // SOLVE_PRE2
  TrdBufs tb{w.VW, w.WV, w.ybuf, w.hs, w.part, w.dd, w.ee, w.tau, project ? w.yvec : nullptr};
  if ((phase & SOLVE_SWEEP) && !tridiagonalise(Hm, n, ld, tb, info, s)) return BSE_ERR_HIP;
  if (!(phase & SOLVE_POST)) return BSE_OK;
  BSE_LAUNCH(k_tri_prep, dim3(1), dim3(1024), 0, s, w.dd, w.ee, (int)n, w.ds, w.es, w.e2s,
             w.stat, info);
  BSE_LAUNCH(k_sturm_grid, dim3(BS_G / 64), dim3(64), 0, s, w.ds, w.e2s, (int)n, w.stat, w.grid,
             info);
  BSE_LAUNCH(k_bisect, dim3(cdiv(n, 4 * (64 / BS_L))), dim3(256), 0, s, w.ds, w.e2s, (int)n,
             w.stat, w.grid, w.mu, info);
  BSE_LAUNCH(k_monotone, dim3(1), dim3(1024), 0, s, w.mu, (int)n, info);
  constexpr double ortol_rel = 1e-5;  // gap, relative to ||T - c I||, of a cluster
  BSE_LAUNCH(k_eigvec, dim3(2 * cdiv(n, 64)), dim3(64), 0, s, w.ds, w.es, (int)n, w.mu,
             w.stat, ortol_rel, w.Ztri, w.Dp, w.Dm, w.zs, project ? w.yvec : nullptr,
             XpY ? 1 : 0, w.tproj, info);
  BSE_LAUNCH(k_cluster_orth, dim3((unsigned)n), dim3(256), 0, s, w.mu, (int)n, w.stat, ortol_rel,
             w.Ztri,
             project ? w.yvec : nullptr, w.tproj, info);
  BSE_LAUNCH(k_eigvals, dim3(cdiv(n, 256)), dim3(256), 0, s, w.mu, w.stat, w.zs, (int)n,
             full ? 1 : 0, E,
             w.colscale, project ? w.tproj : nullptr, osc, info);

  if (XpY) {
    const int64_t npnl = (n - 1 + TRD_NB - 1) / TRD_NB;
    if (npnl > 0)
      BSE_LAUNCH(k_larft, dim3((unsigned)npnl), dim3(256), 0, s, Hm, ld, (int)n, w.tau, w.Tall,
                 info);
    const int nt = cdiv(n, 32);
    double2* Z = full ? w.Wk : XpY;
    const int64_t ldz = full ? n : ldx;
    BSE_LAUNCH(k_ztri_to_complex, dim3(nt, nt), dim3(256), 0, s, w.Ztri, (int)n, w.colscale, Z,
               ldz, info);
    if (n > 1 && !apply_q(Hm, n, ld, Z, ldz, n, w, info, s)) return BSE_ERR_HIP;
    if (full) {
      ZgemmParams g;  // X+Y = U^H Z (columns already scaled by E^-1/2)
      g.M = (int)n;
      g.N = (int)n;
      g.K = (int)n;
      g.A = H1;
      g.a_rs = ld;
      g.a_cs = 1;
      g.conjA = 1;
      g.a_tri = 2;
      g.B = w.Wk;
      g.b_rs = 1;
      g.b_cs = n;
      g.C = XpY;
      g.c_rs = 1;
      g.c_cs = ldx;
      g.info = info;
      g.tag = "zgemm_recon";
      g.tile = tune_choice(BSE_TUNE_GEMM_VECTORS, n, 32);
      if (zgemm(g, 1, s) != hipSuccess) return BSE_ERR_HIP;
      if (XmY) {
        // X-Y = U^-1 Z E^1/2 = U^-1 (Z E^-1/2) E: the triangular solve in place on
        // the scaled Z (free after the product above), columns then scaled by E
        if (!trsm_upper(H1, ld, n, w.Wk, n, n, info, s)) return BSE_ERR_HIP;
        BSE_LAUNCH(k_copy_scale_cols, cgrid, dim3(256), 0, s, w.Wk, n, XmY, ldx, n, E, info);
      }
    } else if (XmY) {  // TDA: Y = 0, X-Y = X+Y = X
      BSE_LAUNCH(k_copy_mat, cgrid, dim3(256), 0, s, XpY, ldx, XmY, ldx, n);
    }
    if (probe && osc && launch_oscillator(n, XpY, ldx, probe, osc, s) != hipSuccess)
      return BSE_ERR_HIP;
  }
  return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
}

TrdItem solve_sweep_item(const bse_desc* d, void* H0, void* ws, bool project, int32_t* info) {
  const SolveWs w = carve(d, ws);
  TrdItem it;
  it.M = (double2*)H0;
  it.n = (int64_t)d->nk * d->nv * d->nc;
  it.ld = d->ld;
  it.w = TrdBufs{w.VW, w.WV, w.ybuf, w.hs, w.part, w.dd, w.ee, w.tau, project ? w.yvec : nullptr};
  it.info = info;
  return it;
}

CholItem solve_chol_item(const bse_desc* d, void* H1, void* ws, int32_t* info) {
  const SolveWs w = carve(d, ws);
  CholItem it;
  it.A = (double2*)H1;
  it.ld = d->ld;
  it.n = (int64_t)d->nk * d->nv * d->nc;
  it.u11 = w.W1;
  it.info = info;
  return it;
}
