// FP64 eigensolver of the BSE (paper Sec. 4.3).
//
// Full problem (squared form): with A-B = U^H U (Cholesky),
//   S = U (A+B) U^H  has the spectrum E^2 of (A-B)^1/2 (A+B) (A-B)^1/2,
//   S Z = E^2 Z,  X+Y = U^H Z E^-1/2.
// TDA: A X = E X.
// The Hermitian matrix (S or A) is reduced to a real symmetric tridiagonal
// T = Q^H S Q by Householder reflectors (blocked, lower), T is solved by
// multisection bisection and inverse iteration, and the eigenvectors are
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

__global__ void k_zero_ints(int32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
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
// stores U11.
constexpr int PCOLS = 256;
constexpr int PEL = CH_NB * CH_NB / PCOLS;  // diagonal-block elements per thread
__global__ __launch_bounds__(PCOLS) void k_potrf_panel(double2* __restrict__ A, int64_t ld,
                                                       int64_t n, int j0, int jb,
                                                       int32_t* info) {
  __shared__ double2 u[CH_NB][CH_NB + 1];  // rows of U11 as they are finished
  __shared__ double dsh[CH_NB];
  if (failed(info)) return;
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)j0 + jb + (int64_t)blockIdx.x * PCOLS;
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
      if (tid == 0 && blockIdx.x == 0) set_info(info, j0 + j + 1);
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
  if (blockIdx.x == 0)
    for (int e = tid; e < jb * jb; e += PCOLS) {
      const int r = e % jb, c = e / jb;
      if (r <= c) A[(int64_t)(j0 + r) + (int64_t)(j0 + c) * ld] = u[r][c];
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
// e2, Gershgorin bounds, pivmin and the norm of T.  stat[0]=gl, [1]=gu, [2]=pivmin, [3]=tnorm
__global__ __launch_bounds__(1024) void k_tri_prep(const double* __restrict__ d,
                                                   const double* __restrict__ e, int n,
                                                   double* __restrict__ e2, double* stat,
                                                   const int32_t* info) {
  __shared__ double slo[16], shi[16], sem[16];
  if (failed(info)) return;
  double lo = INFINITY, hi = -INFINITY, emax = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const double em = (k > 0) ? fabs(e[k - 1]) : 0.0, ep = (k < n - 1) ? fabs(e[k]) : 0.0;
    lo = fmin(lo, d[k] - em - ep);
    hi = fmax(hi, d[k] + em + ep);
    if (k < n - 1) {
      e2[k] = e[k] * e[k];
      emax = fmax(emax, e2[k]);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
    emax = fmax(emax, __shfl_xor(emax, off, 64));
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    slo[w] = lo;
    shi[w] = hi;
    sem[w] = emax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) {
      lo = fmin(lo, slo[i]);
      hi = fmax(hi, shi[i]);
      emax = fmax(emax, sem[i]);
    }
    const double tnorm = fmax(fabs(lo), fabs(hi));
    const double eps = 2.220446049250313e-16;
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);
    stat[0] = lo - 2.0 * eps * tnorm * n - 2.0 * pivmin;
    stat[1] = hi + 2.0 * eps * tnorm * n + 2.0 * pivmin;
    stat[2] = pivmin;
    stat[3] = tnorm;
  }
}

BSE_DEV int sturm_count(const double* __restrict__ d, const double* __restrict__ e2, int n, double x,
                        double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// 1/q to full double precision: hardware reciprocal refined by two Newton steps.
BSE_DEV double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(fma(-q, r, 1.0), r, r);
  r = fma(fma(-q, r, 1.0), r, r);
  return r;
}

// Eigenvalue k (ascending) by multisection: the 64 lanes of a wavefront probe
// 64 interior points of the bracket per round with Sturm counts of the
// LDL^T factorisation of T - x I.
__global__ __launch_bounds__(256) void k_bisect(const double* __restrict__ d,
                                                const double* __restrict__ e2, int n,
                                                const double* __restrict__ stat,
                                                double* __restrict__ w, const int32_t* info) {
  if (failed(info)) return;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n) return;
  double lo = stat[0], hi = stat[1];
  const double pivmin = stat[2];
  const double eps = 2.220446049250313e-16;
  constexpr double NP = 65.0;
  for (int it = 0; it < 40; ++it) {
    const double width = hi - lo;
    if (width <= 2.0 * eps * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin) break;
    const double x = lo + width * (double)(lane + 1) / NP;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    int cnt = q < 0.0;
    int i = 1;
    for (; i + 4 <= n; i += 4) {
      const double d0 = d[i], d1 = d[i + 1], d2 = d[i + 2], d3 = d[i + 3];
      const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
      q = (d0 - x) - f0 * recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      q = (d1 - x) - f1 * recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      q = (d2 - x) - f2 * recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
      q = (d3 - x) - f3 * recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    for (; i < n; ++i) {
      q = (d[i] - x) - e2[i - 1] * recip(q);
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += q < 0.0;
    }
    const unsigned long long mask = __ballot(cnt > k);
    double nlo, nhi;
    if (mask == 0ull) {
      nlo = lo + width * 64.0 / NP;
      nhi = hi;
    } else {
      const int f = __ffsll((long long)mask) - 1;
      nhi = lo + width * (double)(f + 1) / NP;
      nlo = (f > 0) ? lo + width * (double)f / NP : lo;
    }
    if (nlo == lo && nhi == hi) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) w[k] = 0.5 * (lo + hi);
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

// One inverse-iteration solve (T - lam I) x = s * b with partial pivoting:
// the forward sweep writes U (U0 diagonal, U1, U2 super-diagonals) and the
// eliminated rhs R; the backward sweep writes x into X and returns max |x|,
// sum x^2 and the index of the largest |x|.  The rhs b is X (scaled by s) or,
// when X_in_is_random, the start vector.  Arrays are [component i][eigenvalue j].
struct SolveStats {
  double big, nrm2;
  int ibig;
};

BSE_DEV SolveStats inv_solve(const double* __restrict__ d, const double* __restrict__ e, int n,
                             double lam, double tiny, int j, int64_t N, bool random_rhs,
                             double scale, double* __restrict__ X, double* __restrict__ U0,
                             double* __restrict__ U1, double* __restrict__ U2,
                             double* __restrict__ R) {
  constexpr int CH = 16;  // rows whose loads are issued together
  double di = d[0] - lam, dui = (n > 1) ? e[0] : 0.0;
  double rin = random_rhs ? hash_uniform(0u, (uint32_t)j) : X[j] * scale;
  for (int i0 = 0; i0 < n - 1; i0 += CH) {
    double rb[CH], db[CH], eb[CH], fb[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u;
      if (i < n - 1) {
        rb[u] = random_rhs ? hash_uniform((uint32_t)(i + 1), (uint32_t)j)
                           : X[(int64_t)(i + 1) * N + j] * scale;
        db[u] = d[i + 1];
        eb[u] = e[i];
        fb[u] = (i + 1 < n - 1) ? e[i + 1] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i0 + u;
      if (i < n - 1) {
        const double dl = eb[u];
        double d1 = db[u] - lam, du1 = fb[u], r1 = rb[u];
        double Ud, Uu, Uu2, ri;
        if (fabs(di) >= fabs(dl)) {
          const double f = (di != 0.0) ? dl / di : 0.0;
          Ud = di;
          Uu = dui;
          Uu2 = 0.0;
          ri = rin;
          d1 -= f * dui;
          r1 -= f * rin;
        } else {
          const double f = di / dl;
          Ud = dl;
          Uu = d1;
          Uu2 = du1;
          ri = r1;
          const double nd1 = dui - f * d1;
          du1 = -f * du1;
          r1 = rin - f * r1;
          d1 = nd1;
        }
        const int64_t o = (int64_t)i * N + j;
        U0[o] = Ud;
        U1[o] = Uu;
        U2[o] = Uu2;
        R[o] = ri;
        di = d1;
        dui = du1;
        rin = r1;
      }
    }
  }
  U0[(int64_t)(n - 1) * N + j] = di;
  R[(int64_t)(n - 1) * N + j] = rin;
  SolveStats st{0.0, 0.0, 0};
  double x1 = 0.0, x2 = 0.0;
  for (int i1 = n - 1; i1 >= 0; i1 -= CH) {
    double p0[CH], p1[CH], p2[CH], rr[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i1 - u;
      if (i >= 0) {
        const int64_t o = (int64_t)i * N + j;
        p0[u] = U0[o];
        p1[u] = (i < n - 1) ? U1[o] : 0.0;
        p2[u] = (i < n - 2) ? U2[o] : 0.0;
        rr[u] = R[o];
      }
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int i = i1 - u;
      if (i >= 0) {
        double p = p0[u];
        if (fabs(p) < tiny) p = (p >= 0.0) ? tiny : -tiny;
        const double xi = (rr[u] - p1[u] * x1 - p2[u] * x2) / p;
        X[(int64_t)i * N + j] = xi;
        const double ax = fabs(xi);
        if (ax > st.big) {
          st.big = ax;
          st.ibig = i;
        }
        st.nrm2 += xi * xi;
        x2 = x1;
        x1 = xi;
      }
    }
  }
  return st;
}

// Inverse iteration for every eigenvalue: one thread per cluster of close
// eigenvalues (gap <= ortol_rel * |lambda|); cluster members are orthogonalised
// against the earlier ones.  Two solves per eigenvalue from a pseudo-random
// start, then normalisation with the largest component made positive.
__global__ __launch_bounds__(256) void k_inviter(const double* __restrict__ d,
                                                 const double* __restrict__ e, int n,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ stat, double ortol_rel,
                                                 double* __restrict__ Z, double* __restrict__ U0,
                                                 double* __restrict__ U1, double* __restrict__ U2,
                                                 double* __restrict__ R, int32_t* info) {
  if (failed(info)) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double tnorm = stat[3];
  // close eigenvalues: gap below ortol_rel times the local magnitude (a few
  // outlying eigenvalues must not merge the rest of the spectrum into one cluster)
  auto close = [&](int a) {  // eigenvalues a and a+1
    return w[a + 1] - w[a] <= ortol_rel * fmax(fabs(w[a]), fabs(w[a + 1]));
  };
  if (k > 0 && close(k - 1)) return;  // not the first member of its cluster
  int kend = k;
  while (kend + 1 < n && close(kend)) ++kend;
  const double eps = 2.220446049250313e-16;
  const double tiny = eps * fmax(tnorm, 1e-300);
  const int64_t N = n;
  for (int j = k; j <= kend; ++j) {
    const double lam = w[j];
    SolveStats st = inv_solve(d, e, n, lam, tiny, j, N, true, 1.0, Z, U0, U1, U2, R);
    if (!(st.big > 0.0) || !isfinite(st.big)) {
      set_info(info, BSE_INFO_NO_CONVERGE);
      return;
    }
    st = inv_solve(d, e, n, lam, tiny, j, N, false, 1.0 / st.big, Z, U0, U1, U2, R);
    if (!(st.big > 0.0) || !isfinite(st.big)) {
      set_info(info, BSE_INFO_NO_CONVERGE);
      return;
    }
    double s = 1.0 / sqrt(st.nrm2);
    if (j > k) {
      // orthogonalise against the earlier members of the cluster, renormalise
      for (int i = 0; i < n; ++i) Z[(int64_t)i * N + j] *= s;
      for (int jp = k; jp < j; ++jp) {
        double dot = 0.0;
        for (int i = 0; i < n; ++i) dot += Z[(int64_t)i * N + jp] * Z[(int64_t)i * N + j];
        for (int i = 0; i < n; ++i) Z[(int64_t)i * N + j] -= dot * Z[(int64_t)i * N + jp];
      }
      double nrm2 = 0.0, big = 0.0;
      int ib = 0;
      for (int i = 0; i < n; ++i) {
        const double v = Z[(int64_t)i * N + j];
        nrm2 += v * v;
        if (fabs(v) > big) {
          big = fabs(v);
          ib = i;
        }
      }
      if (!(nrm2 > 0.0)) {
        set_info(info, BSE_INFO_NO_CONVERGE);
        return;
      }
      s = 1.0 / sqrt(nrm2);
      st.ibig = ib;
    }
    if (Z[(int64_t)st.ibig * N + j] < 0.0) s = -s;
    for (int i = 0; i < n; ++i) Z[(int64_t)i * N + j] *= s;
  }
}

// E = sqrt(mu) (full) and the column scale of Z (E^-1/2), or E = mu (TDA).
__global__ void k_eigvals(const double* __restrict__ mu, int n, int full, double* __restrict__ E,
                          double* __restrict__ colscale, int32_t* info) {
  if (failed(info)) return;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double m = mu[k];
  if (full) {
    if (!(m > 0.0)) {
      set_info(info, BSE_INFO_NOT_PD_PLUS);
      return;
    }
    const double ek = sqrt(m);
    E[k] = ek;
    colscale[k] = 1.0 / sqrt(ek);
  } else {
    E[k] = m;
    colscale[k] = 1.0;
  }
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

// osc[l] = |sum_i Ztri[i][l] y[i]|^2 * scale2[l]
__global__ __launch_bounds__(256) void k_osc_tri(const double* __restrict__ Zt, int n,
                                                 const double2* __restrict__ y,
                                                 const double* __restrict__ colscale,
                                                 double* __restrict__ osc, const int32_t* info) {
  if (failed(info)) return;
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  double2 s = make_double2(0.0, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    const double z = Zt[i * n + l];
    const double2 yi = y[i];
    s.x += z * yi.x;
    s.y += z * yi.y;
  }
  const double cs = colscale[l];
  osc[l] = cabs2(s) * cs * cs;
}

}  // namespace

// ------------------------------------------------------------------ host side
namespace {
struct SolveWs {
  double2* Wk;    // n x n complex (T1 of the squared form, then Z)
  double* Ztri;   // n x n real
  double* U0;
  double* U1;
  double* U2;
  double* U3;
  double2* VW;    // n x 2 TRD_NB panel [V | W]
  double2* WV;    // n x 2 TRD_NB panel [W | V]
  double2* W1;    // TRD_NB x n (back-transform)
  double2* W2;    // TRD_NB x n
  double2* ybuf;  // n
  double2* yvec;  // n (probe projection)
  double2* hs;    // small state
  double2* part;  // partial sums
  double2* Tall;  // T factors
  double2* tau;   // n
  double* dd;
  double* ee;
  double* e2;
  double* mu;
  double* colscale;
  double* stat;
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
  w.U0 = (double*)L.add(n * n * 8);
  w.U1 = (double*)L.add(n * n * 8);
  w.U2 = (double*)L.add(n * n * 8);
  w.U3 = (double*)L.add(n * n * 8);
  w.VW = (double2*)L.add(n * 2 * TRD_NB * 16);
  w.WV = (double2*)L.add(n * 2 * TRD_NB * 16);
  w.W1 = (double2*)L.add(n * TRD_NB * 16);
  w.W2 = (double2*)L.add(n * TRD_NB * 16);
  w.ybuf = (double2*)L.add(n * 16);
  w.yvec = (double2*)L.add(n * 16);
  w.hs = (double2*)L.add(HS_SIZE * 16);
  w.part = (double2*)L.add(trd_part_elems(n) * 16);
  w.Tall = (double2*)L.add(npnl * TRD_NB * TRD_NB * 16);
  w.tau = (double2*)L.add(n * 16);
  w.dd = (double*)L.add(n * 8);
  w.ee = (double*)L.add(n * 8);
  w.e2 = (double*)L.add(n * 8);
  w.mu = (double*)L.add(n * 8);
  w.colscale = (double*)L.add(n * 8);
  w.stat = (double*)L.add(8 * 8);
  w.counters = (int32_t*)L.add(64 * 4);
  w.total = L.total;
  return w;
}

bool cholesky(double2* H1, int64_t n, int64_t ld, int32_t* info, hipStream_t s) {
  for (int64_t j0 = 0; j0 < n; j0 += CH_NB) {
    const int jb = (int)std::min<int64_t>(CH_NB, n - j0);
    const int64_t rest = n - j0 - jb;
    BSE_LAUNCH(k_potrf_panel, dim3((unsigned)std::max<int64_t>(1, cdiv(rest, PCOLS))),
               dim3(PCOLS), 0, s, H1, ld, n, (int)j0, jb, info);
    if (rest <= 0) break;
    double2* A12 = H1 + j0 + (j0 + jb) * ld;
    ZgemmParams h;  // A22 -= U12^H U12 (upper)
    h.M = (int)rest;
    h.N = (int)rest;
    h.K = jb;
    h.A = A12;
    h.a_rs = ld;
    h.a_cs = 1;
    h.conjA = 1;
    h.B = A12;
    h.b_rs = 1;
    h.b_cs = ld;
    h.C = H1 + (j0 + jb) + (j0 + jb) * ld;
    h.c_rs = 1;
    h.c_cs = ld;
    h.alpha = make_double2(-1.0, 0.0);
    h.beta = 1.0;
    h.c_uplo = 1;
    h.info = info;
    h.tag = "zgemm_potrf_herk";
    h.tile = tune_choice(BSE_TUNE_GEMM_POTRF, n, 0);
    if (zgemm(h, 1, s) != hipSuccess) return false;
  }
  return true;
}

// Z := Q Z for the n x ncols complex matrix Z (column-major, ldz).
bool apply_q(const double2* M, int64_t n, int64_t ld, double2* Z, int64_t ldz, int64_t ncols,
             SolveWs& w, int32_t* info, hipStream_t s) {
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
    if (zgemm(c, 1, s) != hipSuccess) return false;
  }
  return true;
}
}  // namespace

size_t solve_workspace(const bse_desc* d) { return carve(d, nullptr).total; }

void launch_zero_ints(int32_t* p, int n, hipStream_t s) {
  BSE_LAUNCH(k_zero_ints, dim3(1), dim3(64), 0, s, p, n);
}

bse_status solve_run(const bse_desc* d, void* H0v, void* H1v, double* E, void* XpYv, int64_t ldx,
                     const void* probev, double* osc, void* ws, int32_t* info, hipStream_t s) {
  const int64_t n = (int64_t)d->nk * d->nv * d->nc, ld = d->ld;
  const bool full = d->coupling == BSE_FULL;
  double2* H0 = (double2*)H0v;
  double2* H1 = (double2*)H1v;
  double2* XpY = (double2*)XpYv;
  const double2* probe = (const double2*)probev;
  SolveWs w = carve(d, ws);
  BSE_LAUNCH(k_zero_ints, dim3(1), dim3(64), 0, s, w.counters, 64);

  double2* Hm = H0;  // Hermitian matrix handed to the tridiagonalisation
  if (full) {
    if (!cholesky(H1, n, ld, info, s)) return BSE_ERR_HIP;
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
    b.tile = tune_choice(BSE_TUNE_GEMM_SQUARED, n, 0);
    if (zgemm(b, 1, s) != hipSuccess) return BSE_ERR_HIP;
    const int nt = cdiv(n, 32);
    BSE_LAUNCH(k_hermitize, dim3(nt, nt), dim3(256), 0, s, H0, n, ld, 1, info);
  }

  // spectrum-only: the probe is carried through the reduction, y = Q^H (U p)
  const bool project = (XpY == nullptr) && probe && osc;
  if (project) {
    if (full) {
      ZgemmParams g;  // y = U p
      g.M = (int)n;
      g.N = 1;
      g.K = (int)n;
      g.A = H1;
      g.a_rs = 1;
      g.a_cs = ld;
      g.a_tri = 1;
      g.B = probe;
      g.b_rs = 1;
      g.b_cs = n;
      g.C = w.yvec;
      g.c_rs = 1;
      g.c_cs = n;
      g.info = info;
      g.tag = "zgemm_probe_up";
      if (zgemm(g, 1, s) != hipSuccess) return BSE_ERR_HIP;
    } else {
      BSE_LAUNCH(k_copy_c, dim3(cdiv(n, 256)), dim3(256), 0, s, probe, w.yvec, n);
    }
  }
  TrdBufs tb{w.VW, w.WV, w.ybuf, w.hs, w.part, w.dd, w.ee, w.tau, project ? w.yvec : nullptr};
  if (!tridiagonalise(Hm, n, ld, tb, info, s)) return BSE_ERR_HIP;
  BSE_LAUNCH(k_tri_prep, dim3(1), dim3(1024), 0, s, w.dd, w.ee, (int)n, w.e2, w.stat, info);
  BSE_LAUNCH(k_bisect, dim3(cdiv(n, 4)), dim3(256), 0, s, w.dd, w.e2, (int)n, w.stat, w.mu,
             info);
  BSE_LAUNCH(k_inviter, dim3(cdiv(n, 256)), dim3(256), 0, s, w.dd, w.ee, (int)n, w.mu, w.stat,
             1e-5, w.Ztri, w.U0, w.U1, w.U2, w.U3, info);
  BSE_LAUNCH(k_eigvals, dim3(cdiv(n, 256)), dim3(256), 0, s, w.mu, (int)n, full ? 1 : 0, E,
             w.colscale, info);

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
      if (zgemm(g, 1, s) != hipSuccess) return BSE_ERR_HIP;
    }
    if (probe && osc && launch_oscillator(n, XpY, ldx, probe, osc, s) != hipSuccess)
      return BSE_ERR_HIP;
  } else if (project) {
    BSE_LAUNCH(k_osc_tri, dim3(cdiv(n, 256)), dim3(256), 0, s, w.Ztri, (int)n, w.yvec,
               w.colscale, osc, info);
  }
  return hipGetLastError() == hipSuccess ? BSE_OK : BSE_ERR_HIP;
}
