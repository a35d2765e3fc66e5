/* bse.h -- C ABI of the MI355X (gfx950) Bethe-Salpeter hot path.
 *
 * The library builds the electron-hole Hamiltonian of the Bethe-Salpeter
 * equation in transition space, solves it (full, beyond the Tamm-Dancoff
 * approximation, through the Hermitian squared form; or in the TDA) and
 * forms oscillator strengths and the macroscopic dielectric function, after
 * Vorwerk, Aurich, Cocchi and Draxl, "Bethe-Salpeter equation for absorption
 * and scattering spectroscopy: implementation in the exciting code"
 * (Sec. 2.3 matrix form, Sec. 4.2 matrix elements, Sec. 4.3 eigenvalue
 * problem, Sec. 4.4 dielectric properties).
 *
 * Conventions shared by every entry point
 *  - Every pointer argument is a DEVICE pointer owned by the caller unless
 *    stated otherwise.  The library never allocates, frees or retains
 *    caller memory; scratch space comes from the caller's `ws` buffer,
 *    sized by bse_workspace_size().
 *  - Complex numbers are interleaved (re, im) doubles (16 bytes).
 *  - Transition index a = (ik * nv + iv) * nc + ic  (k-point major, then the
 *    occupied band, then the unoccupied band); n = nk * nv * nc.
 *  - N x N matrices are column-major with leading dimension ld >= n.  On
 *    output of bse_build both triangles are filled and Hermitian.
 *  - k-pairs: only pairs ik <= ik' are stored, in row-major order
 *    (pair p = ik*nk - ik*(ik-1)/2 + (ik' - ik)); P = nk*(nk+1)/2.
 *  - Every call only enqueues work on `stream` (no host synchronisation, no
 *    allocation) and returns a host-side status from argument checks and
 *    launch errors.  Failures found by the kernels are written to the
 *    caller's device word `info` (int32, must be zero on entry):
 *       0   success
 *      >0   Cholesky of A-B stopped at this 1-based column: A-B is not
 *           positive definite (the squared form needs it, Sec. 4.3)
 *      -1   a qmap / qramap entry outside [0, nq)
 *      -2   a non-finite value on the diagonal of an assembled matrix
 *      -3   a squared-form eigenvalue E^2 <= 0: A+B is not positive definite
 *      -4   a tridiagonal eigenvector came out zero or non-finite (the
 *           twisted factorisation, or inverse iteration inside a cluster)
 *      -5   bse_screening: an occupied band is not below an unoccupied one
 *      -6   bse_screening: a pivot of the dielectric-matrix inversion is not
 *           positive (non-finite input)
 *    Once `info` is non-zero, the later kernels of the same calls return at
 *    entry, except the per-column kernels of the Householder sweep, which
 *    index no memory by data and run on; outputs are then undefined.
 */
#ifndef BSE_H
#define BSE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BSE_OK = 0,
  BSE_ERR_ARG = 1,        /* invalid size, null pointer, ld < n, unsupported mode */
  BSE_ERR_WORKSPACE = 2,  /* ws_bytes smaller than bse_workspace_size() */
  BSE_ERR_HIP = 3         /* a HIP launch failed */
} bse_status;

/* Sec. 4.3: full problem through the squared form, or the TDA (B = 0). */
typedef enum { BSE_TDA = 0, BSE_FULL = 1 } bse_coupling;

/* Spin factors (gamma_x, gamma_c) of eqs. diagonalblock / couplingblock,
 * table of calculation types in Appendix B:
 * singlet (1,1), triplet (0,1), RPA (1,0), independent particles (0,0). */
typedef enum { BSE_SINGLET = 0, BSE_TRIPLET = 1, BSE_RPA = 2, BSE_IP = 3 } bse_type;

/* Arithmetic of the kernel assembly; the solve is always FP64.
 *  FP64   : FP64 matrix-core products throughout.
 *  FP32   : the exchange term and the W contraction of both direct terms
 *           (eqs. wrrm, wrabar: conj(M) W(q), 85% of the assembly flops) use
 *           operands rounded to FP32, FP32 products and accumulation inside
 *           chunks of 16 complex terms, FP64 accumulation across chunks.
 *  BF16X3 : as FP32, with operands split into three BF16 terms
 *           (hi + mid + lo); split_terms = 6 (default) keeps the products
 *           hi*hi, hi*mid, mid*hi, hi*lo, lo*hi, mid*mid, split_terms = 3 the
 *           first three.
 * The per-pair second contraction of the direct terms (R x N_G x R' per
 * k-pair, memory-bound) runs in FP64 in every mode.  The reduced modes split
 * W once per call into a part of the BUILD workspace sized for nk slices
 * (2 nk for the full BSE: the q-mesh and the second q-set of -k-k' on a
 * shifted k-mesh), so they require nq <= nk, or nq <= 2 nk for the full BSE
 * (else BSE_ERR_ARG). */
typedef enum { BSE_PREC_FP64 = 0, BSE_PREC_FP32 = 1, BSE_PREC_BF16X3 = 2 } bse_precision;

typedef enum { BSE_STAGE_BUILD = 0, BSE_STAGE_SOLVE = 1 } bse_stage;

typedef struct {
  int32_t nk, nv, nc, ng; /* k-points, occupied and unoccupied bands, plane waves */
  int32_t coupling;       /* bse_coupling */
  int32_t type;           /* bse_type */
  int32_t prec;           /* bse_precision */
  int32_t split_terms;    /* BSE_PREC_BF16X3 only: 3 or 6 products (0 = 6) */
  double kappa;           /* kernel prefactor: 1/V_c of eq. vft in energy units */
  double scissor;         /* rigid shift added to every transition energy */
  int64_t ld;             /* leading dimension of the N x N matrices, >= n */
} bse_desc;

/* Inputs of one BSE problem (all device pointers, read only). */
typedef struct {
  const double* eps_v;   /* [nk][nv] occupied energies */
  const double* eps_c;   /* [nk][nc] unoccupied energies */
  const void* Mcv;       /* complex [n][ng]: M_a(G) of eq. vrrofM (pair a = (k, v, c)) */
  const void* Mvv;       /* complex [P][nv][nv'][ng]: M_{o o'}(G) of eq. wrrm for pair p */
  const void* Mcc;       /* complex [P][nc][nc'][ng]: M_{u u'}(G') of eq. wrrm, or NULL:
                            drawn in place from mcc_env and mcc_key (below) */
  const void* Ncv;       /* complex [P][nc][nv'][ng]: N_{u o'}(G) of eq. wrabar (full only) */
  const void* Nvc;       /* complex [P][nv][nc'][ng]: N_{o u'}(G') of eq. wrabar (full only) */
  const void* W;         /* complex [nq][ng][ng]: screened interaction w_GG'(q), eq. wggq */
  const double* vbar;    /* [ng]: Coulomb potential without the G_Q term, eq. vbar_def */
  const int32_t* qmap;   /* [nk][nk]: class of k - k'  (index into W) */
  const int32_t* qramap; /* [nk][nk]: class of -k - k' (index into W), full only.  On a
                            k-mesh shifted by s (k = (i + s)/n, Sec. 5), -k - k' lies
                            on the q-mesh only when 2s is integral; otherwise its W
                            slices (the second set (j - 2s)/n) follow the nk of the
                            q-mesh in W and qramap indexes them (nq = 2 nk). */
  int32_t nq;            /* number of W slices */
  int32_t reserved;
  /* M_{u u'}(G') given implicitly, for problems where the array would not fit
   * in memory (core-level spectra: P x nc^2 x ng values).  Used when Mcc is
   * NULL:  M[p][u][u'][G] = mcc_env[G] * (x + i y) / sqrt(2), where x, y are
   * the Box-Muller normals sqrt(-2 ln u1) (cos, sin)(2 pi u2) of the uniforms
   * u1 = (k1 + 1) 2^-53 and u2 = k2 2^-53, k1 and k2 the top 53 bits of the
   * 64-bit words (w1:w0) and (w3:w2) of the Philox4x32-10 block (Salmon et al.,
   * SC'11) at counter (p, u, u', G) under key (mcc_key & 0xffffffff,
   * mcc_key >> 32).  The values are drawn inside the direct-term contraction
   * and never stored; results agree with the stored form to rounding. */
  const double* mcc_env; /* [ng] real envelope (device), NULL when Mcc is given */
  uint64_t mcc_key;
} bse_inputs;

/* Bytes of scratch space `ws` needed by bse_build (stage BUILD) or
 * bse_solve (stage SOLVE) for this descriptor; 0 for an invalid one. */
size_t bse_workspace_size(const bse_desc* desc, int32_t stage);

/* Kernel assembly (Sec. 2.3 eqs. diagonalblock and couplingblock with the
 * matrix elements of Sec. 4.2).
 *  full: H0 <- A + B,  H1 <- A - B
 *  TDA : H0 <- A       (H1 unused, may be NULL)
 * with A = E + kappa (2 gx V - gc W^rr), B = kappa (2 gx V - gc W^ra).
 * Only pairs ik <= ik' are evaluated; the lower triangle is their conjugate
 * mirror and the diagonal is real.  H0/H1: complex n x n, column-major, ld. */
bse_status bse_build(const bse_desc* desc, const bse_inputs* in, void* H0, void* H1, void* ws,
                     size_t ws_bytes, int32_t* info, hipStream_t stream);

/* Eigenproblem (Sec. 4.3).
 *  full: A-B = U^H U (Cholesky), S = U (A+B) U^H, S Z = E^2 Z,
 *        X+Y = U^H Z E^-1/2  (same E and, up to phase, the same X+Y as the
 *        (A-B)^1/2 form of eq. auxham),
 *        X-Y = U^-1 Z E^1/2  (the (A-B)^-1/2 E^1/2 Z of the same section in
 *        Cholesky form), by a triangular solve with U; then
 *        (X+Y)^H (X-Y) = I and (A+B)(X+Y) = (X-Y) E.
 *  TDA : A X = E X.
 *  H0, H1: the matrices from bse_build (overwritten).
 *  E     : [n] excitation energies, ascending (output).
 *  XpY   : complex n x n column-major with leading dimension ldx, column l =
 *          (X+Y)_l (X_l in the TDA); may be NULL when only the spectrum is
 *          wanted, which skips the eigenvector back-transform.
 *  XmY   : complex n x n column-major, leading dimension ldx, column l =
 *          (X-Y)_l with the phase of (X+Y)_l (X_l again in the TDA), or NULL.
 *          Needs XpY (else BSE_ERR_ARG) and a buffer of its own; it holds a
 *          copy of A+B while the solve runs.
 *  probe : complex [n] vector p (for eps_M: p_a = conj M_a(G_Q)) or NULL.
 *  osc   : [n] |t_l|^2 = |sum_a conj((X+Y)_al) p_a|^2 (eq. osci), written
 *          when probe != NULL. */
bse_status bse_solve(const bse_desc* desc, void* H0, void* H1, double* E, void* XpY, void* XmY,
                     int64_t ldx, const void* probe, double* osc, void* ws, size_t ws_bytes,
                     int32_t* info, hipStream_t stream);

/* bse_solve without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The scratch space is a fixed array of
 * BSE_NOALLOC_SCRATCH_BYTES inside the library, one per GPU, held until the
 * process ends; its address is looked up on the first call made on each
 * device.  The call allocates nothing (no hipMalloc, no library allocation).
 * Arguments, outputs and device errors are those of bse_solve.
 * BSE_ERR_WORKSPACE when bse_workspace_size(desc, BSE_STAGE_SOLVE) exceeds
 * the array (orders up to about 780 for the full BSE fit).  Calls on one GPU
 * share the array: calls that overlap in time on one GPU race and give
 * undefined results; order them on one stream. */
#define BSE_NOALLOC_SCRATCH_BYTES (32u << 20)
bse_status bse_solve_noalloc(const bse_desc* desc, void* H0, void* H1, double* E, void* XpY,
                             void* XmY, int64_t ldx, const void* probe, double* osc,
                             int32_t* info, hipStream_t stream);

/* The exchange term's Coulomb potential without its macroscopic part (Sec.
 * 4.2, eq. vbar_def), as bse_inputs.vbar takes it:
 *   vbar[G] = 4 pi / |G + q|^2 for every G except G_Q, where vbar[G_Q] = 0;
 * G_Q is the G nearest to the momentum transfer Q (the lowest index among
 * equally near ones) and q = Q - G_Q.  gvec: DEVICE int32 [ng][3], the G
 * vectors in units of 2 pi / alat (bohr); Q: HOST double[3] in bohr^-1 (not
 * kept after return); vbar: DEVICE double[ng] (output); gq: DEVICE int32[1],
 * receives the index of G_Q (for bse_probe).  One kernel on `stream`.
 * BSE_ERR_ARG for ng <= 0, a null pointer, alat <= 0 or a non-finite alat or Q. */
bse_status bse_coulomb(int32_t ng, const int32_t* gvec, double alat, const double* Q,
                       double* vbar, int32_t* gq, hipStream_t stream);

/* Probe vector of the spectrum (Sec. 4.4, eq. osci): probe[a] = conj(Mcv[a][gq[0]])
 * for a = 0..n-1, Mcv complex [n][ng] row-major (the layout bse_inputs.Mcv has),
 * gq: DEVICE int32[1] (as bse_coulomb writes it; 0 <= gq < ng is the caller's
 * to ensure).  probe: DEVICE complex [n] (output).  BSE_ERR_ARG for n <= 0,
 * ng <= 0 or a null pointer. */
bse_status bse_probe(int64_t n, int32_t ng, const void* Mcv, const int32_t* gq, void* probe,
                     hipStream_t stream);

/* Oscillator strengths from eigenvectors: osc[l] = |sum_a conj(XpY[a,l]) probe[a]|^2
 * (eq. osci without the 1/V_c factor, which the prefactor of bse_spectrum carries). */
bse_status bse_oscillator(int64_t n, const void* XpY, int64_t ldx, const void* probe, double* osc,
                          hipStream_t stream);

/* Macroscopic dielectric function on a frequency grid (Sec. 4.4, eq. chir
 * inserted in eps_M = 1 - v Pbar):
 *   eps[j] = 1 - pref * sum_l osc[l] [1/(w_j - E_l + i eta) - 1/(w_j + E_l + i eta)]
 * E, osc: [n]; omega: [nw]; eps: complex [nw] (output).  pref = 2 kappa v(Q)
 * (spin factor 2), eta = half width of the Lorentzian broadening. */
bse_status bse_spectrum(int64_t n, const double* E, const double* osc, double pref, double eta,
                        int64_t nw, const double* omega, void* eps, hipStream_t stream);

/* Transition coefficients along several directions (Sec. 4.4, eq. tlambdai):
 *   t[l + i ldt] = -i sum_a conj(XpY[a, l]) probe[a + i ldp],  l < n, i < nprobe
 * With probe column i = conj(D_{., i}), D the dipole elements of eq.
 * dipolfromp (the D~ of eq. tlambdai), t_{l,i} is the paper's coefficient for
 * Cartesian direction i.  nprobe: 1..4.  XpY: complex n x n, column-major,
 * ldx >= n (from bse_solve); probe: complex n x nprobe, ldp >= n; t: complex
 * n x nprobe (output), ldt >= n.  Device pointers owned by the caller.
 * BSE_ERR_ARG for a non-positive size, a short leading dimension or a NULL
 * pointer. */
bse_status bse_transitions(int64_t n, const void* XpY, int64_t ldx, int32_t nprobe,
                           const void* probe, int64_t ldp, void* t, int64_t ldt,
                           hipStream_t stream);

/* Macroscopic dielectric tensor in the optical limit (Sec. 4.4, eq. epsmij):
 *   eps[(j nd + a) nd + b] = delta_ab - pref sum_l conj(t_la) t_lb
 *                            [1/(w_j - E_l + i eta) - 1/(w_j + E_l + i eta)]
 * nd: 1..3 directions; E: [n] (bse_solve); t: complex n x nd (bse_transitions),
 * ldt >= n; omega: [nw]; eps: complex [nw][nd][nd] (output).  pref = 8 pi kappa
 * (spin factor 2, 1/V_c, and the 4 pi left of v(q) once M = i q.D cancels its
 * 1/q^2, eq. mofd); eta > 0 is the half width.  Contracting eps with a unit
 * direction q gives the scalar eps_M of that direction (eq. epsmtensor).
 * BSE_ERR_ARG for bad sizes, NULL pointers, eta <= 0 or a non-finite pref. */
bse_status bse_dielectric_tensor(int64_t n, const double* E, int32_t nd, const void* t,
                                 int64_t ldt, double pref, double eta, int64_t nw,
                                 const double* omega, void* eps, hipStream_t stream);

/* Electron energy-loss function and dynamic structure factor (Sec. 4.4, eq.
 * Lofeps and the definition of S(Q, w) beside it):
 *   loss[j] = -Im 1/eps[j inc],   sqw[j] = loss[j] vinv / pi
 * eps: complex, element j at index j * inc (inc = 1 for bse_spectrum's output;
 * inc = nd * nd, with the pointer moved to element (a, a) of the first
 * frequency, for a diagonal element of bse_dielectric_tensor's output); vinv = 1 / v_G(q) > 0; loss: [nw] (output); sqw: [nw] (output)
 * or NULL (then vinv is not used).  BSE_ERR_ARG for nw <= 0, inc < 1, NULL
 * eps or loss, or a bad vinv with sqw given. */
bse_status bse_loss(int64_t nw, const void* eps, int64_t inc, double vinv, double* loss,
                    double* sqw, hipStream_t stream);

/* ---- Pair elements from orbitals (Sec. 4.1: plane-wave matrix elements
 * between Bloch states, here with orbitals expanded in plane waves only,
 * phi_n,k(r) = Omega^-1/2 sum_K C_n,k(K) exp(i (k + K) r); the cell integral
 * keeps the plane waves whose wave vectors cancel):
 *   M_mn(k, k', G) = sum_K conj(C_m,k(K)) C_n,k'(K + G)        (q = k' - k)
 *   N_mn(k, k', G) = sum_K conj(C_m,k(K)) conj(C_n,k'(-K - G)) (q = -k - k')
 * For every pair p = (ik <= ik') the call forms the bse_inputs arrays
 *   Mvv[p][v][v'][G] = M_vv'(k, k', G),  Mcc[p][c][c'][G] = M_cc'(k, k', G)
 *   Ncv[p][c][v'][G] = N_cv'(k, k', G),  Nvc[p][v][c'][G] = N_vc'(k, k', G)
 *   Mcv[(k nv + v) nc + c][G] = M_vc(k, k, G)        (momentum transfer Q = 0)
 * (band index v < nv occupied, c the c-th unoccupied band, nv + c in C). */
typedef struct {
  int32_t nk, nv, nc, ng; /* k-points, occupied and unoccupied bands, plane waves G */
  int32_t nkb;            /* plane waves K of each orbital (the sphere) */
  int32_t coupling;       /* bse_coupling: BSE_FULL forms Ncv and Nvc too */
} bse_orb_desc;

/* C: complex [nk][nv + nc][nkb] orbital coefficients (occupied bands first);
 * kpg, mkg: int32 [nkb][ng], position in the sphere of K + G and of -K - G
 * (-1 when outside; mkg may be NULL in the TDA); outputs: device arrays in the
 * layouts of bse_inputs (Ncv, Nvc may be NULL in the TDA).  BSE_ERR_ARG for
 * a bad descriptor, a NULL pointer, or 2 (nv + nc) nkb coefficients beyond
 * 160 KB of LDS. */
bse_status bse_pair_elements(const bse_orb_desc* desc, const void* C, const int32_t* kpg,
                             const int32_t* mkg, void* Mcv, void* Mvv, void* Mcc, void* Ncv,
                             void* Nvc, hipStream_t stream);

/* ---- Static RPA screening (Sec. 4.2: the RPA dielectric matrix at w = 0 and
 * the screened interaction w_GG'(q) = v_G(q) eps^-1_GG'(q), eq. wggq), the
 * W(q) input of bse_build.  An insulator at zero temperature: f = 1 in the nv
 * occupied and 0 in the nc unoccupied bands, so the sum over band pairs runs
 * over (occupied at k, unoccupied at k+q) and (unoccupied at k, occupied at
 * k+q), each with weight 1/|e_j,k+q - e_i,k| (in 1/Hartree). */
typedef struct {
  int32_t nk;                /* k-points of the mesh; W is formed for every q of it */
  int32_t nv, nc;            /* occupied and unoccupied bands */
  int32_t ng;                /* plane waves G (1..512) */
  double inv_vc;             /* 1/V_c = 1/(N_k Omega), bohr^-3 */
  double units_per_hartree;  /* energy units per Hartree: 27.211386245988 for eV */
} bse_screen_desc;

/* Bytes of scratch space `ws` needed by bse_screening (the pair weights);
 * 0 for an invalid descriptor. */
size_t bse_screening_workspace_size(const bse_screen_desc* desc);

/* W[q][G][G'] (complex, row-major, the layout bse_inputs.W takes) for every q:
 *   W = v^1/2 (I + v^1/2 Xt v^1/2)^-1 v^1/2,
 *   Xt[G,G'] = inv_vc sum_{k, pairs} |F| conj(M(G)) M(G')
 * which equals v_G eps^-1_GG' for eps_GG' = delta_GG' - v_G' X_GG', X = -Xt.
 *  eps_v: [nk][nv], eps_c: [nk][nc] band energies (in the units of the desc);
 *  kqmap: int32 [q][k], the mesh index of k + q;
 *  Svc: complex [q][k][nv][nc][ng], elements between occupied band v at k
 *       and unoccupied band c at k+q;
 *  Scv: complex [q][k][nc][nv][ng], unoccupied c at k and occupied v at k+q;
 *  vsqrt: [q][ng], v(q+G)^1/2 (the caller's Coulomb potential, regularised
 *       where q+G = 0);
 *  W: complex [q][ng][ng] (output).
 * Errors on the device: info = -5 when an occupied band is not below an
 * unoccupied one (no gap), -6 when a pivot of the inversion is not positive.
 * BSE_ERR_ARG for a bad descriptor or a NULL pointer, BSE_ERR_WORKSPACE when
 * ws_bytes is short. */
bse_status bse_screening(const bse_screen_desc* desc, const double* eps_v, const double* eps_c,
                         const int32_t* kqmap, const void* Svc, const void* Scv,
                         const double* vsqrt, void* W, void* ws, size_t ws_bytes, int32_t* info,
                         hipStream_t stream);

/* ---- Batches of independent problems (one per momentum transfer Q; the BSE
 * decouples per q, Sec. 2.3 eq. chimatrixq).  The whole pipeline of every
 * problem (bse_build, the spectrum path of bse_solve, bse_spectrum) is
 * recorded once into a HIP graph and replayed with one graph launch.
 * Problems run on `nbranch` concurrent branches (streams the batch creates
 * at default priority), largest N^3 first, each branch with its own slice of
 * the workspace.  With one branch per problem (nbranch >= nprob) the Cholesky
 * factorisations (Sec. 4.3) and the Householder sweeps of all problems run
 * batched on the capture stream, each launch serving every problem (up to 16
 * per launch), between per-problem stages on the branches; each problem's
 * results are bitwise those of the plain entry points (with the default
 * BSE_TUNE_BATCH_SWEEP choice).  The workspace then also holds a small table
 * (the sweep's grid counts, 4 bytes per unit of problem order, after the
 * branch slices), which bse_batch_capture fills with a blocking host-to-device
 * copy: no replay of the batch may be running during a capture.  All pointers given to bse_batch_capture stay
 * baked into the graph: they must stay valid until bse_batch_destroy.  `info`
 * holds one int32 per problem and is cleared at the start of every replay.
 * Capture needs a created stream (not the NULL stream). */
typedef struct bse_batch* bse_batch_t;

size_t bse_batch_workspace_size(int32_t nprob, const bse_desc* descs, int32_t nbranch);
bse_status bse_batch_create(int32_t nprob, const bse_desc* descs, int32_t nbranch,
                            bse_batch_t* out);
/* Per-problem arrays of length nprob: inputs, H0, H1 (full only), E, probe,
 * osc, pref, eta, nw, omega, eps -- the arguments of bse_build / bse_solve /
 * bse_spectrum for that problem (device pointers; pref/eta/nw host values). */
bse_status bse_batch_capture(bse_batch_t batch, const bse_inputs* inputs, void* const* H0,
                             void* const* H1, double* const* E, const void* const* probe,
                             double* const* osc, const double* pref, const double* eta,
                             const int64_t* nw, const double* const* omega, void* const* eps,
                             void* ws, size_t ws_bytes, int32_t* info, hipStream_t stream);
bse_status bse_batch_run(bse_batch_t batch, hipStream_t stream);
void bse_batch_destroy(bse_batch_t batch);

/* Measurement hook: while enabled (on != 0), every kernel launch of the
 * library (or, when `name` is not NULL, every launch of the kernel with that
 * name) is bracketed by two HIP events recorded on the launch stream.  Kernel
 * names carry no template arguments: the instances of one kernel template are
 * timed and reported together.
 * bse_timing_report synchronises on those events, writes one line per kernel
 * name "<name> <launches> <total milliseconds>" into the HOST buffer `buf`
 * (truncated to len-1 bytes, NUL-terminated), clears the records and returns
 * the full length of the report.  With buf == NULL it only returns the length
 * and keeps the records. */
void bse_timing_enable(int32_t on, const char* name);
int64_t bse_timing_report(char* buf, int64_t len);

/* Tuning table: the output of the project's autotuner
 * (paper_1904_05575_amd/tune.py, run on the GPU).  Each entry selects, for one
 * call site and for sizes up to size_max, a tile choice:
 *   BSE_TUNE_HEMV_UNIT     size = trailing order m of a Householder step;
 *                          choice = least number of 64 x 64 tiles per block of
 *                          the Hermitian matrix-vector kernel (blocks take equal
 *                          runs of tiles, at most one per compute unit): 1, 2,
 *                          4 or 8
 *   BSE_TUNE_GEMM_*        size = problem order n; choice = GEMM tile edge
 *                          16, 32 or 64 (squared form S = U (A+B) U^H; Cholesky
 *                          trailing updates; Householder panel updates; the
 *                          second contraction of the direct terms; exchange)
 *   BSE_TUNE_DIRECT        size = problem order n; choice = how the FP64 (and
 *                          FP32) direct terms with stored pair elements and
 *                          N_G <= 128 run: 0 two passes (T = conj(M) W(q) to
 *                          memory on the real view, then a batched product
 *                          per pair and a scatter); 1, 2, 3 one fused pass per
 *                          term (T kept on chip) with 16, 8 or 8 wavefronts per
 *                          block of 64 rows (wavefront tiles 16 x 32, 16 x 64,
 *                          32 x 32), the first product in three real products
 *                          per complex one; 4, 5, 6 that first product (same
 *                          three shapes) writing T, then the two-pass rest;
 *                          7, 8 the first product with N_G unpadded (up to
 *                          3 trailing columns and k on the vector ALU; 64
 *                          rows per block on 4 wavefronts; operands through
 *                          registers or copied straight into LDS) writing T,
 *                          then the two-pass rest (FP64, N_G <= 113; else 4);
 *                          9 (default) one pass per term with both products
 *                          on the matrix cores (FP64, N_G <= 113, 9 <= R <= 16
 *                          rows and at most 16 columns per pair block; else 7)
 *   BSE_TUNE_GEMM_PRODUCTS size = the larger output dimension of a complex GEMM;
 *                          choice = real matrix-core products per complex one
 *                          on 16- and 32-edge tiles: 4 (re = ar br - ai bi,
 *                          im = ar bi + ai br) or 3 (Gauss: ar br, ai bi,
 *                          (ar + ai)(br + bi)); 64-edge tiles always take 4
 *   BSE_TUNE_BATCH_SWEEP   size = largest problem order of a batch; choice =
 *                          blocks of the batched Householder sweep's hemv
 *                          launches: 0 (default) each problem takes the blocks
 *                          it takes on its own (results bitwise equal to the
 *                          single problem path); 1, 2 or 4 that many blocks per
 *                          compute unit in total, shared among the problems in
 *                          proportion to their tiles
 *   BSE_TUNE_GEMM_VECTORS  size = problem order n; choice = GEMM tile edge
 *                          16, 32 or 64 of the eigenvector path's products:
 *                          the back-transform (W = V^H Z, Z -= V Y), X+Y =
 *                          U^H Z and the updates of the triangular solve for
 *                          X-Y (default 32 where no entry applies)
 *   BSE_TUNE_GEMM_SQUARED_S size = problem order n; choice = GEMM tile edge
 *                          16, 32 or 64 of the squared form's second product
 *                          (S = U T1, lower triangle); where no entry applies,
 *                          that of BSE_TUNE_GEMM_SQUARED, which then sets the
 *                          first product T1 = (A+B) U^H
 *   BSE_TUNE_BATCH_ALIGN   size = largest problem order of a batch; choice =
 *                          when each problem's batched Householder sweep
 *                          starts: 0 (default) all at the first step; 1 late
 *                          by the largest multiple of the panel width that
 *                          keeps it within the largest problem's steps, so that
 *                          the sweeps end together (every problem's values
 *                          unchanged)
 * Among the entries of a site, the one with the smallest size_max >= size
 * applies; sizes no entry covers use built-in rules.  Every choice gives the
 * same results up to rounding order.  The table is read on the host when work
 * is enqueued (a captured graph keeps the choices of its capture).
 * bse_tune_set copies `count` entries from HOST memory (count 0 clears the
 * table; BSE_ERR_ARG for an unknown site or choice, nothing changed).
 * bse_tune_get copies at most `cap` entries into HOST memory `out` (may be
 * NULL) and returns the number in the table. */
enum {
  BSE_TUNE_HEMV_UNIT = 0,
  BSE_TUNE_GEMM_SQUARED = 1,
  BSE_TUNE_GEMM_POTRF = 2,
  BSE_TUNE_GEMM_HER2K = 3,
  BSE_TUNE_GEMM_STAGE2 = 4,
  BSE_TUNE_GEMM_EXCHANGE = 5,
  BSE_TUNE_DIRECT = 6,
  BSE_TUNE_GEMM_PRODUCTS = 7,
  BSE_TUNE_BATCH_SWEEP = 8,
  BSE_TUNE_GEMM_VECTORS = 9,
  BSE_TUNE_BATCH_ALIGN = 10,
  BSE_TUNE_GEMM_SQUARED_S = 11
};
typedef struct {
  int32_t site;
  int32_t size_max;
  int32_t choice;
  int32_t reserved;
} bse_tune_entry;
bse_status bse_tune_set(const bse_tune_entry* entries, int32_t count);
int32_t bse_tune_get(bse_tune_entry* out, int32_t cap);

/* Human-readable name of a status. */
const char* bse_status_string(bse_status status);

#ifdef __cplusplus
}
#endif
#endif /* BSE_H */
