// Internal interface between the eigensolver's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

constexpr int TRD_NB = 32;  // Householder panel width

// Small shared state of the tridiagonalisation kernels (complex slots):
//   [0] scal = 1/(alpha_x - beta) of the current reflector, [1] tau,
//   [2] S[b0][b0], the first diagonal element of the trailing matrix the
//       current reflector multiplies (b0 = c + 1),
//   [3] v^H y_probe of the current reflector,
//   [4, 4 + TRD_NB) V^H v and [4 + TRD_NB, 4 + 2 TRD_NB) W^H v over the panel
constexpr int HS_SCAL = 0, HS_TAU = 1, HS_S00 = 2, HS_PDOT = 3, HS_SVV = 4, HS_SWV = 4 + TRD_NB,
              HS_SIZE = 4 + 2 * TRD_NB;

struct TrdBufs {
  double2* VW;      // n x 2*TRD_NB, [V | W] of the current panel (column-major, ld n)
  double2* WV;      // n x 2*TRD_NB, [W | V]
  double2* ybuf;    // n (unused by the lower-triangle sweep)
  double2* hs;      // HS_SIZE
  double2* part;    // trd_part_elems(n)
  double* dd;       // n   diagonal of T
  double* ee;       // n-1 off-diagonal of T
  double2* tau;     // n-1 reflector scalars
  double2* yproj;   // optional: vector y, replaced by Q^H y
};

int64_t trd_part_elems(int64_t n);
bool tridiagonalise(double2* M, int64_t n, int64_t ld, const TrdBufs& w, int32_t* info,
                    hipStream_t s);

// One problem of a batched sweep: its matrix, order, leading dimension,
// buffers and status word (each problem has its own; none may alias another's).
struct TrdItem {
  double2* M;
  int64_t n, ld;
  TrdBufs w;
  int32_t* info;
};

// Per-problem arguments of the batched kernels (grids[c] = blocks of the hemv
// launch for reflector c, in device memory written by trd_batch_table; shift =
// the global panel step, a multiple of TRD_NB, at which this problem's sweep
// starts: column c of the problem is reduced at global column shift + c).  They
// travel by value in the kernel arguments, up to TRD_BATCH_MAX problems per
// launch, so that the compiler knows every pointer to be device memory.
struct TrdProb {
  double2* M;
  int64_t ld;
  int n, ycs;
  double2 *VW, *WV, *hs, *Y, *partA, *partB, *yp, *tau;
  double *dd, *ee;
  const int32_t* grids;
  int shift;
};
constexpr int TRD_BATCH_MAX = 16;
struct TrdBatchArgs {
  TrdProb p[TRD_BATCH_MAX];
};
// A batched launch's blocks, problem after problem: problem p owns blocks
// [b[p], b[p+1]); entries past the group's last problem equal the total, so a
// problem with nothing to do at a step owns no block.
struct TrdFirst {
  int32_t b[TRD_BATCH_MAX + 1];
};

// Bytes of the device table (the hemv grid counts of every step) for problems
// of orders n[0..np-1].
size_t trd_batch_table_bytes(const int64_t* n, int np);
// Fill the table `dev` (trd_batch_table_bytes long) for these problems: a
// blocking host-to-device copy, made before the sweep is enqueued or captured.
bool trd_batch_table(const TrdItem* it, int np, void* dev, size_t bytes);
// The sweep of every problem at once (in groups of up to TRD_BATCH_MAX): per
// column step one column-kernel launch and one hemv launch serve all problems
// of a group still reducing.  With the per-problem grid choice each problem's
// values are those of tridiagonalise() on its own; with blocks shared among the
// problems they differ from those in rounding order only.
bool tridiagonalise_batch(const TrdItem* it, int np, const void* dev, hipStream_t s);
