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
