// Complex FP64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
//   C(m, n) = alpha * sum_k opA(m, k) opB(k, n) + beta * C(m, n)
//
// Operands are addressed through element strides (complex units), so one
// kernel covers row- and column-major layouts, conjugate transposes and
// batched products.  Triangular operands and triangular outputs skip the
// zero tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct ZgemmParams {
  int M = 0, N = 0, K = 0;
  const double2* A = nullptr;
  int64_t a_rs = 0, a_cs = 0, a_bs = 0;  // A(m,k) = A[b*a_bs + m*a_rs + k*a_cs]
  const double2* B = nullptr;
  int64_t b_rs = 0, b_cs = 0, b_bs = 0;  // B(k,n) = B[bb*b_bs + k*b_rs + n*b_cs]
  double2* C = nullptr;
  int64_t c_rs = 0, c_cs = 0, c_bs = 0;  // C(m,n) = C[b*c_bs + m*c_rs + n*c_cs]
  const int32_t* b_batch_idx = nullptr;  // bb = b_batch_idx[b] (else bb = b)
  double2 alpha = {1.0, 0.0};
  double beta = 0.0;  // beta == 0: C is not read
  int conjA = 0, conjB = 0;
  int c_uplo = 0;  // 0 all; 1 store only m <= n; 2 store only m >= n
  int a_tri = 0;   // 1: A(m,k) = 0 for k < m; 2: A(m,k) = 0 for k > m
  int b_tri = 0;   // 1: B(k,n) = 0 for k > n; 2: B(k,n) = 0 for k < n
  const double* kscale = nullptr;  // A(m,k) *= kscale[b*ks_bs + k]
  int64_t ks_bs = 0;
  const double* ndiv = nullptr;     // C(m,n) = alpha * sum(...) / ndiv[n] (+ beta C)
  const int32_t* info = nullptr;   // skip all work when *info != 0
  const char* tag = "zgemm";        // name under which the launch is timed
  int tile = 0;                     // 16, 32 or 64: tile edge; 0: chosen from the shape
  int products = 0;                 // real MFMA products per complex one on 16- and 32-edge
                                    // tiles: 3 (Gauss) or 4; 0: the tuning table's choice
                                    // (default 3); 64-edge tiles always take 4
};

// Enqueue `batch` products on `stream`.
hipError_t zgemm(const ZgemmParams& p, int batch, hipStream_t stream);

// One product of a group: its own shape, operands, strides and status word.
struct ZgemmItem {
  const double2* A = nullptr;
  const double2* B = nullptr;
  double2* C = nullptr;
  const int32_t* info = nullptr;
  int M = 0, N = 0, K = 0;
  int a_tri = 0, b_tri = 0;  // as in ZgemmParams (the base's are not used)
  int64_t a_rs = 0, a_cs = 0, b_rs = 0, b_cs = 0, c_rs = 0, c_cs = 0;
};
constexpr int ZGEMM_GROUP_MAX = 16;
struct ZgemmGroup {
  ZgemmItem it[ZGEMM_GROUP_MAX];
  // the launch's blocks, item after item: item i owns [first[i], first[i+1])
  // (entries past the last item equal the total)
  int32_t first[ZGEMM_GROUP_MAX + 1];
};
// Enqueue the products `items` (every other parameter from `base`, whose
// shape, operand, stride, triangle and info fields are ignored): each item's values are
// those zgemm(item, 1) gives (same tile edge and products per complex one);
// items that share them run in launches of up to ZGEMM_GROUP_MAX items; items
// with an empty output are skipped.
hipError_t zgemm_group(const ZgemmParams& base, const ZgemmItem* items, int count,
                       hipStream_t stream);
