// Driver for hardware-counter runs of the Householder sweep at a given order
// (the counter runs of rocprofv3 do not start under the Python benchmark).
//
// It launches one plain copy kernel of known size, whose FETCH_SIZE and
// WRITE_SIZE calibrate the counters, then one bse_solve of a Hermitian matrix
// of order n in TDA form on the spectrum path (probe carried through the
// reduction, no eigenvectors).  The tridiagonalisation kernels, their grids
// and the bytes they move depend only on n, not on the matrix values or on
// how the matrix was assembled.
//
//   usage: trd_counters [n = 6144]
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../include/bse.h"

#define CHECK(x)                                                               \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                  \
      return 1;                                                                \
    }                                                                          \
  } while (0)

constexpr int64_t COPY_BYTES = 1ll << 30;  // read once and written once by k_copy

__global__ __launch_bounds__(256) void k_copy(const double2* __restrict__ a,
                                              double2* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// a deterministic Hermitian test matrix (column-major): distinct real diagonal,
// off-diagonal values from an integer hash, mirrored
__device__ double hval(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return (double)x * 0x1p-32 - 0.5;
}
__global__ __launch_bounds__(256) void k_fill(double2* __restrict__ A, int64_t n) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % n, j = e / n;
    const int64_t lo = i > j ? i : j, hi = i > j ? j : i;
    const uint32_t key = (uint32_t)(lo * 2654435761u + hi);
    double2 v = make_double2(hval(2 * key), (i == j) ? 0.0 : hval(2 * key + 1));
    if (i < j) v.y = -v.y;
    if (i == j) v.x = (double)i / (double)n;
    A[e] = v;
  }
}
__global__ void k_probe(double2* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = make_double2(1.0 / (1.0 + (double)i), 0.5);
}

int main(int argc, char** argv) {
  const int64_t n = argc > 1 ? atoll(argv[1]) : 6144;
  if (n < 2 || n > 40000) {
    fprintf(stderr, "order out of range\n");
    return 2;
  }
  bse_desc d = {};
  d.nk = 1;
  d.nv = 1;
  d.nc = (int32_t)n;
  d.ng = 1;
  d.coupling = BSE_TDA;
  d.type = BSE_SINGLET;
  d.prec = BSE_PREC_FP64;
  d.ld = n;
  const size_t wsb = bse_workspace_size(&d, BSE_STAGE_SOLVE);
  if (wsb == 0) {
    fprintf(stderr, "bad descriptor\n");
    return 2;
  }
  double2 *A, *probe, *src, *dst;
  double *E, *osc;
  void* ws;
  int32_t* info;
  CHECK(hipMalloc(&A, sizeof(double2) * n * n));
  CHECK(hipMalloc(&probe, sizeof(double2) * n));
  CHECK(hipMalloc(&E, sizeof(double) * n));
  CHECK(hipMalloc(&osc, sizeof(double) * n));
  CHECK(hipMalloc(&ws, wsb));
  CHECK(hipMalloc(&info, sizeof(int32_t)));
  CHECK(hipMalloc(&src, COPY_BYTES));
  CHECK(hipMalloc(&dst, COPY_BYTES));
  CHECK(hipMemset(info, 0, sizeof(int32_t)));
  CHECK(hipMemset(src, 0, COPY_BYTES));
  hipLaunchKernelGGL(k_fill, dim3(4096), dim3(256), 0, 0, A, n);
  hipLaunchKernelGGL(k_probe, dim3(64), dim3(256), 0, 0, probe, n);
  hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, 0, src, dst,
                     COPY_BYTES / (int64_t)sizeof(double2));
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  const bse_status st = bse_solve(&d, A, nullptr, E, nullptr, n, probe, osc, ws, wsb, info,
                                  nullptr);
  if (st != BSE_OK) {
    fprintf(stderr, "bse_solve: %s\n", bse_status_string(st));
    return 1;
  }
  CHECK(hipDeviceSynchronize());
  int32_t hinfo = 0;
  double e0 = 0.0, e1 = 0.0;
  CHECK(hipMemcpy(&hinfo, info, sizeof hinfo, hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(&e0, E, sizeof e0, hipMemcpyDeviceToHost));
  CHECK(hipMemcpy(&e1, E + n - 1, sizeof e1, hipMemcpyDeviceToHost));
  printf("n=%lld info=%d E[0]=%.12f E[n-1]=%.12f copy_bytes=%lld\n", (long long)n, hinfo, e0, e1,
         (long long)COPY_BYTES);
  return hinfo == 0 ? 0 : 1;
}
