// Shared device helpers of the BSE library (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4 __attribute__((ext_vector_type(4)));

#define BSE_DEV __device__ __forceinline__

struct cplx {
  double re, im;
};

BSE_DEV double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
BSE_DEV double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
BSE_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
BSE_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
BSE_DEV double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
BSE_DEV double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
BSE_DEV double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// 64-lane wavefront sum (deterministic butterfly order).
BSE_DEV double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
BSE_DEV double2 wave_sum2(double2 v) {
  return make_double2(wave_sum(v.x), wave_sum(v.y));
}

// Block-wide sum of one double; every thread gets the result.  `sh` needs
// blockDim.x / 64 doubles of shared memory.  Deterministic.
BSE_DEV double block_sum(double v, double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  return s;
}

// Device status word shared by every kernel of one call sequence: kernels
// return at entry when an earlier kernel recorded a failure.
BSE_DEV bool failed(const int32_t* info) { return info != nullptr && *(volatile const int32_t*)info != 0; }

// Record the first failure (0 -> code); later failures keep the first code.
BSE_DEV void set_info(int32_t* info, int32_t code) {
  if (info) atomicCAS(info, 0, code);
}

__host__ __device__ static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
