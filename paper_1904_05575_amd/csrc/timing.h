// Opt-in per-kernel timing with HIP events recorded on the launch stream.
// Disabled by default; when enabled every instrumented launch is bracketed
// by two events and bse_timing_report() sums their elapsed times by name.
#pragma once
#include <hip/hip_runtime.h>

bool timing_on();
void timing_begin(const char* name, hipStream_t s);
void timing_end(hipStream_t s);

struct TimedLaunch {
  hipStream_t s;
  bool on;
  TimedLaunch(const char* name, hipStream_t st) : s(st), on(timing_on()) {
    if (on) timing_begin(name, s);
  }
  ~TimedLaunch() {
    if (on) timing_end(s);
  }
};

#define BSE_LAUNCH(kern, grid, block, shmem, stream, ...)            \
  do {                                                               \
    TimedLaunch _tl(#kern, stream);                                  \
    hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__); \
  } while (0)
