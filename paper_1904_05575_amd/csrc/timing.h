// Opt-in per-kernel timing with HIP events on the launch stream.  Disabled by
// default.  When enabled, instrumented launches go through hipExtLaunchKernel
// with a start and a stop event, which the runtime stamps at the kernel's own
// start and end (no separate event packets around it); bse_timing_report()
// sums the elapsed times by kernel name.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <string>

bool timing_on();
// Timing switched off for a stretch of work (graph capture records no
// events) and switched back on afterwards with the same kernel-name filter.
struct TimingState {
  bool on = false;
  std::string only;
};
TimingState timing_suspend();
void timing_resume(const TimingState& st);
// Registers a launch of `name`; *a / *b receive the events to launch with, or
// nullptr when this launch is not timed.
void timing_begin(const char* name, hipEvent_t* a, hipEvent_t* b);

struct TimedLaunch {
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(const char* name, hipStream_t) {
    if (timing_on()) timing_begin(name, &a, &b);
  }
};

// Launch failures: the first kernel after which the runtime reports an error
// is remembered (per thread) until the next public call starts, so that the
// status string can name it.
void launch_check(const char* name);
void launch_failure_reset();
const char* launch_failure();

#define BSE_LAUNCH(kern, grid, block, shmem, stream, ...)                                 \
  do {                                                                                    \
    TimedLaunch _tl(#kern, stream);                                                       \
    if (_tl.a)                                                                            \
      hipExtLaunchKernelGGL(kern, grid, block, shmem, stream, _tl.a, _tl.b, 0, __VA_ARGS__); \
    else                                                                                  \
      hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);                  \
    launch_check(#kern);                                                                  \
  } while (0)
