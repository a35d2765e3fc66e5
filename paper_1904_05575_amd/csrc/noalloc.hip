// bse_solve_noalloc: the eigenproblem of bse_solve with its scratch space in
// a fixed device array of the library instead of a caller's workspace, for
// callers that cannot allocate device memory.
//
// The array lives once per GPU for the life of the process.  Its device
// address is looked up once per device (hipGetSymbolAddress, with that
// device current) on the first call made there and kept; the kernels receive
// that address, never the array's host-side name.  Calls on one GPU share the
// array: two calls that overlap in time on one GPU (different streams, or
// different host threads without ordering) race on it.  Everything the solve
// needs zeroed it clears itself on the stream.
#include <mutex>

#include "bse_internal.h"
#include "timing.h"

namespace {

constexpr size_t kScratchBytes = BSE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex mu;
void* scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's array (nullptr on failure).
void* device_scratch(int dev) {
  std::lock_guard<std::mutex> g(mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    scratch_ptr[dev] = p;
  }
  return scratch_ptr[dev];
}

}  // namespace

extern "C" bse_status bse_solve_noalloc(const bse_desc* d, void* H0, void* H1, double* E,
                                        void* XpY, void* XmY, int64_t ldx, const void* probe,
                                        double* osc, int32_t* info, hipStream_t stream) {
  launch_failure_reset();
  if (!d || !H0 || !E || !info) return BSE_ERR_ARG;
  const size_t need = bse_workspace_size(d, BSE_STAGE_SOLVE);
  if (need == 0) return BSE_ERR_ARG;
  if (need > kScratchBytes) return BSE_ERR_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return BSE_ERR_HIP;
  void* ws = device_scratch(dev);
  if (!ws) return BSE_ERR_HIP;
  // the same checks and kernels as bse_solve, with the array as its workspace
  return bse_solve(d, H0, H1, E, XpY, XmY, ldx, probe, osc, ws, need, info, stream);
}
