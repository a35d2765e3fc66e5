// Tuning table: per call site and size bucket, the tile choice found by the
// project's autotuner; the host-side dispatch reads it when work is enqueued.
#include <mutex>
#include <vector>

#include "bse_internal.h"

namespace {
std::mutex mu;
std::vector<bse_tune_entry> table;

bool valid(const bse_tune_entry& e) {
  if (e.size_max <= 0) return false;
  switch (e.site) {
    case BSE_TUNE_HEMV_UNIT:
      return e.choice == 1 || e.choice == 2 || e.choice == 4 || e.choice == 8;
    case BSE_TUNE_GEMM_SQUARED:
    case BSE_TUNE_GEMM_POTRF:
    case BSE_TUNE_GEMM_HER2K:
    case BSE_TUNE_GEMM_STAGE2:
    case BSE_TUNE_GEMM_EXCHANGE:
    case BSE_TUNE_GEMM_VECTORS:
    case BSE_TUNE_GEMM_SQUARED_S:
      return e.choice == 16 || e.choice == 32 || e.choice == 64;
    case BSE_TUNE_DIRECT:
      return e.choice >= 0 && e.choice <= 9;
    case BSE_TUNE_GEMM_PRODUCTS:
      return e.choice == 3 || e.choice == 4;
    case BSE_TUNE_BATCH_SWEEP:
      return e.choice == 0 || e.choice == 1 || e.choice == 2 || e.choice == 4;
    case BSE_TUNE_BATCH_ALIGN:
      return e.choice == 0 || e.choice == 1;
    default:
      return false;
  }
}
}  // namespace

int tune_choice(int site, int64_t size, int deflt) {
  std::lock_guard<std::mutex> g(mu);
  int best = deflt;
  int64_t best_max = -1;
  for (const auto& e : table)
    if (e.site == site && size <= e.size_max && (best_max < 0 || e.size_max < best_max)) {
      best = e.choice;
      best_max = e.size_max;
    }
  return best;
}

extern "C" {

bse_status bse_tune_set(const bse_tune_entry* entries, int32_t count) {
  if (count < 0 || (count > 0 && !entries)) return BSE_ERR_ARG;
  for (int i = 0; i < count; ++i)
    if (!valid(entries[i])) return BSE_ERR_ARG;
  std::lock_guard<std::mutex> g(mu);
  table.assign(entries, entries + count);
  return BSE_OK;
}

int32_t bse_tune_get(bse_tune_entry* out, int32_t cap) {
  std::lock_guard<std::mutex> g(mu);
  const int32_t n = (int32_t)table.size();
  if (out)
    for (int32_t i = 0; i < n && i < cap; ++i) out[i] = table[i];
  return n;
}

}  // extern "C"
