// Event-based kernel timing registry (see timing.h).
#include "timing.h"

#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bse_internal.h"

namespace {
struct Rec {
  std::string name;  // kernel name without template arguments
  hipEvent_t a, b;
};
std::mutex mu;
bool enabled = false;
std::string only;  // when non-empty, only launches with this name are timed
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;

hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool timing_on() { return enabled; }

TimingState timing_suspend() {
  std::lock_guard<std::mutex> g(mu);
  TimingState st{enabled, only};
  enabled = false;
  return st;
}

void timing_resume(const TimingState& st) {
  std::lock_guard<std::mutex> g(mu);
  enabled = st.on;
  only = st.only;
}

namespace {
thread_local char fail_msg[256];
}

void launch_check(const char* name) {
  const hipError_t e = hipPeekAtLastError();
  if (e != hipSuccess && fail_msg[0] == 0)
    snprintf(fail_msg, sizeof fail_msg, "HIP launch failed after %s: %s", name,
             hipGetErrorString(e));
}
void launch_failure_reset() {
  fail_msg[0] = 0;
  (void)hipGetLastError();  // an error left by other code is not this call's
}
const char* launch_failure() { return fail_msg[0] ? fail_msg : nullptr; }

void timing_begin(const char* name, hipEvent_t* a, hipEvent_t* b) {
  std::lock_guard<std::mutex> g(mu);
  while (*name == '(') ++name;  // launch macros may parenthesise template names
  std::string base(name, strcspn(name, "<"));
  *a = *b = nullptr;
  if (!only.empty() && only != base) {
    recs.push_back(Rec{std::move(base), nullptr, nullptr});
    return;
  }
  Rec r{std::move(base), get_event(), get_event()};
  if (r.a && r.b) {
    *a = r.a;
    *b = r.b;
  }
  recs.push_back(r);
}

extern "C" {

void bse_timing_enable(int32_t on, const char* name) {
  std::lock_guard<std::mutex> g(mu);
  enabled = on != 0;
  only = name ? name : "";
}

int64_t bse_timing_report(char* buf, int64_t len) {
  std::lock_guard<std::mutex> g(mu);
  std::map<std::string, std::pair<long, double>> acc;
  for (auto& r : recs) {
    float ms = 0.0f;
    if (r.a && r.b && hipEventSynchronize(r.b) == hipSuccess &&
        hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& e = acc[r.name];
      e.first += 1;
      e.second += ms;
    }
  }
  std::string out;
  char line[256];
  for (auto& kv : acc) {
    snprintf(line, sizeof(line), "%s %ld %.6f\n", kv.first.c_str(), kv.second.first,
             kv.second.second);
    out += line;
  }
  if (buf && len > 0) {
    const int64_t n = (int64_t)out.size() < len - 1 ? (int64_t)out.size() : len - 1;
    memcpy(buf, out.data(), (size_t)n);
    buf[n] = 0;
    // a report written into a buffer consumes the records
    for (auto& r : recs) {
      if (r.a) pool.push_back(r.a);
      if (r.b) pool.push_back(r.b);
    }
    recs.clear();
  }
  return (int64_t)out.size();
}

}  // extern "C"
