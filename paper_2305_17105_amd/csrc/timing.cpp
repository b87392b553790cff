// Optional per-kernel timing for measurement: while enabled, HIP events are recorded
// on the launch stream around every launch of the timed kernels.  Off by default; the
// hot path pays one relaxed flag test per launch.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <mutex>
#include <vector>

#include "ntc_internal.h"

namespace ntc {

namespace {
struct Timer {
  std::mutex mu;
  std::atomic<bool> on{false};
  int cap = 0;
  std::vector<hipEvent_t> start[TK_COUNT], stop[TK_COUNT];
  int used[TK_COUNT] = {0};
};
Timer& timer() {
  static Timer t;
  return t;
}
const char* kNames[TK_COUNT] = {"train_fused", "decode"};

void destroy_events(Timer& t) {
  for (int k = 0; k < TK_COUNT; ++k) {
    for (auto e : t.start[k]) (void)hipEventDestroy(e);
    for (auto e : t.stop[k]) (void)hipEventDestroy(e);
    t.start[k].clear();
    t.stop[k].clear();
    t.used[k] = 0;
  }
}
}  // namespace

int timing_before(TimedKernel k, hipStream_t s) {
  Timer& t = timer();
  if (!t.on.load(std::memory_order_relaxed)) return -1;
  std::lock_guard<std::mutex> lock(t.mu);
  if (!t.on || t.used[k] >= t.cap) return -1;
  const int i = t.used[k]++;
  (void)hipEventRecord(t.start[k][i], s);
  return i;
}

void timing_after(TimedKernel k, hipStream_t s, int slot) {
  if (slot < 0) return;
  Timer& t = timer();
  std::lock_guard<std::mutex> lock(t.mu);
  if (t.on && slot < (int)t.stop[k].size()) (void)hipEventRecord(t.stop[k][slot], s);
}

}  // namespace ntc

using namespace ntc;

extern "C" ntc_status ntc_timing_begin(int32_t max_launches) {
  if (max_launches < 1 || max_launches > (1 << 20)) {
    set_error("ntc_timing_begin: max_launches must be in 1 .. 2^20");
    return NTC_E_INVALID;
  }
  Timer& t = timer();
  std::lock_guard<std::mutex> lock(t.mu);
  destroy_events(t);
  t.cap = max_launches;
  for (int k = 0; k < TK_COUNT; ++k) {
    t.start[k].resize(max_launches);
    t.stop[k].resize(max_launches);
    for (int i = 0; i < max_launches; ++i) {
      if (hipEventCreate(&t.start[k][i]) != hipSuccess || hipEventCreate(&t.stop[k][i]) != hipSuccess) {
        t.start[k].resize(i);
        t.stop[k].resize(i);
        destroy_events(t);
        set_error("ntc_timing_begin: hipEventCreate failed");
        return NTC_E_HIP;
      }
    }
  }
  t.on = true;
  return NTC_OK;
}

extern "C" ntc_status ntc_timing_read(const char* kernel, double* total_ms, int32_t* launches) {
  if (!kernel || !total_ms || !launches) {
    set_error("ntc_timing_read: NULL argument");
    return NTC_E_INVALID;
  }
  int k = -1;
  for (int i = 0; i < TK_COUNT; ++i)
    if (std::strcmp(kernel, kNames[i]) == 0) k = i;
  if (k < 0) {
    set_error("ntc_timing_read: unknown kernel name");
    return NTC_E_INVALID;
  }
  Timer& t = timer();
  std::lock_guard<std::mutex> lock(t.mu);
  double sum = 0.0;
  for (int i = 0; i < t.used[k]; ++i) {
    float ms = 0.f;
    if (hipEventSynchronize(t.stop[k][i]) != hipSuccess ||
        hipEventElapsedTime(&ms, t.start[k][i], t.stop[k][i]) != hipSuccess) {
      set_error("ntc_timing_read: event query failed");
      return NTC_E_HIP;
    }
    sum += ms;
  }
  *total_ms = sum;
  *launches = t.used[k];
  return NTC_OK;
}

extern "C" ntc_status ntc_timing_end(void) {
  Timer& t = timer();
  std::lock_guard<std::mutex> lock(t.mu);
  t.on = false;
  (void)hipDeviceSynchronize();
  destroy_events(t);
  return NTC_OK;
}
