// Kernel-level instrumentation: HIP events on the launch stream around each
// kernel launch while enabled, read back per kernel id.
#include "dsps_internal.hpp"

#include <atomic>
#include <mutex>
#include <vector>

namespace dsps {

namespace {
struct Record {
  int kid;
  hipEvent_t start, stop;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Record> g_records;
std::vector<hipEvent_t> g_pool;
thread_local int g_quiet = 0;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void recycle_all() {
  for (const Record &r : g_records) {
    g_pool.push_back(r.start);
    g_pool.push_back(r.stop);
  }
  g_records.clear();
}
}  // namespace

ProfQuiet::ProfQuiet() { ++g_quiet; }
ProfQuiet::~ProfQuiet() { --g_quiet; }

ProfScope::ProfScope(int kernel_id, hipStream_t stream) : kid_(kernel_id), stream_(stream) {
  if (g_quiet || !g_on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lock(g_mu);
  start_ = take_event();
  stop_ = take_event();
  if (start_ && stop_ && hipEventRecord(start_, stream_) == hipSuccess) return;
  if (start_) g_pool.push_back(start_);
  if (stop_) g_pool.push_back(stop_);
  start_ = stop_ = nullptr;
}

ProfScope::~ProfScope() {
  if (!start_) return;
  std::lock_guard<std::mutex> lock(g_mu);
  if (hipEventRecord(stop_, stream_) == hipSuccess) {
    g_records.push_back({kid_, start_, stop_});
  } else {
    g_pool.push_back(start_);
    g_pool.push_back(stop_);
  }
}

}  // namespace dsps

using namespace dsps;

extern "C" {

int dsps_profile_enable(int on) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (on) {
    for (const Record &r : g_records) (void)hipEventSynchronize(r.stop);
    recycle_all();
  }
  g_on.store(on != 0);
  return DSPS_OK;
}

int dsps_profile_read(int kernel_id, double *total_ms, int *launches) {
  if (!total_ms || !launches || kernel_id < 0 || kernel_id >= DSPS_KERNEL_COUNT) {
    set_error("dsps_profile_read: bad arguments");
    return DSPS_ERR_ARG;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  double sum = 0.0;
  int n = 0;
  for (const Record &r : g_records) {
    if (r.kid != kernel_id) continue;
    if (int rc = hip_fail(hipEventSynchronize(r.stop), "hipEventSynchronize")) return rc;
    float ms = 0.0f;
    if (int rc = hip_fail(hipEventElapsedTime(&ms, r.start, r.stop), "hipEventElapsedTime")) return rc;
    sum += ms;
    ++n;
  }
  *total_ms = sum;
  *launches = n;
  return DSPS_OK;
}

}  // extern "C"
