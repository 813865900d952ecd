// tc_profile_enable / tc_profile_read: per-kernel-class hipEvent timing.
#include <atomic>
#include <mutex>
#include <vector>

#include "profile.h"

namespace tcm {
namespace {

struct Rec {
  int kind;
  hipEvent_t start, stop;
  bool closed;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void release_all() {
  for (auto& r : g_recs) {
    if (r.start) g_pool.push_back(r.start);
    if (r.stop) g_pool.push_back(r.stop);
  }
  g_recs.clear();
}

}  // namespace

thread_local bool t_suspended = false;

bool profile_enabled() { return g_on.load(std::memory_order_relaxed) && !t_suspended; }

void profile_suspend(bool on) { t_suspended = on; }

void profile_begin(int kind, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r{kind, get_event(), nullptr, false};
  if (r.start) (void)hipEventRecord(r.start, s);
  g_recs.push_back(r);
}

void profile_end(int kind, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto it = g_recs.rbegin(); it != g_recs.rend(); ++it) {
    if (it->kind == kind && !it->closed) {
      it->stop = get_event();
      if (it->stop) (void)hipEventRecord(it->stop, s);
      it->closed = true;
      return;
    }
  }
}

}  // namespace tcm

using namespace tcm;

extern "C" {

int tc_profile_enable(int32_t enable) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  release_all();
  g_on.store(enable != 0);
  return TC_OK;
}

int tc_profile_read(int32_t kernel, double* total_ms, int64_t* launches) {
  clear_error();
  TC_CHECK_ARG(total_ms != nullptr && launches != nullptr, "output is NULL");
  TC_CHECK_ARG(kernel >= 0 && kernel <= 2, "unknown kernel class");
  std::lock_guard<std::mutex> lk(g_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto& r : g_recs) {
    if (r.kind != kernel || !r.closed || !r.start || !r.stop) continue;
    TC_TRY_HIP(hipEventSynchronize(r.stop));
    float ms = 0.f;
    TC_TRY_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return TC_OK;
}

}  // extern "C"
