// Opt-in per-kernel timing with HIP events recorded on the launch stream.
//
// When enabled, every launcher brackets its kernel with a pair of events on
// the stream it launches on; mipq_profile_collect() waits for them and reports
// the number of launches and their summed duration per kernel.  Disabled (the
// default), the brackets cost one relaxed atomic load.  Launches recorded into
// a graph (stream capture) are not bracketed.
#include <atomic>
#include <mutex>
#include <vector>

#include "mipq_internal.h"

namespace mipq {

namespace {

struct Pair {
  hipEvent_t a, b;
};

std::atomic<int> g_on{0};
std::mutex g_mu;
std::vector<Pair> g_pending[MIPQ_KERNEL_COUNT];
std::vector<Pair> g_pool;

hipEvent_t take_event() {
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

ProfScope::ProfScope(int kernel, hipStream_t s) : kernel_(kernel), s_(s) {
  if (!g_on.load(std::memory_order_relaxed)) return;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return;   // graph capture
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_pool.empty()) {
    Pair p = g_pool.back();
    g_pool.pop_back();
    a_ = p.a;
    b_ = p.b;
  } else {
    a_ = take_event();
    b_ = take_event();
  }
  if (a_ && b_ && hipEventRecord(a_, s_) != hipSuccess) a_ = nullptr;
}

ProfScope::~ProfScope() {
  if (!a_ || !b_) return;
  if (hipEventRecord(b_, s_) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending[kernel_].push_back({a_, b_});
}

}  // namespace mipq

using namespace mipq;

extern "C" {

int mipq_profile_enable(int on) {
  g_on.store(on ? 1 : 0);
  return MIPQ_OK;
}

int mipq_profile_collect(int kernel, int64_t* launches, double* total_ms) {
  if (kernel < 0 || kernel >= MIPQ_KERNEL_COUNT) return fail(MIPQ_EINVAL, "unknown kernel id %d", kernel);
  std::vector<Pair> got;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    got.swap(g_pending[kernel]);
  }
  int64_t cnt = 0;
  double tot = 0.0;
  int rc = MIPQ_OK;
  for (const Pair& p : got) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(p.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess && rc == MIPQ_OK) rc = hip_fail(e, "hipEventElapsedTime");
    tot += ms;
    ++cnt;
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const Pair& p : got) g_pool.push_back(p);
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = tot;
  return rc;
}

}  // extern "C"
