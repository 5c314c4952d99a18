// Per-stage HIP-event timing (off unless enabled).  When enabled, every launch
// of a timed stage is bracketed by two events recorded on the stream the
// stage runs on; skmp_timing_read waits for the events and sums the elapsed
// times, so the figures are the stages' own device durations.  Launches made
// while the stream is being captured into a graph are not timed.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "skmp_common.hpp"

namespace skmp {

namespace {
struct Pending {
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending[SKMP_TIMER_COUNT];
double g_ms[SKMP_TIMER_COUNT];
int64_t g_n[SKMP_TIMER_COUNT];
}  // namespace

StageTimer::StageTimer(int which, hipStream_t st) : which_(which), st_(st) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || which < 0 || which >= SKMP_TIMER_COUNT) return;
  if (stream_capturing(st)) return;  // events inside a graph would time the capture, not a run
  if (hipEventCreate(&a_) != hipSuccess) return;
  if (hipEventCreate(&b_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    return;
  }
  if (hipEventRecord(a_, st_) != hipSuccess) {
    (void)hipEventDestroy(a_);
    (void)hipEventDestroy(b_);
    return;
  }
  live_ = true;
}

StageTimer::~StageTimer() {
  if (!live_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (hipEventRecord(b_, st_) == hipSuccess) g_pending[which_].push_back({a_, b_});
}

}  // namespace skmp

using namespace skmp;

extern "C" int skmp_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return SKMP_OK;
}

extern "C" int skmp_timing_read(int32_t which, int32_t reset, double* total_ms, int64_t* launches) {
  clear_error();
  SKMP_REQUIRE(which >= 0 && which < SKMP_TIMER_COUNT, "unknown timer");
  std::lock_guard<std::mutex> lk(g_mu);
  for (const Pending& p : g_pending[which]) {
    float ms = 0.f;
    SKMP_CHECK_HIP(hipEventSynchronize(p.b));
    SKMP_CHECK_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    g_ms[which] += ms;
    g_n[which] += 1;
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending[which].clear();
  if (total_ms) *total_ms = g_ms[which];
  if (launches) *launches = g_n[which];
  if (reset) {
    g_ms[which] = 0.0;
    g_n[which] = 0;
  }
  return SKMP_OK;
}
