// Opt-in timing of the kernel-matrix product launches with HIP events recorded
// on the launching stream (per host thread). Disabled by default; when enabled,
// each main product kernel is bracketed by an event pair from a pool, and
// gpl_timing_read() waits on the recorded events and sums their elapsed times.
#include <vector>

#include "common.hpp"
#include "timing.hpp"

namespace gpl {

namespace {
struct TimingState {
  bool on = false;
  std::vector<hipEvent_t> pool;  // pairs: 2k = start, 2k+1 = stop
  int used = 0;                  // pairs recorded since the last read
  double total_ms = 0.0;
  long count = 0;
};
thread_local TimingState g_t;
}  // namespace

hipEvent_t timing_begin(hipStream_t stream) {
  if (!g_t.on) return nullptr;
  if ((int)g_t.pool.size() < 2 * (g_t.used + 1)) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      g_t.pool.push_back(e);
    }
  }
  hipEvent_t e = g_t.pool[2 * g_t.used];
  if (hipEventRecord(e, stream) != hipSuccess) return nullptr;
  return e;
}

void timing_end(hipEvent_t begin, hipStream_t stream) {
  if (!g_t.on || begin == nullptr) return;
  hipEvent_t e = g_t.pool[2 * g_t.used + 1];
  if (hipEventRecord(e, stream) == hipSuccess) ++g_t.used;
}

static int flush() {
  for (int k = 0; k < g_t.used; ++k) {
    float ms = 0.f;
    GPL_HIP(hipEventSynchronize(g_t.pool[2 * k + 1]));
    GPL_HIP(hipEventElapsedTime(&ms, g_t.pool[2 * k], g_t.pool[2 * k + 1]));
    g_t.total_ms += ms;
    ++g_t.count;
  }
  g_t.used = 0;
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" int gpl_timing_enable(int on) {
  if (!on) GPL_TRY(flush());
  g_t.on = on != 0;
  return GPL_OK;
}

extern "C" int gpl_timing_read(double* total_ms, long* launches, int reset) {
  GPL_REQUIRE(total_ms && launches, "NULL argument");
  GPL_TRY(flush());
  *total_ms = g_t.total_ms;
  *launches = g_t.count;
  if (reset) {
    g_t.total_ms = 0.0;
    g_t.count = 0;
  }
  return GPL_OK;
}
