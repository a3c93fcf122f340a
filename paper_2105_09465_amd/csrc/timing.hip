// Opt-in timing of the kernel-matrix product launches with HIP events recorded
// on the launching stream (per host thread). Disabled by default; when enabled
// with stride k, every k-th main product kernel is bracketed by an event pair
// from a pool (an event pair costs the stream a few microseconds, so a stride
// keeps the timed work close to the untimed one), and the read functions wait
// on the recorded events and report their elapsed times.
#include <algorithm>
#include <vector>

#include "common.hpp"
#include "timing.hpp"

namespace gpl {

namespace {
struct TimingState {
  int stride = 0;                // 0: off
  long seq = 0;                  // launches seen since enabled
  std::vector<hipEvent_t> pool;  // pairs: 2k = start, 2k+1 = stop
  int used = 0;                  // pairs recorded and not yet read
  std::vector<float> samples;    // elapsed ms of the read pairs since the last reset
};
thread_local TimingState g_t;
}  // namespace

hipEvent_t timing_begin(hipStream_t stream) {
  if (g_t.stride <= 0) return nullptr;
  if (g_t.seq++ % g_t.stride != 0) return nullptr;
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
  if (begin == nullptr) return;
  hipEvent_t e = g_t.pool[2 * g_t.used + 1];
  if (hipEventRecord(e, stream) == hipSuccess) ++g_t.used;
}

static int flush() {
  for (int k = 0; k < g_t.used; ++k) {
    float ms = 0.f;
    GPL_HIP(hipEventSynchronize(g_t.pool[2 * k + 1]));
    GPL_HIP(hipEventElapsedTime(&ms, g_t.pool[2 * k], g_t.pool[2 * k + 1]));
    g_t.samples.push_back(ms);
  }
  g_t.used = 0;
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" int gpl_timing_enable(int stride) {
  GPL_REQUIRE(stride >= 0, "stride must be >= 0");
  if (stride == 0) GPL_TRY(flush());
  g_t.stride = stride;
  g_t.seq = 0;
  return GPL_OK;
}

extern "C" int gpl_timing_read(double* total_ms, long* launches, int reset) {
  GPL_REQUIRE(total_ms && launches, "NULL argument");
  GPL_TRY(flush());
  double s = 0.0;
  for (float v : g_t.samples) s += v;
  *total_ms = s;
  *launches = (long)g_t.samples.size();
  if (reset) g_t.samples.clear();
  return GPL_OK;
}

extern "C" int gpl_timing_samples(float* ms, int cap, int* count, int reset) {
  GPL_REQUIRE(count != nullptr && cap >= 0 && (ms != nullptr || cap == 0), "bad argument");
  GPL_TRY(flush());
  const int n = (int)g_t.samples.size();
  std::copy(g_t.samples.begin(), g_t.samples.begin() + std::min(n, cap), ms);
  *count = n;
  if (reset) g_t.samples.clear();
  return GPL_OK;
}
