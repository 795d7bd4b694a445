// Kernel timing: when enabled, selected launches are bracketed by HIP events
// recorded on the launch stream, together with the launch's algorithmic
// byte count; ah_profile_read sums them per kernel tag.
#include <map>
#include <mutex>

#include "prof.h"

namespace ah {

bool g_prof = false;

namespace {
struct Rec {
  std::string tag;
  hipEvent_t a, b;
  double bytes;
};
std::mutex mu;
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;

hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  // timing only (read after the stream has been synchronized): no
  // system-scope fence at each record, whose cache writeback would both
  // stall the stream between the bracketed launches and start the next
  // launch with cold caches
  hipEvent_t e;
  (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
  return e;
}
}  // namespace

void prof_begin(ProfScope& s, const char* tag, hipStream_t st, double bytes) {
  if (!g_prof || !tag) return;
  std::lock_guard<std::mutex> g(mu);
  s.active = true;
  s.tag = tag;
  s.st = st;
  s.bytes = bytes;
  s.a = get_event();
  s.b = get_event();
  (void)hipEventRecord(s.a, st);
}

void prof_end(ProfScope& s) {
  if (!s.active) return;
  std::lock_guard<std::mutex> g(mu);
  (void)hipEventRecord(s.b, s.st);
  recs.push_back({s.tag, s.a, s.b, s.bytes});
  s.active = false;
}

}  // namespace ah

using namespace ah;

extern "C" void ah_profile_enable(int on) {
  std::lock_guard<std::mutex> g(mu);
  g_prof = on != 0;
}

extern "C" void ah_profile_reset(void) {
  std::lock_guard<std::mutex> g(mu);
  for (auto& r : recs) {
    (void)hipEventSynchronize(r.b);
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
}

extern "C" ah_status ah_profile_read(const char* tag, int64_t* launches, double* total_ms, double* bytes) {
  if (!tag) { set_error("ah_profile_read: null tag"); return AH_EINVAL; }
  std::lock_guard<std::mutex> g(mu);
  int64_t n = 0;
  double ms = 0.0, by = 0.0;
  for (auto& r : recs) {
    if (r.tag != tag) continue;
    AH_HIP(hipEventSynchronize(r.b));
    float t = 0.f;
    AH_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ++n;
    ms += t;
    by += r.bytes;
  }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  if (bytes) *bytes = by;
  return AH_OK;
}
