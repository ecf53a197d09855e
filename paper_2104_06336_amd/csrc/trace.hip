// Kernel tracing: when enabled, every launch of the library is bracketed by two hipEvents
// recorded on the launch stream; stem_trace_get() reports per-kernel launch counts and the
// summed event-to-event durations.  Disabled (the default) it costs one flag test per launch.
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "trace.h"

namespace stem {

namespace {
struct Rec {
  std::string name;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;  // events released by a previous trace session

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

void release_all() {
  for (auto& r : g_recs)
    for (auto& p : r.ev) {
      if (p.first) g_pool.push_back(p.first);
      if (p.second) g_pool.push_back(p.second);
    }
  g_recs.clear();
}
}  // namespace

bool trace_enabled() { return g_on; }

TraceScope::TraceScope(const char* name, hipStream_t s) : stream_(s), stop_(nullptr) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t a = take_event(), b = take_event();
  if (!a || !b) return;
  Rec* rec = nullptr;
  for (auto& r : g_recs)
    if (r.name == name) rec = &r;
  if (!rec) {
    g_recs.push_back(Rec{name, {}});
    rec = &g_recs.back();
  }
  rec->ev.emplace_back(a, b);
  (void)hipEventRecord(a, s);
  stop_ = b;
}

TraceScope::~TraceScope() {
  if (stop_) (void)hipEventRecord(stop_, stream_);
}

}  // namespace stem

using namespace stem;

extern "C" int stem_trace_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (on) release_all();
  g_on = on != 0;
  return STEM_OK;
}

extern "C" int stem_trace_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (int)g_recs.size();
}

extern "C" int stem_trace_get(int i, char* name, size_t name_len, int64_t* launches, double* total_ms) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (i < 0 || i >= (int)g_recs.size() || !launches || !total_ms) return STEM_EINVAL;
  const Rec& r = g_recs[i];
  if (name && name_len > 0) {
    size_t n = r.name.size() < name_len - 1 ? r.name.size() : name_len - 1;
    r.name.copy(name, n);
    name[n] = 0;
  }
  double tot = 0.0;
  for (const auto& p : r.ev) {
    if (hipEventSynchronize(p.second) != hipSuccess) return STEM_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.first, p.second) != hipSuccess) return STEM_EHIP;
    tot += ms;
  }
  *launches = (int64_t)r.ev.size();
  *total_ms = tot;
  return STEM_OK;
}
