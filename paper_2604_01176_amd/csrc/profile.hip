// Per-kernel timing with HIP events.  When enabled, every kernel launch of
// the library is bracketed by two events recorded on the launch stream; the
// collected durations are summed per kernel name on demand.  Disabled (the
// default) it costs one branch per launch.
#include "hyp_internal.h"

#include <cstring>
#include <map>
#include <mutex>

namespace hyp {

namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_pending;
std::vector<hipEvent_t> g_free;
struct Total {
  double ms = 0.0;
  int64_t calls = 0;
};
std::map<std::string, Total> g_tot;

hipEvent_t take_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain_locked() {
  for (Rec& r : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      Total& t = g_tot[r.name];
      t.ms += ms;
      t.calls += 1;
    }
    g_free.push_back(r.a);
    g_free.push_back(r.b);
  }
  g_pending.clear();
}
}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t st) : name_(name), st_(st) {
  if (!g_on) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st_, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a_ = take_event();
  if (a_ && hipEventRecord((hipEvent_t)a_, st_) != hipSuccess) a_ = nullptr;
}

ProfScope::~ProfScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t b = take_event();
  if (!b) return;
  if (hipEventRecord(b, st_) != hipSuccess) return;
  g_pending.push_back({name_, (hipEvent_t)a_, b});
  if (g_pending.size() > 4096) drain_locked();
}

}  // namespace hyp

using namespace hyp;

extern "C" {

hyp_status hyp_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return HYP_OK;
}

hyp_status hyp_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  g_tot.clear();
  return HYP_OK;
}

int hyp_profile_count(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  return (int)g_tot.size();
}

hyp_status hyp_profile_get(int i, char* name, int name_len, double* total_ms, int64_t* calls) {
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  if (i < 0 || i >= (int)g_tot.size() || !name || name_len < 1 || !total_ms || !calls)
    return fail(HYP_ERR_ARG, "hyp_profile_get: bad index or NULL output");
  auto it = g_tot.begin();
  std::advance(it, i);
  std::strncpy(name, it->first.c_str(), (size_t)name_len - 1);
  name[name_len - 1] = 0;
  *total_ms = it->second.ms;
  *calls = it->second.calls;
  return HYP_OK;
}

}  // extern "C"
