#include "prof.h"

#include <mutex>
#include <vector>

#include "../../include/hps.h"

namespace hps {

namespace {
struct Rec {
  int cls;
  hipEvent_t a, b;
  double flops, bytes;
};
std::mutex g_mu;
unsigned g_mask = 0;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

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
}  // namespace

thread_local int t_paused = 0;

bool prof_on(int cls) { return t_paused == 0 && ((g_mask >> cls) & 1u); }

ProfPause::ProfPause() { ++t_paused; }
ProfPause::~ProfPause() { --t_paused; }

ProfScope::ProfScope(int cls, hipStream_t s, double flops, double bytes) : s_(s) {
  if (!prof_on(cls)) return;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r{cls, take_event(), take_event(), flops, bytes};
  if (!r.a || !r.b) return;
  (void)hipEventRecord(r.a, s);
  rec_ = (int)g_recs.size();
  g_recs.push_back(r);
}

ProfScope::~ProfScope() {
  if (rec_ < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord(g_recs[rec_].b, s_);
}

}  // namespace hps

extern "C" {

hps_status hps_prof_enable(unsigned mask) {
  std::lock_guard<std::mutex> lk(hps::g_mu);
  hps::g_mask = mask;
  return HPS_OK;
}

hps_status hps_prof_reset(void) {
  std::lock_guard<std::mutex> lk(hps::g_mu);
  for (auto& r : hps::g_recs) {
    (void)hipEventSynchronize(r.b);
    hps::g_pool.push_back(r.a);
    hps::g_pool.push_back(r.b);
  }
  hps::g_recs.clear();
  return HPS_OK;
}

hps_status hps_prof_query(int cls, double* ms, long long* launches, double* flops, double* bytes) {
  std::lock_guard<std::mutex> lk(hps::g_mu);
  double t = 0, f = 0, b = 0;
  long long n = 0;
  for (auto& r : hps::g_recs) {
    if (r.cls != cls) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return HPS_EDEVICE;
    float e = 0.f;
    if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) return HPS_EDEVICE;
    t += e;
    f += r.flops;
    b += r.bytes;
    ++n;
  }
  if (ms) *ms = t;
  if (launches) *launches = n;
  if (flops) *flops = f;
  if (bytes) *bytes = b;
  return HPS_OK;
}

}  // extern "C"
