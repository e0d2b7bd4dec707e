// Optional per-launch kernel timing with HIP events (dks_profile_enable /
// dks_profile_report).  Events are pooled per thread and reused.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "dks_internal.h"

namespace dks {

namespace {
struct Rec {
  const char *name;
  hipEvent_t a, b;
};
struct ProfState {
  bool on = false;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
};
thread_local ProfState g_prof;
}  // namespace

ProfScope::ProfScope(const char *name, hipStream_t st) : st_(st) {
  if (!g_prof.on) return;
  hipEvent_t a = g_prof.get(), b = g_prof.get();
  if (!a || !b) return;
  (void)hipEventRecord(a, st);
  g_prof.recs.push_back(Rec{name, a, b});
  idx_ = (int)g_prof.recs.size() - 1;
}

ProfPause::ProfPause() : was_on_(g_prof.on) { g_prof.on = false; }
ProfPause::~ProfPause() { g_prof.on = was_on_; }

ProfScope::~ProfScope() {
  if (idx_ >= 0 && g_prof.on && idx_ < (int)g_prof.recs.size())
    (void)hipEventRecord(g_prof.recs[idx_].b, st_);
}

}  // namespace dks

using namespace dks;

extern "C" {

void dks_profile_enable(int on) { g_prof.on = (on != 0); }

dks_status dks_profile_report(char *buf, size_t len) {
  if (!buf || len == 0) {
    set_error("null buffer");
    return DKS_EINVAL;
  }
  if (hipDeviceSynchronize() != hipSuccess) {
    set_error("hipDeviceSynchronize failed");
    return DKS_EHIP;
  }
  std::map<std::string, std::pair<int, double>> agg;
  for (auto &r : g_prof.recs) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    auto &e = agg[r.name];
    e.first += 1;
    e.second += ms;
  }
  g_prof.recs.clear();
  g_prof.used = 0;
  std::string out = "{";
  bool first = true;
  for (auto &kv : agg) {
    char tmp[256];
    std::snprintf(tmp, sizeof(tmp), "%s\"%s\": {\"count\": %d, \"total_ms\": %.6f}", first ? "" : ", ",
                  kv.first.c_str(), kv.second.first, kv.second.second);
    out += tmp;
    first = false;
  }
  out += "}";
  size_t n = std::min(len - 1, out.size());
  std::memcpy(buf, out.data(), n);
  buf[n] = 0;
  return DKS_OK;
}

}  // extern "C"
