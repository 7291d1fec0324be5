// Optional per-kernel timing: when enabled, the library brackets its main
// kernel launches with HIP events on the launch stream; the report
// aggregates the elapsed times by kernel name.  Off by default; not for use
// under graph capture.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "profile.hpp"

namespace spg {

namespace {
struct Rec {
  const char *name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
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

bool profiling() { return g_on; }

ProfScope::ProfScope(const char *name, hipStream_t st) : name_(name), st_(st), a_(nullptr) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a_ = take_event();
  if (a_) (void)hipEventRecord((hipEvent_t)a_, st_);
}

ProfScope::~ProfScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t b = take_event();
  if (!b) return;
  (void)hipEventRecord(b, st_);
  g_recs.push_back(Rec{name_, (hipEvent_t)a_, b});
}

}  // namespace spg

using namespace spg;

extern "C" {

int spgemm_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto &r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  g_on = on != 0;
  return SPGEMM_OK;
}

int spgemm_profile_report(char *buf_host, size_t buf_bytes) {
  if (!buf_host || buf_bytes == 0) return SPGEMM_E_INVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  std::map<std::string, std::pair<double, long>> agg;
  for (auto &r : g_recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return SPGEMM_E_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SPGEMM_E_HIP;
    auto &e = agg[r.name];
    e.first += ms;
    e.second += 1;
  }
  size_t off = 0;
  buf_host[0] = 0;
  for (auto &kv : agg) {
    int n = snprintf(buf_host + off, buf_bytes - off, "%s %.6f %ld\n", kv.first.c_str(), kv.second.first,
                     kv.second.second);
    if (n < 0 || (size_t)n >= buf_bytes - off) return SPGEMM_E_INVAL;
    off += (size_t)n;
  }
  return SPGEMM_OK;
}

}  // extern "C"
