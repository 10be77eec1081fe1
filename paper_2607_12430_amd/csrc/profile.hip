// Kernel-class timing registry behind msqrt_profile_* (include/msqrt.h).
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/msqrt.h"
#include "profile.hpp"

namespace msqrt {

namespace {
struct Pending {
  std::string cls;
  hipEvent_t a, b;
  double flops, bytes;
};
struct Stats {
  int64_t launches = 0;
  double ms = 0, flops = 0, bytes = 0;
};
std::mutex g_mu;
bool g_on = false;
std::vector<hipEvent_t> g_pool;
std::vector<hipEvent_t> g_open;  // indexed by token
std::vector<Pending> g_pend;
std::map<std::string, Stats> g_stats;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  MSQRT_HIP(hipEventCreate(&e));
  return e;
}

void resolve_locked() {
  for (auto& p : g_pend) {
    float ms = 0.f;
    (void)hipEventSynchronize(p.b);
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      Stats& s = g_stats[p.cls];
      s.launches++;
      s.ms += ms;
      s.flops += p.flops;
      s.bytes += p.bytes;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_pend.clear();
}
}  // namespace

bool prof_enabled() { return g_on; }

void prof_release() {
  std::lock_guard<std::mutex> lk(g_mu);
  resolve_locked();
  g_open.clear();  // every recorded begin event is also in the pool now
  for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
  g_pool.clear();
}

int prof_begin(hipStream_t st) {
  if (!g_on) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = get_event();
  MSQRT_HIP(hipEventRecord(e, st));
  g_open.push_back(e);
  return (int)g_open.size() - 1;
}

void prof_end(int token, hipStream_t st, const char* cls, double flops, double bytes) {
  if (token < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  hipEvent_t e = get_event();
  MSQRT_HIP(hipEventRecord(e, st));
  g_pend.push_back({cls, g_open[token], e, flops, bytes});
  if (g_pend.size() > 4096) resolve_locked();
}

}  // namespace msqrt

extern "C" {

void msqrt_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(msqrt::g_mu);
  msqrt::resolve_locked();
  msqrt::g_open.clear();
  msqrt::g_stats.clear();
  msqrt::g_on = on != 0;
}

int msqrt_profile_query(const char* cls, int64_t* launches, double* total_ms, double* flops,
                        double* bytes) {
  std::lock_guard<std::mutex> lk(msqrt::g_mu);
  msqrt::resolve_locked();
  auto it = msqrt::g_stats.find(cls ? cls : "");
  if (it == msqrt::g_stats.end()) return 1;
  if (launches) *launches = it->second.launches;
  if (total_ms) *total_ms = it->second.ms;
  if (flops) *flops = it->second.flops;
  if (bytes) *bytes = it->second.bytes;
  return 0;
}

int msqrt_profile_list(char* buf, int buflen) {
  std::lock_guard<std::mutex> lk(msqrt::g_mu);
  msqrt::resolve_locked();
  std::string s;
  for (auto& kv : msqrt::g_stats) {
    if (!s.empty()) s += ",";
    s += kv.first;
  }
  if (buf && buflen > 0) {
    std::strncpy(buf, s.c_str(), (size_t)buflen - 1);
    buf[buflen - 1] = 0;
  }
  return (int)s.size();
}

}  // extern "C"
