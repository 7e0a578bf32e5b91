// Optional per-kernel timing: when enabled, every kernel launch of the
// library is bracketed by HIP events recorded on the launch stream, and
// kaldo_profile_end() reports total time and launch count per kernel name.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace kaldo {

namespace {
struct Mark {
  const char* name;
  hipEvent_t start, stop;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Mark> g_marks;
std::vector<hipEvent_t> g_pool;
hipEvent_t g_pending = nullptr;

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

bool prof_on() { return g_on; }

void prof_mark(const char* name, hipStream_t st, bool start) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  hipEvent_t e = take_event();
  if (!e) return;
  (void)hipEventRecord(e, st);
  if (start) {
    g_pending = e;
  } else if (g_pending) {
    g_marks.push_back({name, g_pending, e});
    g_pending = nullptr;
  } else {
    g_pool.push_back(e);
  }
}

}  // namespace kaldo

using namespace kaldo;

extern "C" int kaldo_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& m : g_marks) {
    g_pool.push_back(m.start);
    g_pool.push_back(m.stop);
  }
  g_marks.clear();
  g_on = true;
  return KALDO_OK;
}

extern "C" int kaldo_profile_end(kaldo_kernel_time* out, int32_t capacity, int32_t* n_out) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = false;
  KALDO_REQUIRE(n_out != nullptr && (capacity == 0 || out != nullptr), "kaldo_profile_end: NULL argument");
  std::map<std::string, std::pair<int64_t, double>> agg;
  std::vector<std::string> order;
  for (auto& m : g_marks) {
    KALDO_HIP(hipEventSynchronize(m.stop));
    float ms = 0.f;
    KALDO_HIP(hipEventElapsedTime(&ms, m.start, m.stop));
    auto it = agg.find(m.name);
    if (it == agg.end()) {
      order.push_back(m.name);
      agg[m.name] = {1, ms};
    } else {
      it->second.first += 1;
      it->second.second += ms;
    }
  }
  int32_t n = 0;
  for (auto& name : order) {
    if (n < capacity) {
      std::memset(out[n].name, 0, sizeof(out[n].name));
      std::strncpy(out[n].name, name.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = agg[name].first;
      out[n].total_ms = agg[name].second;
    }
    ++n;
  }
  *n_out = n;
  for (auto& m : g_marks) {
    g_pool.push_back(m.start);
    g_pool.push_back(m.stop);
  }
  g_marks.clear();
  return KALDO_OK;
}
