// Event pool and per-kernel aggregation behind spike_profile_enable() and
// spike_profile_report().
#include "spike_profile.hpp"

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spike.h"

namespace spike {

namespace {

struct Rec {
  std::string name;
  hipEvent_t start, end;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::string g_only;    // the one kernel to bracket, empty for all
std::string g_armed;   // g_only as of the last spike_profile_enable
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

void recycle_all() {
  for (auto& r : g_recs) {
    if (r.start) g_pool.push_back(r.start);
    if (r.end) g_pool.push_back(r.end);
  }
  g_recs.clear();
}

}  // namespace

bool prof_enabled() { return g_on.load(std::memory_order_relaxed); }

int prof_begin(const char* name, hipStream_t st) {
  // no timing events inside a stream capture (they would become graph nodes)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_armed.empty() && g_armed != name) return -1;
  Rec r{name, take_event(), take_event()};
  if (!r.start || !r.end) return -1;
  hipEventRecord(r.start, st);
  g_recs.push_back(r);
  return (int)g_recs.size() - 1;
}

void prof_end(int slot, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot >= 0 && slot < (int)g_recs.size()) hipEventRecord(g_recs[slot].end, st);
}

}  // namespace spike

extern "C" {

int spike_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(spike::g_mu);
  spike::recycle_all();
  spike::g_armed = spike::g_only;
  spike::g_on.store(on != 0);
  return 0;
}

int spike_profile_only(const char* name) {
  if (name && std::strlen(name) > 47) return -1;
  std::lock_guard<std::mutex> lk(spike::g_mu);
  spike::g_only = name ? name : "";
  return 0;
}

int spike_profile_report(spike_kernel_time* out, int cap, int* count) {
  std::lock_guard<std::mutex> lk(spike::g_mu);
  std::map<std::string, std::pair<int, double>> agg;
  for (auto& r : spike::g_recs) {
    if (hipEventSynchronize(r.end) != hipSuccess) return SPIKE_ERR_HIP - (int)hipErrorUnknown;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.end) != hipSuccess) continue;
    auto& a = agg[r.name];
    a.first += 1;
    a.second += ms;
  }
  int i = 0;
  for (auto& kv : agg) {
    if (out && i < cap) {
      std::memset(&out[i], 0, sizeof(out[i]));
      std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
      out[i].calls = kv.second.first;
      out[i].total_ms = kv.second.second;
    }
    ++i;
  }
  if (count) *count = i;
  return 0;
}

}  // extern "C"
