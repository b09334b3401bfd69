// Tuned launch parameters.  A process-wide table maps a shape key (kernel,
// device architecture, sizes) to the chosen value; launchers look their
// parameter up and fall back to a heuristic.  spp_autotune() fills it by
// timing the candidates on the factor's own shapes; the table can be read
// from and written to a text file ("key value" per line) named by the
// SPP_TUNE_CACHE environment variable, so later processes skip the search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "common.hpp"
#include "kernels.hpp"

namespace spp {
namespace {

std::mutex g_tune_mu;
auto& g_table = *new std::map<std::string, int>();
auto& g_forced = *new std::map<std::string, int>();
bool g_loaded = false;

const std::string& arch() {
  static const std::string a = [] {
    std::string s;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) s = prop.gcnArchName;
    const size_t colon = s.find(':');
    if (colon != std::string::npos) s = s.substr(0, colon);
    return s.empty() ? std::string("unknown") : s;
  }();
  return a;
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("SPP_TUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ss(line);
    std::string key;
    int v;
    if (ss >> key >> v) g_table[key] = v;
  }
}

}  // namespace

std::string tune_key(const char* kind, std::initializer_list<int64_t> sizes) {
  std::string k = std::string(kind) + "@" + arch();
  for (int64_t s : sizes) k += ":" + std::to_string(s);
  return k;
}

int tune_get(const std::string& key, int fallback) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto f = g_forced.find(key);
  if (f != g_forced.end()) return f->second;
  load_locked();
  auto it = g_table.find(key);
  return it == g_table.end() ? fallback : it->second;
}

void tune_force(const std::string& key, int value) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  if (value < 0) g_forced.erase(key);
  else g_forced[key] = value;
}

void tune_set(const std::string& key, int value) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  load_locked();
  if (value < 0) g_table.erase(key);
  else g_table[key] = value;
}

bool tune_has(const std::string& key) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  load_locked();
  return g_table.count(key) != 0;
}

void tune_save() {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const char* path = std::getenv("SPP_TUNE_CACHE");
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp);
    for (const auto& kv : g_table) out << kv.first << " " << kv.second << "\n";
  }
  std::rename(tmp.c_str(), path);
}

// Median-free minimum of `reps` timed runs of fn on stream st (milliseconds).
float tune_time(hipStream_t st, int reps, const std::function<void()>& fn, void* flush, size_t flush_bytes) {
  hipEvent_t a, b;
  SPP_HIP(hipEventCreate(&a));
  SPP_HIP(hipEventCreate(&b));
  fn();   // warm-up
  float best = 1e30f;
  for (int r = 0; r < reps; ++r) {
    // Operands that stay in the last-level cache between repetitions would
    // time a candidate faster than it runs inside a solve, where every level
    // streams its factors from HBM: overwrite a buffer larger than that
    // cache first.
    if (flush) SPP_HIP(hipMemsetAsync(flush, r & 0xff, flush_bytes, st));
    SPP_HIP(hipEventRecord(a, st));
    fn();
    SPP_HIP(hipEventRecord(b, st));
    SPP_HIP(hipEventSynchronize(b));
    float ms = 0;
    SPP_HIP(hipEventElapsedTime(&ms, a, b));
    best = std::min(best, ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

}  // namespace spp
