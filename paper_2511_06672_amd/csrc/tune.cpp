// Launch-parameter tuner (see tune.h): a process-wide cache of timed choices, optionally mirrored
// to a JSON file.
#include "tune.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

namespace gc {
namespace {

using Key = std::tuple<std::string, int, int, int, int>;  // knob, prec, d, s0, s1

struct Entry {
  int choice;
  std::vector<double> us;
};

struct Cache {
  std::mutex mu;
  std::map<Key, Entry> map;
  std::string path;  // the file the map mirrors ("" when none)
};

Cache& cache() {
  static Cache c;
  return c;
}

bool tuning_on() {
  const char* e = std::getenv("GCAMPS_AUTOTUNE");
  return !(e && std::strcmp(e, "0") == 0);
}

void trace(const Key& key, int choice, const char* source) {
  if (!std::getenv("GCAMPS_TRACE_TUNE")) return;
  std::fprintf(stderr, "gcamps-tune knob=%s prec=%d d=%d shape=%dx%d choice=%d source=%s\n",
               std::get<0>(key).c_str(), std::get<1>(key), std::get<2>(key), std::get<3>(key), std::get<4>(key),
               choice, source);
}

// Reads the entry lines of a cache file; other lines are skipped.
void load(std::map<Key, Entry>& map, const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  char line[4096];
  while (std::fgets(line, sizeof(line), f)) {
    const char* p = std::strstr(line, "{\"knob\"");
    if (!p) continue;
    char knob[64];
    int prec, d, s0, s1, choice;
    if (std::sscanf(p, "{\"knob\": \"%63[^\"]\", \"prec\": %d, \"d\": %d, \"shape\": [%d, %d], \"choice\": %d", knob,
                    &prec, &d, &s0, &s1, &choice) != 6)
      continue;
    Entry e{choice, {}};
    if (const char* u = std::strstr(p, "\"us\": [")) {
      u += 7;
      while (*u && *u != ']') {
        char* end = nullptr;
        const double v = std::strtod(u, &end);
        if (end == u) break;
        e.us.push_back(v);
        u = end;
        while (*u == ',' || *u == ' ') ++u;
      }
    }
    map[Key{knob, prec, d, s0, s1}] = e;
  }
  std::fclose(f);
}

// Writes the whole map (to a temporary file first, then renamed over the target).
void save(const std::map<Key, Entry>& map, const std::string& path) {
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\"entries\": [\n");
  size_t i = 0;
  for (const auto& kv : map) {
    const Key& k = kv.first;
    std::fprintf(f, "  {\"knob\": \"%s\", \"prec\": %d, \"d\": %d, \"shape\": [%d, %d], \"choice\": %d, \"us\": [",
                 std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k),
                 kv.second.choice);
    for (size_t j = 0; j < kv.second.us.size(); ++j) std::fprintf(f, "%s%.3f", j ? ", " : "", kv.second.us[j]);
    std::fprintf(f, "]}%s\n", ++i < map.size() ? "," : "");
  }
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  if (ok) std::rename(tmp.c_str(), path.c_str());
}

bool allowed(int choice, const int* choices, int n) {
  for (int i = 0; i < n; ++i)
    if (choices[i] == choice) return true;
  return false;
}

// Event pair that is destroyed on every exit path.
struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  Events() {
    GC_HIP(hipEventCreate(&e0));
    GC_HIP(hipEventCreate(&e1));
  }
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

}  // namespace

int tuned_choice(hipStream_t s, const char* knob, int prec, int d, int s0, int s1, const int* choices, int nchoices,
                 int fallback, const std::function<void(int)>& run) {
  if (!tuning_on() || nchoices <= 1) return fallback;
  Cache& c = cache();
  const Key key{knob, prec, d, s0, s1};
  const char* env_path = std::getenv("GCAMPS_TUNE_FILE");
  const std::string path = env_path ? env_path : "";
  // The lock is held while a new shape is timed, so concurrent lanes time each shape once.
  std::lock_guard<std::mutex> lock(c.mu);
  if (path != c.path) {  // a new file: its entries replace the map
    c.map.clear();
    if (!path.empty()) load(c.map, path);
    c.path = path;
    for (const auto& kv : c.map) trace(kv.first, kv.second.choice, "file");
  }
  auto it = c.map.find(key);
  if (it != c.map.end() && allowed(it->second.choice, choices, nchoices)) {
    trace(key, it->second.choice, "cache");
    return it->second.choice;
  }
  Events ev;
  Entry e{fallback, {}};
  double best = -1.0;
  for (int i = 0; i < nchoices; ++i) {
    run(choices[i]);  // first run: instruction cache and operands warm
    GC_HIP(hipEventRecord(ev.e0, s));
    run(choices[i]);
    GC_HIP(hipEventRecord(ev.e1, s));
    GC_HIP(hipEventSynchronize(ev.e1));
    float ms = 0.0f;
    GC_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    e.us.push_back(1e3 * ms);
    if (best < 0.0 || 1e3 * ms < best) {
      best = 1e3 * ms;
      e.choice = choices[i];
    }
  }
  c.map[key] = e;
  if (!c.path.empty()) save(c.map, c.path);
  trace(key, e.choice, "timed");
  return e.choice;
}

}  // namespace gc
