// Process-wide table of tuned launch parameters of libdopinf, keyed by
// (parameter, problem size).  Written by the autotuner (or by the caller),
// read by the host code that plans launches.  A mutex guards it, so calls on
// several host threads may read and write it concurrently.
//
// Persistence: when the environment variable DOPINF_TUNE_CACHE names a file,
// the table is loaded from it on first use (lines "param key value"; lines
// that do not parse or hold invalid values are ignored) and the whole table
// is written back (to a temporary file, then renamed) after every change.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "../../include/dopinf.h"

namespace dopinf {
int fail(int code, const char* fmt, ...);

namespace tune {
namespace {
std::mutex g_mu;

bool valid(int param, int64_t key, int value) {
  const bool p = param == DOPINF_TUNE_CHOL_KB || param == DOPINF_TUNE_TRSM_KB || param == DOPINF_TUNE_CHOL_KB2 ||
                 param == DOPINF_TUNE_TRSM_KB2;
  return p && key >= 1 && value >= 64 && value <= 4096 && value % 64 == 0;
}

const char* cache_path() {
  const char* p = std::getenv("DOPINF_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// the table, loaded from the cache file on first use (caller holds g_mu)
std::map<std::pair<int, int64_t>, int>& table() {
  static std::map<std::pair<int, int64_t>, int> t;
  static bool loaded = false;
  if (!loaded) {
    loaded = true;
    if (const char* path = cache_path()) {
      if (FILE* f = std::fopen(path, "r")) {
        int param = 0, value = 0;
        long long key = 0;
        char line[256];
        while (std::fgets(line, sizeof(line), f))
          if (std::sscanf(line, "%d %lld %d", &param, &key, &value) == 3 && valid(param, key, value))
            t[{param, int64_t(key)}] = value;
        std::fclose(f);
      }
    }
  }
  return t;
}

// write the table back to the cache file (caller holds g_mu)
void save() {
  const char* path = cache_path();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto& e : table()) std::fprintf(f, "%d %lld %d\n", e.first.first, (long long)e.first.second, e.second);
  const bool ok = std::fclose(f) == 0;
  if (ok) std::rename(tmp.c_str(), path);
}
}  // namespace

int get(int param, int64_t key) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = table().find({param, key});
  return it == table().end() ? 0 : it->second;
}

void set(int param, int64_t key, int value) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (value == 0)
    table().erase({param, key});
  else
    table()[{param, key}] = value;
  save();
}

bool persisted() { return cache_path() != nullptr; }

}  // namespace tune
}  // namespace dopinf

extern "C" int dopinf_tune_set(int param, int64_t key, int value) {
  if (param != DOPINF_TUNE_CHOL_KB && param != DOPINF_TUNE_TRSM_KB && param != DOPINF_TUNE_CHOL_KB2 &&
      param != DOPINF_TUNE_TRSM_KB2)
    return dopinf::fail(DOPINF_E_ARG, "unknown tuning parameter %d", param);
  if (key < 1) return dopinf::fail(DOPINF_E_ARG, "tuning key must be >= 1");
  if (value != 0 && (value < 64 || value > 4096 || value % 64 != 0))
    return dopinf::fail(DOPINF_E_ARG, "block-column width must be a multiple of 64 in [64, 4096], or 0");
  dopinf::tune::set(param, key, value);
  return DOPINF_OK;
}

extern "C" int dopinf_tune_get(int param, int64_t key) { return dopinf::tune::get(param, key); }
