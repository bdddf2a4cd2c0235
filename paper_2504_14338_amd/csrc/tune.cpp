// Process-wide table of tuned launch parameters of libdopinf, keyed by
// (parameter, problem size).  Written by the autotuner (or by the caller),
// read by the host code that plans launches.  A mutex guards it, so calls on
// several host threads may read and write it concurrently.
#include <cstdint>
#include <map>
#include <mutex>
#include <utility>

#include "../../include/dopinf.h"

namespace dopinf {
int fail(int code, const char* fmt, ...);

namespace tune {
namespace {
std::mutex g_mu;
std::map<std::pair<int, int64_t>, int>& table() {
  static std::map<std::pair<int, int64_t>, int> t;
  return t;
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
}

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
