// Row-split (split-K) planning shared by the Gram kernels: splits never
// straddle a state variable, so a workgroup applies a single scale factor.
#pragma once

#include "common.hpp"

namespace dopinf {
namespace gramplan {

struct SplitPlan {
  int nvars;
  int nsplit;
  int xcd_map;
  int64_t row0[DOPINF_MAX_VARS + 1];
  int split0[DOPINF_MAX_VARS + 1];
};


// Row range [lo, hi) and variable of split s; the chunk length is a multiple
// of `align` rows.
__device__ __forceinline__ void split_range(const SplitPlan& sp, int s, int align, int64_t& lo, int64_t& hi,
                                            int& v) {
  int vv = 0;
  while (vv + 1 < sp.nvars && s >= sp.split0[vv + 1]) ++vv;
  const int nv = sp.split0[vv + 1] - sp.split0[vv];
  const int64_t rows = sp.row0[vv + 1] - sp.row0[vv];
  int64_t chunk = (rows + nv - 1) / nv;
  chunk = (chunk + align - 1) / align * align;
  lo = sp.row0[vv] + int64_t(s - sp.split0[vv]) * chunk;
  hi = min(sp.row0[vv + 1], lo + chunk);
  if (lo > hi) lo = hi;
  v = vv;
}

// Lower-triangle tile index t -> (I, J), t = I(I+1)/2 + J.
__device__ __forceinline__ void tri_coords(int t, int& I, int& J) {
  int i = int((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// Row splits of a Gram launch of ntiles tiles.  With slots > 0 (resident
// workgroups of the launch on the whole device) the count is rounded up, by
// at most a quarter, to make nsplit x ntiles whole rounds of slots, so that
// no partial last round idles the device (n = 4e6, k = 2000: 64 splits x 136
// tiles = 17 rounds of 512, ~1% faster than 56 splits).
inline int choose_splits(int64_t n, int ntiles, int wgs_target = 8192, int slots = 0) {
  int target = (wgs_target + ntiles - 1) / ntiles;
  int64_t max_by_rows = n / 256;
  if (max_by_rows < 1) max_by_rows = 1;
  if (target > max_by_rows) target = int(max_by_rows);
  if (target >= 8) target = target / 8 * 8;
  if (target < 1) target = 1;
  if (slots > 0 && target >= 8) {
    int a = ntiles, b = slots;
    while (b) {
      const int t = a % b;
      a = b;
      b = t;
    }
    const int step = slots / a;
    const int up = (target + step - 1) / step * step;
    if (up <= target + target / 4 && up <= max_by_rows) target = up;
  }
  return target;
}

inline SplitPlan make_plan(int64_t n, int nvars, const int64_t* var_rows_h, int nsplit_target, int align) {
  SplitPlan sp{};
  sp.nvars = nvars;
  int acc = 0;
  for (int v = 0; v < nvars; ++v) {
    sp.row0[v] = var_rows_h[v];
    sp.split0[v] = acc;
    const int64_t rows = var_rows_h[v + 1] - var_rows_h[v];
    int nv = int((double(nsplit_target) * double(rows) / double(n)) + 0.5);
    if (nv < 1) nv = 1;
    const int64_t max_nv = (rows + align - 1) / align;
    if (nv > max_nv) nv = int(max_nv);
    acc += nv;
  }
  sp.row0[nvars] = var_rows_h[nvars];
  sp.split0[nvars] = acc;
  sp.nsplit = acc;
  sp.xcd_map = (acc % 8 == 0) ? 1 : 0;
  return sp;
}

}  // namespace gramplan
}  // namespace dopinf
