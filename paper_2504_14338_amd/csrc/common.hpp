// Shared helpers of libdopinf: status codes, the thread-local error message,
// argument checks and 64-lane wavefront reductions for gfx950.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/dopinf.h"

namespace dopinf {

// ---- error state ---------------------------------------------------------

void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

// ---- tuned launch parameters (tune.cpp) ------------------------------------
namespace tune {
int get(int param, int64_t key);  // 0 when untuned
void set(int param, int64_t key, int value);
bool persisted();  // DOPINF_TUNE_CACHE names a cache file
}  // namespace tune

#define DOPINF_HIP(call)                                                        \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      return ::dopinf::fail(DOPINF_E_HIP, "%s failed: %s (%s:%d)", #call,       \
                            hipGetErrorString(e_), __FILE__, __LINE__);         \
  } while (0)

#define DOPINF_LAUNCHED()                                                       \
  do {                                                                          \
    hipError_t e_ = hipGetLastError();                                          \
    if (e_ != hipSuccess)                                                       \
      return ::dopinf::fail(DOPINF_E_HIP, "kernel launch failed: %s (%s:%d)",   \
                            hipGetErrorString(e_), __FILE__, __LINE__);         \
  } while (0)

#define DOPINF_REQUIRE(cond, ...)                                               \
  do {                                                                          \
    if (!(cond)) return ::dopinf::fail(DOPINF_E_ARG, __VA_ARGS__);              \
  } while (0)

// Workspaces must be 256-byte aligned: blocks carved from them feed 16-byte
// vector and LDS-DMA loads and 8-byte atomics.  Checked before anything else,
// so a misaligned workspace returns with nothing enqueued.
#define DOPINF_REQUIRE_WS_ALIGNED(ws)                                                    \
  do {                                                                                   \
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)                                      \
      return ::dopinf::fail(DOPINF_E_WORKSPACE, "workspace must be 256-byte aligned");   \
  } while (0)

// ---- workspace carving -----------------------------------------------------

// Bump allocator over a caller-provided workspace; every block 256-B aligned.
struct Carver {
  char* base;
  size_t used = 0;
  size_t cap;
  Carver(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  bool ok() const { return used <= cap; }
};

__host__ __device__ inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---- device helpers --------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the 64 lanes with DPP moves inside each 16-lane row (quad swaps,
// then rotations by 4 and 8 lanes) and four lane reads across the rows; the
// result is the same in every lane and its rounding does not depend on the
// lane.  All 64 lanes must be active (wave-uniform control flow).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124>(v);  // row_ror:4
  v += dpp_move<0x128>(v);  // row_ror:8
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_move<0xB1>(v));
  v = fmax(v, dpp_move<0x4E>(v));
  v = fmax(v, dpp_move<0x124>(v));
  v = fmax(v, dpp_move<0x128>(v));
  return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum; every thread gets the total.  `red` holds >= nwaves doubles.
// Summation order is fixed (wave tree, then waves in index order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += red[i];
  return t;
}

__device__ __forceinline__ bool finite_d(double x) { return isfinite(x); }

}  // namespace dopinf
