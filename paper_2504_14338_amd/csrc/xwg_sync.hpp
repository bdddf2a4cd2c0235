// Cross-workgroup communication for persistent (co-resident) kernels of
// libdopinf on gfx950.  All data shared between workgroups (and the flags
// that publish it) is written and read with relaxed device-scope atomics,
// which are coherent across the XCDs' L2 caches; a writer drains its memory
// counter (s_waitcnt) before it signals, so no cache-wide release/acquire
// fences are needed.  Every wait has a spin cap: a waiter that hits it raises
// a shared abort flag so that all workgroups leave and the host reports a
// timeout instead of a hang.
#pragma once

#include "common.hpp"

namespace dopinf {
namespace xwg {

constexpr long kSpinLimit = 1L << 30;  // polls before a wait gives up (seconds)

__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(__double_as_longlong(v)),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double* p) {
  return __longlong_as_double(static_cast<long long>(__hip_atomic_load(
      reinterpret_cast<unsigned long long*>(const_cast<double*>(p)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)));
}
__device__ __forceinline__ unsigned ld_flag(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Spin (thread 0) until *p >= target; false if the abort flag was raised or
// the spin cap was hit (then the abort flag is raised for everybody).
__device__ __forceinline__ bool wait_ge(unsigned* p, unsigned target, int* abort_flag, long spin_limit = kSpinLimit) {
  __shared__ int ok_sh;
  if (threadIdx.x == 0) {
    long spins = 0;
    int ok = 1;
    while (ld_flag(p) < target) {
      if ((++spins & 255) == 0) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || spins > spin_limit) {
          __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    ok_sh = ok;
  }
  __syncthreads();
  return ok_sh != 0;
}

// all threads: drain this workgroup's memory operations, then synchronize
__device__ __forceinline__ void drain_then_sync() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

// barrier of nblocks workgroups on one counter: arrive, wait for all arrivals
// of this round (gen counts the rounds passed by this workgroup)
__device__ __forceinline__ bool team_barrier(unsigned* bar, unsigned nblocks, unsigned& gen, int* abort_flag,
                                             long spin_limit = kSpinLimit) {
  drain_then_sync();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  ++gen;
  return wait_ge(bar, gen * nblocks, abort_flag, spin_limit);
}

}  // namespace xwg
}  // namespace dopinf
