// Grid-wide synchronization for persistent (cooperative) launches.
//
// Data passed between the phases of such a launch is read and written with
// device-scope relaxed atomics (ld_dev / st_dev): those are coherent across
// the XCDs, whose L2 caches are not coherent with each other for plain
// accesses, so the barrier itself needs no cache write-back or invalidation.
#pragma once

#include <hip/hip_runtime.h>

namespace hps {

__device__ inline double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two-level barrier: the workgroups count in at one of eight group counters
// (blockIdx mod 8, the XCD the dispatcher sends them to), the last of a
// group counts the group in at the top counter, and everyone polls the top
// counter.  bar[0] is the top counter, bar[1..8] the groups' (each in its
// own 128-byte line).
__device__ inline void grid_barrier(unsigned* bar, unsigned nblk, unsigned& gen, int* err) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    ++gen;
    const unsigned g = blockIdx.x & 7u;
    const unsigned gsize = nblk / 8 + (g < nblk % 8 ? 1u : 0u);
    const unsigned ngroups = nblk < 8 ? nblk : 8u;
    const unsigned old =
        __hip_atomic_fetch_add(bar + 32 * (1 + g), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == gen * gsize)
      __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = gen * ngroups;
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1u << 25)) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}

}  // namespace hps
