// Exchanges between workgroups of one launch without cache maintenance.
//
// Data another workgroup reads is written with device-scope relaxed atomic
// stores, which complete at the device's coherence point, and read with
// device-scope relaxed atomic loads, which are served from it.  A writer
// waits for its stores to complete (stores_done) before it publishes a flag or
// takes a ticket; a reader issues its data loads only after it has seen that
// flag or ticket value, behind a compiler fence.  Agent-scope acquire/release
// fences would order the same accesses with an L2 writeback or invalidation
// per workgroup, which serialises within each XCD.
#pragma once

#include <hip/hip_runtime.h>

namespace ds {

__device__ __forceinline__ long long ld_dev(const long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_dev(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(long long *p, long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(unsigned *p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// This wave's earlier stores have completed before anything after this point.
__device__ __forceinline__ void stores_done() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}

// Loads after this point are not moved above the flag or ticket access before it.
__device__ __forceinline__ void after_flag() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup"); }

// True in exactly one workgroup of the grid: the last to arrive.  Every
// workgroup's st_dev stores made before the call are visible to ld_dev loads
// of the elected workgroup after it.  The ticket returns to 0 for the next
// launch.  Called by all threads of the workgroup.
__device__ __forceinline__ bool last_arrival(unsigned *ticket) {
  __shared__ int last_sh;
  stores_done();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool last = prev == gridDim.x - 1;
    if (last) st_dev(ticket, 0u);
    last_sh = last ? 1 : 0;
  }
  __syncthreads();
  after_flag();
  return last_sh != 0;
}

}  // namespace ds
