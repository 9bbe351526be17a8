// Device-side synchronisation primitives shared by the solve kernels and by
// the empty-level measurements that price them (k_floor.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

// Workgroup barrier that orders LDS only: global stores may still be in
// flight. Separates consecutive levels inside a thin run.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The same for a window run by a single wave: no workgroup barrier at all.
__device__ __forceinline__ void wave_lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Device-wide barrier number `round` (1, 2, ...) of a persistent launch whose
// gridDim.x workgroups are all resident. Values exchanged across it are
// written and read with device-scope atomic stores and loads (coherent across
// the dies' L2 caches without writing them back), so the barrier only waits
// for this thread's stores to complete, then counts one arrival per
// workgroup on bar[0] and waits for all of them. The wait is bounded by the
// wall clock: returns false (in every thread) when it expired. Every thread
// of the workgroup must call it.
__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned round, unsigned long long t0,
                                             unsigned long long tlimit, int *s_abort) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = round * gridDim.x;
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0u && wall_clock64() - t0 > tlimit) {
        *s_abort = 1;
        break;
      }
    }
  }
  __syncthreads();
  return *s_abort == 0;
}

// End of a persistent launch that used grid_barrier: the last workgroup to
// leave resets bar[0] and the departure count bar[1], so the launch can be
// replayed with no host-side reset. Every thread must call it.
__device__ __forceinline__ void grid_barrier_reset(unsigned *bar) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(bar + 1, 1u) == gridDim.x - 1) {
      atomicExch(bar, 0u);
      atomicExch(bar + 1, 0u);
      __threadfence();
    }
  }
}
