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
// for this thread's stores to complete before its workgroup arrives.
//
// Arrivals are counted in two stages, so that no single word takes one atomic
// per workgroup (same-address atomics are serialised where the word lives,
// about 15 ns each: 2,048 arrivals on one word cost ~30 us). Workgroup b
// arrives on the counter of group b mod NG (NG = ceil(G / 32), at most 64;
// each counter in its own 128-byte line); the last arrival of a group
// arrives on the top counter, and the last of those publishes the round in a
// release word that every workgroup polls. Counters only grow within a
// launch (round r is complete at r * size), so nothing is cleared between
// rounds. The wait is bounded by the wall clock: returns false (in every
// thread) when it expired. Every thread of the workgroup must call it.
// Layout of the barrier block (kGridBarWords words, zero before the first
// launch): [0] top counter, [32] release word, [64] departures, [96 + 32 g]
// counter of group g.
constexpr int kGridBarGroups = 64;
constexpr int kGridBarWords = 96 + 32 * kGridBarGroups;

__device__ __forceinline__ unsigned grid_bar_groups() {
  const unsigned g = (gridDim.x + 31u) / 32u;
  return g < (unsigned)kGridBarGroups ? g : (unsigned)kGridBarGroups;
}

// The barrier in two halves, so that a workgroup can issue loads that do not
// depend on the round (the next level's indices and weights) between its
// arrival and its wait. grid_barrier_arrive: wait for this thread's memory
// operations, then one arrival per workgroup.
__device__ __forceinline__ void grid_barrier_arrive(unsigned *bar, unsigned round) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned G = gridDim.x, ng = grid_bar_groups(), g = blockIdx.x % ng;
    const unsigned size = G / ng + (g < G % ng ? 1u : 0u);
    const unsigned old = __hip_atomic_fetch_add(bar + 96 + 32 * g, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1u == round * size) {
      const unsigned top = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (top + 1u == round * ng) __hip_atomic_store(bar + 32, round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// grid_barrier_wait: every workgroup has arrived for `round` (false in every
// thread when the wall-clock limit expired first).
__device__ __forceinline__ bool grid_barrier_wait(unsigned *bar, unsigned round, unsigned long long t0,
                                                  unsigned long long tlimit, int *s_abort) {
  if (threadIdx.x == 0) {
    unsigned spins = 0;
    while (__hip_atomic_load(bar + 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < round) {
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

__device__ __forceinline__ bool grid_barrier(unsigned *bar, unsigned round, unsigned long long t0,
                                             unsigned long long tlimit, int *s_abort) {
  grid_barrier_arrive(bar, round);
  return grid_barrier_wait(bar, round, t0, tlimit, s_abort);
}

// End of a persistent launch that used grid_barrier: the last workgroup to
// leave clears the barrier block, so the launch can be replayed with no
// host-side reset. Every thread must call it.
__device__ __forceinline__ void grid_barrier_reset(unsigned *bar) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(bar + 64, 1u) == gridDim.x - 1) {
      const unsigned ng = grid_bar_groups();
      for (unsigned g = 0; g < ng; ++g) atomicExch(bar + 96 + 32 * g, 0u);
      atomicExch(bar, 0u);
      atomicExch(bar + 32, 0u);
      atomicExch(bar + 64, 0u);
      __threadfence();
    }
  }
}
