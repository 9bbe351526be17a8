// The cost of an empty level under each way the solve separates levels
// (a level floor: what a level costs when it holds no work), measured on the
// device with the same synchronisation the solve kernels use:
//  * a level inside a thin run: an LDS-only workgroup barrier (or, in a
//    one-wave window, none) and one dependent LDS read and write, as phase 2
//    does per level;
//  * a kernel launch per level, on a stream and as a node of a hipGraph;
//  * a device-wide barrier of a persistent launch over resident workgroups;
//  * a value handed from one workgroup to the next through a device-coherent
//    store and load (what every dependency hop of the synchronisation-free
//    executor needs at least).
#include <algorithm>
#include <vector>

#include "common.h"
#include "sync.h"

namespace {

constexpr int kLevels = 4096;  // empty levels per in-kernel measurement

template <int WG, bool kOneWave>
__global__ __launch_bounds__(WG) void k_floor_thin(int32_t nlev, unsigned long long *ticks, double *sink) {
  __shared__ double v[WG];
  const int tid = threadIdx.x;
  v[tid] = (double)tid;
  __syncthreads();
  const unsigned long long t0 = wall_clock64();
  for (int32_t l = 0; l < nlev; ++l) {
    // every level reads a value another thread wrote in the level before
    const double a = v[(tid + 1) % (kOneWave ? 64 : WG)];
    if (kOneWave) {
      wave_lds_barrier();
    } else {
      lds_barrier();
    }
    v[tid] = a + 1.0;
    if (kOneWave) {
      wave_lds_barrier();
    } else {
      lds_barrier();
    }
  }
  const unsigned long long t1 = wall_clock64();
  if (tid == 0) {
    ticks[0] = t1 - t0;
    sink[blockIdx.x] = v[0];
  }
}

__global__ void k_empty(int *p) {
  if (p && threadIdx.x == 1024) *p = 0;  // never true: keeps the launch
}

__global__ __launch_bounds__(256) void k_floor_grid(int32_t rounds, unsigned *bar, unsigned long long *ticks, int *err,
                                                    unsigned long long tlimit) {
  __shared__ int s_abort;
  if (threadIdx.x == 0) s_abort = 0;
  const unsigned long long t0 = wall_clock64();
  for (int32_t r = 1; r <= rounds; ++r)
    if (!grid_barrier(bar, (unsigned)r, t0, tlimit, &s_abort)) {
      if (threadIdx.x == 0) atomicOr(err, EB_TIMEOUT);
      break;
    }
  const unsigned long long t1 = wall_clock64();
  if (blockIdx.x == 0 && threadIdx.x == 0) ticks[0] = t1 - t0;
  grid_barrier_reset(bar);
}

// A chain of hand-overs: the workgroup with ticket k waits until word k - 1
// holds the launch's tag, then publishes its own; ticks = time from the first
// publication to the last.
__global__ __launch_bounds__(64) void k_floor_hop(unsigned *words, unsigned *ticket, unsigned tag,
                                                  unsigned long long *ticks, int *err, unsigned long long tlimit) {
  if (threadIdx.x != 0) return;
  const unsigned k = atomicAdd(ticket, 1u);
  const unsigned long long t0 = wall_clock64();
  if (k > 0) {
    unsigned spins = 0;
    while (__hip_atomic_load(words + k - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tag) {
      if ((++spins & 255u) == 0u && wall_clock64() - t0 > tlimit) {
        atomicOr(err, EB_TIMEOUT);
        break;
      }
    }
  }
  const unsigned long long t = wall_clock64();
  __hip_atomic_store(words + k, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (k == 0) ticks[0] = t;
  if (k == gridDim.x - 1) ticks[1] = t;
}

}  // namespace

extern "C" {

sptrsv_status_t sptrsv_measure_level_costs(sptrsv_handle_t h, hipStream_t s, sptrsv_level_costs_t *out) {
  if (!h || !out) return SPTRSV_ERR_ARG;
  h->last_error.clear();
  *out = sptrsv_level_costs_t{};
  const double ns_per_tick = 10.0;  // the 100 MHz device wall clock
  DArr<unsigned long long> ticks;
  DArr<double> sink;
  DArr<unsigned> words;
  HIPCHK(h, ticks.alloc(4));
  HIPCHK(h, sink.alloc(4));
  const unsigned long long limit = 100000000ull * 2;  // 2 s
  int *err = h->d_err.p;
  unsigned long long ht[2];
  // thin-run levels: warm-up launch, then the measured one
  for (int rep = 0; rep < 2; ++rep)
    hipLaunchKernelGGL((k_floor_thin<1024, false>), dim3(1), dim3(1024), 0, s, kLevels, ticks.p, sink.p);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(ht, ticks.p, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  out->thin_level_ns = (double)ht[0] * ns_per_tick / kLevels;
  for (int rep = 0; rep < 2; ++rep)
    hipLaunchKernelGGL((k_floor_thin<64, true>), dim3(1), dim3(64), 0, s, kLevels, ticks.p, sink.p);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemcpyAsync(ht, ticks.p, 8, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  out->thin_wave_level_ns = (double)ht[0] * ns_per_tick / kLevels;
  // a launch per level, on the stream
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  constexpr int kLaunches = 2000;
  for (int i = 0; i < 100; ++i) hipLaunchKernelGGL(k_empty, dim3(64), dim3(256), 0, s, (int *)nullptr);
  (void)hipEventRecord(e0, s);
  for (int i = 0; i < kLaunches; ++i) hipLaunchKernelGGL(k_empty, dim3(64), dim3(256), 0, s, (int *)nullptr);
  (void)hipEventRecord(e1, s);
  HIPCHK(h, hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
  out->launch_ns = (double)ms * 1e6 / kLaunches;
  // a node per level of a replayed graph (captured on a stream of its own)
  {
    hipStream_t cs = nullptr;
    HIPCHK(h, hipStreamCreate(&cs));
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      for (int i = 0; i < kLaunches; ++i) hipLaunchKernelGGL(k_empty, dim3(64), dim3(256), 0, cs, (int *)nullptr);
      e = hipStreamEndCapture(cs, &g);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(ge, cs);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, cs);
    if (e == hipSuccess) e = hipGraphLaunch(ge, cs);
    if (e == hipSuccess) e = hipEventRecord(e1, cs);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return set_err(h, SPTRSV_ERR_HIP, "graph timing: %s", hipGetErrorString(e));
    out->graph_node_ns = (double)ms * 1e6 / kLaunches;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // a device-wide barrier over every workgroup the persistent wide runs keep resident
  {
    const int grid = std::max(1, wide_run_resident_blocks(256));
    HIPCHK(h, words.alloc(kGridBarWords));
    HIPCHK(h, hipMemsetAsync(words.p, 0, kGridBarWords * sizeof(unsigned), s));
    constexpr int kRounds = 1000;
    for (int rep = 0; rep < 2; ++rep)
      hipLaunchKernelGGL(k_floor_grid, dim3(grid), dim3(256), 0, s, kRounds, words.p, ticks.p, err, limit);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(ht, ticks.p, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    out->grid_barrier_ns = (double)ht[0] * ns_per_tick / kRounds;
  }
  // hand-overs between workgroups (all resident: one 64-thread workgroup per slot)
  {
    constexpr int kHops = 1024;
    HIPCHK(h, words.alloc(kHops + 1));
    HIPCHK(h, hipMemsetAsync(words.p, 0, (kHops + 1) * sizeof(unsigned), s));
    for (unsigned tag = 1; tag <= 2; ++tag) {
      HIPCHK(h, hipMemsetAsync(words.p + kHops, 0, sizeof(unsigned), s));
      hipLaunchKernelGGL(k_floor_hop, dim3(kHops), dim3(64), 0, s, words.p, words.p + kHops, tag, ticks.p, err, limit);
    }
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(ht, ticks.p, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    out->flag_hop_ns = (double)(ht[1] - ht[0]) * ns_per_tick / (kHops - 1);
  }
  return sptrsv_check(h, s);
}

}  // extern "C"
