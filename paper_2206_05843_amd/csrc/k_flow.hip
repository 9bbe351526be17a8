// Dataflow runs (schedule mode 4): a run of consecutive wide levels solved in
// one persistent launch in which no level waits for the whole level before
// it. Each level is cut into chunks of consecutive positions (one
// workgroup's items). Chunk i of a level belongs to workgroup i mod G, and
// every workgroup walks the run's levels in order; a chunk waits only for the
// chunks of the same run that hold the rows its rows depend on (a list built
// with the schedule), so a workgroup whose next chunk's dependencies are done
// goes on while other parts of the level before are still being solved, and
// it requests the chunk's matrix entries and right-hand sides before it waits.
// Rows before the run were finished by earlier launches. The rows of a level
// are independent (Sec. II.A), so a chunk's rows are solved in parallel.
//
// Completion is a per-chunk word holding the launch's tag (epoch + 1); the
// epoch advances at the end of every launch, so the words never need
// clearing. A chunk's values of x are written and its dependencies' values
// read with device-scope atomic stores and loads (coherent across the dies'
// L2 caches without writing them back); its workgroup waits for its stores
// to complete before the word is set. A chunk depends only on chunks of
// earlier levels, and the grid is kept to the workgroups that are resident
// at once, so every workgroup reaches every level and every wait ends; waits
// are bounded by the wall clock all the same.
#include <algorithm>

#include "common.h"

namespace {

constexpr int kItems = 2;  // items (row, right-hand side) per thread in flight

template <int WG, bool kOne>
__global__ __launch_bounds__(WG) void k_flow_run(FlowArgs A, int32_t nlev, int32_t nrhs, int *err,
                                                 unsigned long long tlimit) {
  __shared__ int s_abort;
  const int tid = threadIdx.x;
  const int32_t nr = kOne ? 1 : nrhs;
  unsigned *ctl = A.ctl;  // [1] workgroups done, [2] epoch
  const unsigned tag = __hip_atomic_load(ctl + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
  const unsigned long long t0 = wall_clock64();
  if (tid == 0) s_abort = 0;
  __syncthreads();
  const int32_t run_p0 = A.chunk_pos[0];  // rows before the run are final
  const int32_t G = (int32_t)gridDim.x;
  int bits = 0;
  int32_t pos[kItems], cc[kItems], qb[kItems], deg[kItems];
  int4 ec[kItems];
  double2 e0[kItems], e1[kItems];
  double acc[kItems], dg[kItems];
  int32_t p0 = 0, items = 0;
  auto load_batch = [&](int32_t base) {
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const int32_t it = base + tid + j * WG;
      const int32_t itc = it < items ? it : items - 1;
      pos[j] = kOne ? p0 + itc : p0 + itc / nr;
      cc[j] = kOne ? 0 : itc - (pos[j] - p0) * nr;
      qb[j] = A.srp[pos[j]];
      deg[j] = it < items ? A.srp[pos[j] + 1] - qb[j] : 0;
      ec[j] = A.ell_c[pos[j]];
      e0[j] = A.ell_v[2 * (int64_t)pos[j]];
      e1[j] = A.ell_v[2 * (int64_t)pos[j] + 1];
      acc[j] = A.bp[(int64_t)pos[j] * nr + cc[j]];
      dg[j] = A.sdg[pos[j]];
    }
  };
  auto xload = [&](int32_t q, int32_t col) -> double {
    double *a = A.xp + (int64_t)q * nr + col;
    return q < run_p0 ? *a : __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  // chunk i of level l (of the run) belongs to workgroup i mod G, levels in order
  for (int32_t l = 0; l < nlev && !s_abort; ++l) {
    const int32_t cb = A.level_chunk[l], ce = A.level_chunk[l + 1];
    for (int32_t c = cb + (int32_t)blockIdx.x; c < ce; c += G) {
      p0 = A.chunk_pos[c];
      items = (A.chunk_pos[c + 1] - p0) * nr;
      // what does not depend on other chunks is requested before the wait
      load_batch(0);
      if (tid < 64) {  // one wave waits for the chunks this chunk reads
        const int32_t d0 = A.dptr[c], d1 = A.dptr[c + 1];
        unsigned spins = 0;
        for (int32_t i = d0 + tid; i < d1; i += 64) {
          const int32_t dc = A.dlist[i];
          while (__hip_atomic_load(A.flags + dc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != tag) {
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 255u) == 0u && wall_clock64() - t0 > tlimit) {
              s_abort = 1;
              break;
            }
          }
          if (s_abort) break;
        }
      }
      __syncthreads();
      if (s_abort) {
        bits |= EB_TIMEOUT;
        break;
      }
      // a chunk holds at most kItems * WG items unless one row has more
      // right-hand sides than that; then the items go in batches
      for (int32_t base = 0; base < items; base += kItems * WG) {
        if (base > 0) load_batch(base);
        double xv[kItems][4];
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
          const int32_t kk[4] = {ec[j].x, ec[j].y, ec[j].z, ec[j].w};
#pragma unroll
          for (int d = 0; d < 4; ++d) xv[j][d] = d < deg[j] ? xload(kk[d], cc[j]) : 0.0;
        }
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
          if (base + tid + j * WG >= items) continue;
          const double vv[4] = {e0[j].x, e0[j].y, e1[j].x, e1[j].y};
          double a = acc[j];
#pragma unroll
          for (int d = 0; d < 4; ++d)
            if (d < deg[j]) a -= vv[d] * xv[j][d];
          const int32_t qe = qb[j] + deg[j];
          for (int32_t q0 = qb[j] + 4; q0 < qe; q0 += 4) {  // dependencies beyond the first four, four at a time
            int32_t k4[4];
            double w4[4], x4[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              k4[d] = q0 + d < qe ? A.sci[q0 + d] : -1;
              w4[d] = q0 + d < qe ? A.sva[q0 + d] : 0.0;
            }
#pragma unroll
            for (int d = 0; d < 4; ++d) x4[d] = k4[d] >= 0 ? xload(k4[d], cc[j]) : 0.0;
#pragma unroll
            for (int d = 0; d < 4; ++d)
              if (k4[d] >= 0) a -= w4[d] * x4[d];
          }
          const double x = a / dg[j];
          if (!isfinite(x)) bits |= EB_NONFINITE;
          __hip_atomic_store(A.xp + (int64_t)pos[j] * nr + cc[j], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      __builtin_amdgcn_s_waitcnt(0);  // this thread's values of x have completed
      __syncthreads();
      if (tid == 0) __hip_atomic_store(A.flags + c, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (bits) atomicOr(err, bits);
  // the last workgroup to leave advances the epoch
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    if (atomicAdd(ctl + 1, 1u) == gridDim.x - 1) {
      atomicExch(ctl + 1, 0u);
      __hip_atomic_store(ctl + 2, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
    }
  }
}

template <int WG, bool kOne>
int resident(int dev) {
  int cus = 0, occ = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(&k_flow_run<WG, kOne>), WG,
                                                     0);
  return cus * (occ > 0 ? occ : 1);
}

}  // namespace

int flow_items_per_thread() { return kItems; }

hipError_t launch_flow_run(int wg, int grid, const FlowArgs &a, int32_t nlev, int32_t max_chunks, int32_t nrhs,
                           int *err, unsigned long long tlimit, hipStream_t s) {
  if (nlev <= 0 || max_chunks <= 0) return hipSuccess;
  static int cap[2][3] = {};
  int dev = 0;
  (void)hipGetDevice(&dev);
  const bool one = nrhs == 1;
  const int wi = wg == 128 ? 0 : wg == 256 ? 1 : 2;
  if (!cap[one][wi])
    cap[one][wi] = one ? (wg == 128 ? resident<128, true>(dev) : wg == 256 ? resident<256, true>(dev)
                                                                           : resident<512, true>(dev))
                       : (wg == 128 ? resident<128, false>(dev) : wg == 256 ? resident<256, false>(dev)
                                                                            : resident<512, false>(dev));
  int g = grid > 0 ? grid : cap[one][wi];
  g = std::max(1, std::min(g, std::min(cap[one][wi], max_chunks)));  // all resident: every level is reached
#define FLOW(W)                                                                                                 \
  if (one)                                                                                                      \
    hipLaunchKernelGGL((k_flow_run<W, true>), dim3(g), dim3(W), 0, s, a, nlev, nrhs, err, tlimit);              \
  else                                                                                                          \
    hipLaunchKernelGGL((k_flow_run<W, false>), dim3(g), dim3(W), 0, s, a, nlev, nrhs, err, tlimit);
  if (wg == 128) {
    FLOW(128)
  } else if (wg == 256) {
    FLOW(256)
  } else {
    FLOW(512)
  }
#undef FLOW
  return hipGetLastError();
}
