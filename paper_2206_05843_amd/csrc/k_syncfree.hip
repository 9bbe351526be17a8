// Synchronisation-free forward substitution (Algorithm 1 without level
// barriers): every (row, right-hand side) item waits only for the x values it
// reads. It is the comparison executor for the level-set schedules, and a
// schedule the autotuner can pick (mode 3).
//
// Items are taken in level order (positions of the level-ordered copy) from a
// ticket counter, 64 per wave; a row's dependencies sit at smaller positions,
// so they were claimed earlier by a running wave and every wait ends. x starts
// as a signalling-NaN pattern that arithmetic never produces (division quiets
// every NaN), so one device-coherent 64-bit load returns both "done" and the
// value (a plain load is tried first and trusted when it is not the pending
// pattern). A lane requests its next four dependencies' values at once and takes
// the ready ones in column order, so the sum keeps the row's order; while it
// waits on a batch it keeps the batch's columns and weights in registers and
// polls past the caches directly, so a pass costs one memory round trip. A wave
// none of whose lanes moved in an iteration sleeps briefly before it polls
// again, and the launch is kept to a few thousand waves: the waiting lanes'
// polling otherwise saturates the memory system and slows every hop (on a
// 4M-row power-law matrix, 8,192 waves without the pause ran past the time
// limit; 2,048 waves with it solve in 5 ms). Waits are bounded by the device
// wall clock (timeout error).
#include "common.h"

namespace {

constexpr unsigned long long kPending = 0x7ff4dead5eed5a1dull;
constexpr int kBlock = 256;
constexpr int kDeps = 4;  // dependencies requested together (6 or 8 were slower)
// pause of a wave none of whose lanes moved, in units of 64 cycles: on the 2D
// stencil + chain 4 took 1.49 ms per solve against 1.52 with 8 and 1.58 with 16
// (2: 1.48, but slower on the power law)
constexpr int kSleep = 4;

__global__ void k_sf_init(int64_t total, unsigned long long *xb, unsigned long long *ticket) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    xb[i] = kPending;
  if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0ull;
}

template <bool kOne, bool kStamp>
__global__ __launch_bounds__(kBlock) void k_sf_solve(int32_t n, int32_t nrhs, const int32_t *__restrict__ srp,
                                                     const int32_t *__restrict__ sci, const double *__restrict__ sva,
                                                     const double *__restrict__ sdg, const double *__restrict__ bp,
                                                     double *xp, unsigned long long *ticket, int *err,
                                                     unsigned long long tlimit, unsigned long long *stamp) {
  const int lane = threadIdx.x & 63;
  const int32_t nr = kOne ? 1 : nrhs;
  const int64_t total = (int64_t)n * nr;
  unsigned long long *xb = reinterpret_cast<unsigned long long *>(xp);
  const unsigned long long t0 = wall_clock64();
  int bits = 0;
  bool timed_out = false;
  while (!timed_out) {
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(ticket, 64ull);
    base = __shfl(base, 0, 64);
    if ((int64_t)base >= total) break;
    const int64_t it = (int64_t)base + lane;
    bool pend = it < total;
    int32_t q = 0, qe = 0, c = 0;
    double acc = 0.0, d = 1.0;
    if (pend) {
      const int32_t pos = kOne ? (int32_t)it : (int32_t)(it / nr);
      c = kOne ? 0 : (int32_t)(it - (int64_t)pos * nr);
      q = srp[pos];
      qe = srp[pos + 1];
      acc = bp[it];
      d = sdg[pos];
    }
    unsigned spins = 0;
    bool seen_pending = false;  // the dependency at q read as pending in the last pass
    int32_t k[kDeps];           // columns and weights of the batch at kq, kept across passes
    double w[kDeps];
    int32_t kq = -1;
    while (__ballot(pend) != 0ull) {
      bool moved = false;
      if (pend) {
        const int32_t q_in = q;
        bool first = true;
        while (q < qe) {
          const int32_t cnt = qe - q < kDeps ? qe - q : kDeps;
          unsigned long long v[kDeps];
          if (q != kq) {  // a new batch: its columns and weights
#pragma unroll
            for (int j = 0; j < kDeps; ++j) {
              const int32_t qq = q + (j < cnt ? j : 0);
              k[j] = sci[qq];
              w[j] = sva[qq];
            }
            kq = q;
          }
          // a plain (cached) load first: it returns either the pending
          // pattern or the final value, since caches hold no line of x from
          // before this launch (the fill kernel ran in between) and every
          // value is written once; only what still reads as pending is
          // fetched again past the caches. A batch whose first dependency
          // read as pending in the last pass goes past the caches at once
          // (its cached line can only say pending again).
          if (first && seen_pending) {
#pragma unroll
            for (int j = 0; j < kDeps; ++j)
              v[j] = __hip_atomic_load(xb + (int64_t)k[j] * nr + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else {
#pragma unroll
            for (int j = 0; j < kDeps; ++j) v[j] = xb[(int64_t)k[j] * nr + c];
#pragma unroll
            for (int j = 0; j < kDeps; ++j)
              if (v[j] == kPending)
                v[j] = __hip_atomic_load(xb + (int64_t)k[j] * nr + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          first = false;
          int32_t done = 0;
#pragma unroll
          for (int j = 0; j < kDeps; ++j) {
            if (j < cnt && done == j && v[j] != kPending) {
              acc -= w[j] * __longlong_as_double((long long)v[j]);
              done = j + 1;
            }
          }
          q += done;
          seen_pending = done < cnt;
          if (seen_pending) break;  // a dependency is still pending
        }
        moved = q != q_in;
        if (q == qe) {
          const double x = acc / d;
          if (!isfinite(x)) bits |= EB_NONFINITE;
          __hip_atomic_store(xb + it, (unsigned long long)__double_as_longlong(x), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          if (kStamp) stamp[it] = wall_clock64();  // when this item's value was written
          pend = false;
          moved = true;
        }
      }
      if (__ballot(moved) == 0ull) __builtin_amdgcn_s_sleep(kSleep);
      if ((++spins & 63u) == 0u && wall_clock64() - t0 > tlimit) {
        bits |= EB_TIMEOUT;
        timed_out = true;
        break;
      }
    }
  }
  if (bits) atomicOr(err, bits);
}

// Per-level finish times of a stamped solve: the latest stamp of each level's
// items and the earliest stamp of all (atomicMin), then the levels' latest
// stamps relative to that earliest one, in ns.
__global__ void k_stamp_level_max(int32_t nlev, int32_t nrhs, const int32_t *__restrict__ level_ptr,
                                  const unsigned long long *__restrict__ stamp, unsigned long long *lmax,
                                  unsigned long long *gmin) {
  __shared__ unsigned long long s_hi[4], s_lo[4];
  for (int32_t l = blockIdx.x; l < nlev; l += gridDim.x) {
    const int64_t i0 = (int64_t)level_ptr[l] * nrhs, i1 = (int64_t)level_ptr[l + 1] * nrhs;
    unsigned long long hi = 0ull, lo = ~0ull;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      const unsigned long long t = stamp[i];
      hi = t > hi ? t : hi;
      lo = t < lo ? t : lo;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long h2 = __shfl_xor(hi, o, 64), l2 = __shfl_xor(lo, o, 64);
      hi = h2 > hi ? h2 : hi;
      lo = l2 < lo ? l2 : lo;
    }
    if ((threadIdx.x & 63) == 0) {
      s_hi[threadIdx.x >> 6] = hi;
      s_lo[threadIdx.x >> 6] = lo;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
        hi = s_hi[w] > hi ? s_hi[w] : hi;
        lo = s_lo[w] < lo ? s_lo[w] : lo;
      }
      lmax[l] = hi;
      atomicMin(gmin, lo);
    }
    __syncthreads();
  }
}

__global__ void k_stamp_finish(int32_t nlev, const unsigned long long *__restrict__ lmax,
                               const unsigned long long *__restrict__ gmin, float ns_per_tick, float *times) {
  for (int32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < nlev; l += gridDim.x * blockDim.x)
    times[l] = (float)(lmax[l] - *gmin) * ns_per_tick;
}

}  // namespace

hipError_t launch_syncfree(int32_t n, int32_t nrhs, const int32_t *srp, const int32_t *sci, const double *sva,
                           const double *sdg, const double *bp, double *xp, unsigned long long *ticket, int *err,
                           int32_t blocks, unsigned long long limit, hipStream_t s, unsigned long long *stamp) {
  if (n == 0) return hipSuccess;
  const int64_t total = (int64_t)n * nrhs;
  unsigned long long *xb = reinterpret_cast<unsigned long long *>(xp);
  hipLaunchKernelGGL(k_sf_init, dim3(grid_for(total, kBlock, 8192)), dim3(kBlock), 0, s, total, xb, ticket);
  const dim3 grid(grid_for(total, kBlock, blocks > 0 ? blocks : 512));
#define SF(ONE, ST)                                                                                               \
  hipLaunchKernelGGL((k_sf_solve<ONE, ST>), grid, dim3(kBlock), 0, s, n, nrhs, srp, sci, sva, sdg, bp, xp, ticket, \
                     err, limit, stamp)
  if (stamp) {
    if (nrhs == 1)
      SF(true, true);
    else
      SF(false, true);
  } else if (nrhs == 1) {
    SF(true, false);
  } else {
    SF(false, false);
  }
#undef SF
  return hipGetLastError();
}

hipError_t launch_stamp_levels(int32_t nlev, int32_t nrhs, const int32_t *level_ptr, const unsigned long long *stamp,
                               unsigned long long *lmax, unsigned long long *gmin, float ns_per_tick, float *times,
                               hipStream_t s) {
  if (nlev <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stamp_level_max, dim3(nlev < 4096 ? nlev : 4096), dim3(256), 0, s, nlev, nrhs, level_ptr,
                     stamp, lmax, gmin);
  hipLaunchKernelGGL(k_stamp_finish, dim3((nlev + 255) / 256), dim3(256), 0, s, nlev, lmax, gmin, ns_per_tick, times);
  return hipGetLastError();
}
