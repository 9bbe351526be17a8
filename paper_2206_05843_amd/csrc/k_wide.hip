// Wide-level solve kernels: the rows of one level of the level-ordered L (or
// L') are independent (Sec. II.A), so a wide level is spread over the whole
// device. Either one launch per level (kernel boundaries order the levels), or
// one persistent launch for a run of consecutive wide levels with a
// device-wide barrier between levels.
#include "common.h"
#include "sync.h"

namespace {

// Workgroups are dealt to the eight dies (XCDs, each with its own L2) in
// turn: workgroup b runs on die b mod 8. A wide level launch renumbers them
// so that each die takes one contiguous slice of the level (a bijection of
// the workgroup indices): the rows that read one x value (neighbours in the
// level order) then mostly sit on the die that fetched it into its L2 (1.8 %
// faster on the 3D stencil with 32 right-hand sides).
__device__ inline int32_t wide_block() {
  const int32_t nb = (int32_t)gridDim.x, b = (int32_t)blockIdx.x;
  const int32_t q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// One wide level, items (row, rhs) spread over the device (two per thread in
// flight with one right-hand side, one with several: 1.6 % faster on the 3D
// stencil with 32): a row's first four dependencies come from the fixed-width copy
// indexed by position (no row pointer on the load chain), the rest from the
// CSR four at a time; all loads of a step are issued before they are used and
// the products are subtracted in the row's column order.
template <bool kOne>
__global__ void k_wide_level(int32_t pb, int32_t pe, int32_t nrhs, const int32_t *__restrict__ srp,
                             const int32_t *__restrict__ sci, const double *__restrict__ sva,
                             const double *__restrict__ sdg, const int4 *__restrict__ ell_c,
                             const double2 *__restrict__ ell_v, const double *__restrict__ bp, double *xp, int *err,
                             RowsIO rio) {
  constexpr int kI = kOne ? 2 : 1;  // several right-hand sides: one item per thread spreads a level wider
  const int32_t nr = kOne ? 1 : nrhs;
  const int64_t items = (int64_t)(pe - pb) * nr;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bits = 0;
  for (int64_t base = (int64_t)wide_block() * blockDim.x + threadIdx.x; base < items; base += stride * kI) {
    int32_t pos[kI], c[kI], qb[kI], deg[kI], row[kI];
    int4 ec[kI];
    double2 e0[kI], e1[kI];
    double acc[kI], dg[kI];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int64_t it = base + j * stride;
      const int64_t itc = it < items ? it : items - 1;
      pos[j] = kOne ? pb + (int32_t)itc : pb + (int32_t)(itc / nr);
      c[j] = kOne ? 0 : (int32_t)(itc - (int64_t)(pos[j] - pb) * nr);
      qb[j] = srp[pos[j]];
      deg[j] = it < items ? srp[pos[j] + 1] - qb[j] : 0;
      ec[j] = rio.x ? rio.ell_r[pos[j]] : ell_c[pos[j]];
      e0[j] = ell_v[2 * (int64_t)pos[j]];
      e1[j] = ell_v[2 * (int64_t)pos[j] + 1];
      row[j] = rio.b ? rio.perm[pos[j]] : 0;
      // right-hand sides stored by rows: the caller's b through the level
      // order, except rows of T with off-diagonals (b' in bp)
      if (rio.b && !(rio.tflag && rio.tflag[pos[j]]))
        acc[j] = rio.b[(int64_t)row[j] * nr + c[j]];
      else
        acc[j] = bp[(int64_t)pos[j] * nr + c[j]];
      dg[j] = sdg[pos[j]];
    }
    // by rows the caller's x is the work vector: dependencies as caller rows
    const double *xs = rio.x ? rio.x : xp;
    double xv[kI][4];
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      const int32_t kk[4] = {ec[j].x, ec[j].y, ec[j].z, ec[j].w};
#pragma unroll
      for (int d = 0; d < 4; ++d) xv[j][d] = d < deg[j] ? xs[(int64_t)kk[d] * nr + c[j]] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kI; ++j) {
      if (base + j * stride >= items) continue;
      const double vv[4] = {e0[j].x, e0[j].y, e1[j].x, e1[j].y};
      double a = acc[j];
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (d < deg[j]) a -= vv[d] * xv[j][d];
      const int32_t qe = qb[j] + deg[j];
      const int32_t *cols = rio.x ? rio.sci_r : sci;  // by rows: columns as caller rows
      for (int32_t q0 = qb[j] + 4; q0 < qe; q0 += 4) {
        int32_t k4[4];
        double w4[4], x4[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          k4[d] = q0 + d < qe ? cols[q0 + d] : -1;
          w4[d] = q0 + d < qe ? sva[q0 + d] : 0.0;
        }
#pragma unroll
        for (int d = 0; d < 4; ++d) x4[d] = k4[d] >= 0 ? xs[(int64_t)k4[d] * nr + c[j]] : 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d)
          if (k4[d] >= 0) a -= w4[d] * x4[d];
      }
      const double x = a / dg[j];
      if (!isfinite(x)) bits |= EB_NONFINITE;
      if (rio.x)
        rio.x[(int64_t)row[j] * nr + c[j]] = x;
      else
        xp[(int64_t)pos[j] * nr + c[j]] = x;
    }
  }
  if (bits) atomicOr(err, bits);
}

// One wide level, single RHS, G lanes per row: lanes split the row's products
// and combine them with a fixed butterfly, so the result is deterministic.
template <int G>
__global__ void k_wide_level_group(int32_t pb, int32_t pe, const int32_t *__restrict__ srp,
                                   const int32_t *__restrict__ sci, const double *__restrict__ sva,
                                   const double *__restrict__ sdg, const double *__restrict__ bp, double *xp,
                                   int *err) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sub = threadIdx.x & (G - 1);
  int bits = 0;
  const int64_t rows = pe - pb;
  for (int64_t rr = gid / G; rr < (rows + 0); rr += ((int64_t)gridDim.x * blockDim.x) / G) {
    const int32_t pos = pb + (int32_t)rr;
    double acc = 0.0;
    const int32_t b = srp[pos], e = srp[pos + 1];
    for (int32_t q = b + sub; q < e; q += G) acc -= sva[q] * xp[sci[q]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
    if (sub == 0) {
      const double xv = (bp[pos] + acc) / sdg[pos];
      if (!isfinite(xv)) bits |= EB_NONFINITE;
      xp[pos] = xv;
    }
  }
  if (bits) atomicOr(err, bits);
}

// One wide level whose rows have many dependencies, with several right-hand
// sides: one workgroup per row. Its threads form G = WG / nrhs groups of nrhs
// lanes (lane c takes column c, so a group's loads of one dependency's x are
// contiguous); group g sums the row's products g, g + G, g + 2G, ... for its
// column, four requested at a time, and the G partial sums are added in group
// order, so the result does not depend on timing (it is not the row's column
// order, so it can differ from the other executors in the last bits).
template <int WG>
__global__ __launch_bounds__(WG) void k_wide_long(int32_t pb, int32_t nrhs, const int32_t *__restrict__ srp,
                                                  const int32_t *__restrict__ sci, const double *__restrict__ sva,
                                                  const double *__restrict__ sdg, const double *__restrict__ bp,
                                                  double *xp, int *err, RowsIO rio) {
  __shared__ double part[WG];
  const int32_t nr = nrhs;
  const int32_t G = WG / nr;  // the host keeps nrhs <= WG
  const int32_t t = (int32_t)threadIdx.x, g = t / nr, c = t - g * nr;
  const int32_t pos = pb + (int32_t)blockIdx.x;
  const int32_t qb = srp[pos], qe = srp[pos + 1];
  const int32_t *cols = rio.x ? rio.sci_r : sci;  // by rows: columns as caller rows
  const double *xs = rio.x ? rio.x : xp;
  const int32_t row = rio.b ? rio.perm[pos] : 0;
  double bv = 0.0;
  if (g == 0) {
    if (rio.b && !(rio.tflag && rio.tflag[pos]))
      bv = rio.b[(int64_t)row * nr + c];
    else
      bv = bp[(int64_t)pos * nr + c];
  }
  double acc = 0.0;
  if (g < G) {
    for (int32_t q0 = qb + g; q0 < qe; q0 += 4 * G) {
      int32_t k[4];
      double w[4], xv[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const int32_t q = q0 + d * G;
        k[d] = q < qe ? cols[q] : -1;
        w[d] = q < qe ? sva[q] : 0.0;
      }
#pragma unroll
      for (int d = 0; d < 4; ++d) xv[d] = k[d] >= 0 ? xs[(int64_t)k[d] * nr + c] : 0.0;
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (k[d] >= 0) acc += w[d] * xv[d];
    }
  }
  part[t] = acc;
  __syncthreads();
  if (g == 0) {
    double sum = part[c];
    for (int32_t gg = 1; gg < G; ++gg) sum += part[gg * nr + c];
    const double x = (bv - sum) / sdg[pos];
    if (!isfinite(x)) atomicOr(err, EB_NONFINITE);
    if (rio.x)
      rio.x[(int64_t)row * nr + c] = x;
    else
      xp[(int64_t)pos * nr + c] = x;
  }
}

// What one item (row, right-hand side) of a wide level needs apart from the
// x values it reads: position, column, CSR range, the fixed-width copy of its
// first four dependencies, its b (or b'), the diagonal and the caller's row.
struct WideItem {
  int32_t pos, c, qb, deg, row;
  int4 ec;
  double2 e0, e1;
  double acc, dg;
};

template <bool kOne>
__device__ __forceinline__ void wide_fetch(int64_t it, int32_t pb, int32_t nr, const int32_t *__restrict__ srp,
                                           const double *__restrict__ sdg, const int4 *__restrict__ ell_c,
                                           const double2 *__restrict__ ell_v, const double *__restrict__ bp,
                                           const RowsIO &rio, WideItem &w) {
  w.pos = kOne ? pb + (int32_t)it : pb + (int32_t)(it / nr);
  w.c = kOne ? 0 : (int32_t)(it - (int64_t)(w.pos - pb) * nr);
  w.qb = srp[w.pos];
  w.deg = srp[w.pos + 1] - w.qb;
  w.ec = rio.x ? rio.ell_r[w.pos] : ell_c[w.pos];
  w.e0 = ell_v[2 * (int64_t)w.pos];
  w.e1 = ell_v[2 * (int64_t)w.pos + 1];
  w.row = rio.b ? rio.perm[w.pos] : 0;
  if (rio.b && !(rio.tflag && rio.tflag[w.pos]))
    w.acc = rio.b[(int64_t)w.row * nr + w.c];
  else
    w.acc = bp[(int64_t)w.pos * nr + w.c];
  w.dg = sdg[w.pos];
}

// Solves the fetched items: the x values they read (device-coherent loads,
// since other workgroups of the launch wrote them), all requested before
// they are used, subtracted in the row's column order; x stored coherently
// (and to the caller's x by rows).
template <int kK>
__device__ __forceinline__ void wide_solve(const WideItem (&w)[kK], const bool (&ok)[kK], int32_t nr,
                                           const int32_t *__restrict__ sci, const double *__restrict__ sva,
                                           double *xp, const RowsIO &rio, int &bits) {
  double *xs = rio.x ? rio.x : xp;  // by rows the caller's x is the work vector
  double xv[kK][4];
#pragma unroll
  for (int j = 0; j < kK; ++j) {
    const int32_t kk[4] = {w[j].ec.x, w[j].ec.y, w[j].ec.z, w[j].ec.w};
#pragma unroll
    for (int d = 0; d < 4; ++d)
      xv[j][d] = ok[j] && d < w[j].deg ? __hip_atomic_load(xs + (int64_t)kk[d] * nr + w[j].c, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)
                                        : 0.0;
  }
#pragma unroll
  for (int j = 0; j < kK; ++j) {
    if (!ok[j]) continue;
    const double vv[4] = {w[j].e0.x, w[j].e0.y, w[j].e1.x, w[j].e1.y};
    double a = w[j].acc;
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if (d < w[j].deg) a -= vv[d] * xv[j][d];
    // dependencies beyond the first four, four at a time, in column order
    // (prefetching the next four's columns and weights here cost registers,
    // and with them resident waves, on every level)
    const int32_t qe = w[j].qb + w[j].deg;
    const int32_t *cols = rio.x ? rio.sci_r : sci;  // by rows: columns as caller rows
    for (int32_t q0 = w[j].qb + 4; q0 < qe; q0 += 4) {
      int32_t k4[4];
      double w4[4], x4[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        k4[d] = q0 + d < qe ? cols[q0 + d] : -1;
        w4[d] = q0 + d < qe ? sva[q0 + d] : 0.0;
      }
#pragma unroll
      for (int d = 0; d < 4; ++d)
        x4[d] = k4[d] >= 0 ? __hip_atomic_load(xs + (int64_t)k4[d] * nr + w[j].c, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT)
                           : 0.0;
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (k4[d] >= 0) a -= w4[d] * x4[d];
    }
    const double x = a / w[j].dg;
    if (!isfinite(x)) bits |= EB_NONFINITE;
    __hip_atomic_store(xs + (int64_t)(rio.x ? w[j].row : w[j].pos) * nr + w[j].c, x, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Consecutive wide levels [l0, l1) in one launch of gridDim.x workgroups,
// which must all be resident at once (the host sizes the grid from the
// occupancy): every level's items are spread over all threads, and levels are
// separated by a device-wide barrier. Inside the launch x is written and read
// with device-scope atomic stores and loads, which are coherent across the
// dies' separate L2 caches without writing back or invalidating them. Nothing
// but the x values depends on the previous level, so each thread fetches the
// next level's first kK items (indices, weights, b, diagonal) between its
// workgroup's arrival at the barrier and the wait for the others: after the
// barrier only the loads of x remain on a level's chain. Items beyond kK per
// thread are fetched and solved in a loop after those. Waits are bounded by
// the wall clock: on expiry the launch stops and reports a time-out instead of
// hanging. The last workgroup to leave resets the barrier block, so the
// launch can be replayed with no host-side reset.
template <bool kOne>
__global__ void k_wide_run(int32_t l0, int32_t l1, const int32_t *__restrict__ level_ptr, int32_t nrhs,
                           const int32_t *__restrict__ srp, const int32_t *__restrict__ sci,
                           const double *__restrict__ sva, const double *__restrict__ sdg,
                           const int4 *__restrict__ ell_c, const double2 *__restrict__ ell_v,
                           const double *__restrict__ bp, double *xp, unsigned *bar, int *err,
                           unsigned long long tlimit, RowsIO rio) {
  constexpr int kK = 2;  // 1 was as fast; 3 lowers the occupancy, 4 spills
  __shared__ int s_abort;
  const int32_t nr = kOne ? 1 : nrhs;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (threadIdx.x == 0) s_abort = 0;
  const unsigned long long t0 = wall_clock64();
  int bits = 0;
  int32_t pb = level_ptr[l0], pe = level_ptr[l0 + 1];
  WideItem w[kK];
  bool ok[kK];
#pragma unroll
  for (int j = 0; j < kK; ++j) {
    const int64_t it = gid + j * nthreads;
    ok[j] = it < (int64_t)(pe - pb) * nr;
    if (ok[j]) wide_fetch<kOne>(it, pb, nr, srp, sdg, ell_c, ell_v, bp, rio, w[j]);
  }
  for (int32_t l = l0; l < l1; ++l) {
    const int32_t ne = l + 1 < l1 ? level_ptr[l + 2] : pe;  // end of the next level
    const int64_t items = (int64_t)(pe - pb) * nr;
    wide_solve<kK>(w, ok, nr, sci, sva, xp, rio, bits);
    for (int64_t it = gid + kK * nthreads; it < items; it += nthreads) {
      WideItem v[1];
      const bool one[1] = {true};
      wide_fetch<kOne>(it, pb, nr, srp, sdg, ell_c, ell_v, bp, rio, v[0]);
      wide_solve<1>(v, one, nr, sci, sva, xp, rio, bits);
    }
    if (l + 1 == l1) break;
    const unsigned round = (unsigned)(l - l0 + 1);
    grid_barrier_arrive(bar, round);
    pb = pe;
    pe = ne;
#pragma unroll
    for (int j = 0; j < kK; ++j) {
      const int64_t it = gid + j * nthreads;
      ok[j] = it < (int64_t)(pe - pb) * nr;
      if (ok[j]) wide_fetch<kOne>(it, pb, nr, srp, sdg, ell_c, ell_v, bp, rio, w[j]);
    }
    if (!grid_barrier_wait(bar, round, t0, tlimit, &s_abort)) {
      bits |= EB_TIMEOUT;
      break;
    }
  }
  if (bits) atomicOr(err, bits);
  grid_barrier_reset(bar);
}

}  // namespace

hipError_t launch_wide_level(int threads, int lanes_per_row, int32_t pb, int32_t pe, int32_t nrhs,
                             const int32_t *srp, const int32_t *sci, const double *sva, const double *sdg,
                             const int4 *ell_c, const double2 *ell_v, const double *bp, double *xp, int *err,
                             hipStream_t s, RowsIO rio) {
  const int64_t rows = pe - pb;
  if (rows <= 0) return hipSuccess;
  if (nrhs == 1 && lanes_per_row > 1) {
    const int64_t items = rows * lanes_per_row;
    const int g = grid_for(items, threads, 65536);
#define GRP(G)                                                                                                   \
  hipLaunchKernelGGL((k_wide_level_group<G>), dim3(g), dim3(threads), 0, s, pb, pe, srp, sci, sva, sdg, bp, xp, \
                     err);
    switch (lanes_per_row) {
      case 2: GRP(2) break;
      case 4: GRP(4) break;
      case 8: GRP(8) break;
      case 16: GRP(16) break;
      default: GRP(32) break;
    }
#undef GRP
    return hipGetLastError();
  }
  const int64_t items = rows * nrhs;
  const int per = nrhs == 1 ? 2 : 1;  // items per thread, as in the kernel
  const int g = grid_for((items + per - 1) / per, threads, 65536);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_wide_level<true>), dim3(g), dim3(threads), 0, s, pb, pe, nrhs, srp, sci, sva, sdg, ell_c,
                       ell_v, bp, xp, err, rio);
  else
    hipLaunchKernelGGL((k_wide_level<false>), dim3(g), dim3(threads), 0, s, pb, pe, nrhs, srp, sci, sva, sdg, ell_c,
                       ell_v, bp, xp, err, rio);
  return hipGetLastError();
}

hipError_t launch_wide_long(int32_t pb, int32_t pe, int32_t nrhs, int32_t avg_deg, const int32_t *srp,
                            const int32_t *sci, const double *sva, const double *sdg, const double *bp, double *xp,
                            int *err, hipStream_t s, RowsIO rio) {
  if (pe <= pb) return hipSuccess;
  if (nrhs < 2 || nrhs > 256) return hipErrorInvalidValue;
  // enough groups that each sums about four products: one round of loads
  const int32_t want = (avg_deg + 3) / 4;
  int wg = 64;
  while (wg < 1024 && (wg < nrhs || wg / nrhs < want)) wg *= 2;
#define LONG(W) \
  hipLaunchKernelGGL((k_wide_long<W>), dim3(pe - pb), dim3(W), 0, s, pb, nrhs, srp, sci, sva, sdg, bp, xp, err, rio)
  switch (wg) {
    case 64: LONG(64); break;
    case 128: LONG(128); break;
    case 256: LONG(256); break;
    case 512: LONG(512); break;
    default: LONG(1024); break;
  }
#undef LONG
  return hipGetLastError();
}

int wide_run_resident_blocks(int threads) {
  static int cached[17] = {0};
  const int key = threads / 64;
  if (key < 1 || key > 16) return 0;
  if (!cached[key]) {
    int dev = 0, cus = 0, occ = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(&k_wide_run<false>),
                                                       threads, 0);
    int occ1 = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ1, reinterpret_cast<const void *>(&k_wide_run<true>),
                                                       threads, 0);
    cached[key] = cus * std::max(0, std::min(occ, occ1));
  }
  return cached[key];
}

hipError_t launch_wide_run(int grid, int threads, int32_t l0, int32_t l1, const int32_t *level_ptr, int32_t nrhs,
                           const int32_t *srp, const int32_t *sci, const double *sva, const double *sdg,
                           const int4 *ell_c, const double2 *ell_v, const double *bp, double *xp, unsigned *bar,
                           int *err, unsigned long long limit, hipStream_t s, RowsIO rio) {
  if (l1 <= l0) return hipSuccess;
  const int cap = wide_run_resident_blocks(threads);
  if (cap < 1) return hipErrorInvalidConfiguration;
  grid = std::max(1, std::min(grid, cap));  // every workgroup must be resident for the barrier
  if (nrhs == 1)
    hipLaunchKernelGGL((k_wide_run<true>), dim3(grid), dim3(threads), 0, s, l0, l1, level_ptr, nrhs, srp, sci, sva,
                       sdg, ell_c, ell_v, bp, xp, bar, err, limit, rio);
  else
    hipLaunchKernelGGL((k_wide_run<false>), dim3(grid), dim3(threads), 0, s, l0, l1, level_ptr, nrhs, srp, sci, sva,
                       sdg, ell_c, ell_v, bp, xp, bar, err, limit, rio);
  return hipGetLastError();
}
