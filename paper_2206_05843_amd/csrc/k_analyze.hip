// Analysis kernels: validation, level sets by longest path, stable bucketing of
// rows by level, the level-ordered copy the solve streams, level statistics,
// and the device-wide scans they use.
#include "common.h"

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Validation (Algorithm 1 reads the diagonal at the last slot of each row):
// one thread per row; row ranges are checked before they are dereferenced so
// malformed row pointers never lead to an out-of-range access.
__global__ void k_validate(int32_t n, int32_t nnz, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ va, int *err) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bits = 0;
  if (r == 0 && (rp[0] != 0 || rp[n] != nnz)) bits |= EB_ARG;
  if (r < n) {
    int32_t b = rp[r], e = rp[r + 1];
    if (b < 0 || e < b || e > nnz) {
      bits |= EB_ARG;
    } else {
      int32_t prev = -1;
      for (int32_t p = b; p < e; ++p) {
        int32_t c = ci[p];
        double v = va[p];
        if (c < 0 || c > r) bits |= EB_NOT_LOWER;
        if (p > b && c <= prev) bits |= EB_UNSORTED;
        if (!isfinite(v)) bits |= EB_NONFINITE;
        prev = c;
      }
      if (e == b || ci[e - 1] != r)
        bits |= EB_MISSING_DIAG;
      else if (va[e - 1] == 0.0)
        bits |= EB_ZERO_PIVOT;
    }
  }
  if (bits) atomicOr(err, bits);
}

// ---------------------------------------------------------------------------
// Level sets by longest path, synchronisation-free. Waves claim 64 consecutive
// rows from a ticket counter, so every row a claimed row depends on (a smaller
// index) is already claimed by a running wave. lev1[r] holds level+1 once row r
// is done (0 = not yet). A lane finishes its row when all dependencies are
// published; lanes waiting on lower lanes of their own wave are released as the
// wave keeps iterating. A row with more than kLongRow dependencies left is
// swept by the whole wave first, kLongRow entries per step, one step after
// another while every entry of a step is published (the dependents lists of a
// power-law matrix's hub columns have millions of entries; one lane reading
// them one by one took seconds). Waits are bounded by a wall-clock limit.
constexpr int kLongRow = 256;

__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

__global__ void k_levels(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, int32_t *lev1,
                         unsigned *ticket, int *err, unsigned long long tlimit) {
  const int lane = threadIdx.x & 63;
  const unsigned long long t0 = wall_clock64();
  for (;;) {
    int base = 0;
    if (lane == 0) base = (int)atomicAdd(ticket, 64u);
    base = __shfl(base, 0, 64);
    if (base >= n) return;
    const int32_t r = base + lane;
    bool pend = r < n;
    int32_t p = 0, e = 0, mx = 0;
    if (pend) {
      p = rp[r];
      e = rp[r + 1] - 1;
    }
    unsigned spins = 0;
    while (__ballot(pend) != 0ull) {
      const int32_t p_in = p;
      const bool pend_in = pend;
      unsigned long long lm = __ballot(pend && e - p > kLongRow);
      while (lm != 0ull) {  // long rows, one at a time, by the whole wave
        const int src = __builtin_ctzll(lm);
        lm &= lm - 1ull;
        int32_t sp = __shfl(p, src, 64), smx = __shfl(mx, src, 64);
        const int32_t se = __shfl(e, src, 64);
        for (int step = 0; step < 64 && se - sp > kLongRow; ++step) {
          int32_t v[kLongRow / 64];
#pragma unroll
          for (int j = 0; j < kLongRow / 64; ++j)
            v[j] = __hip_atomic_load(lev1 + ci[sp + j * 64 + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          bool ready = true;
          int32_t m = 0;
#pragma unroll
          for (int j = 0; j < kLongRow / 64; ++j) {
            ready = ready && v[j] != 0;
            m = v[j] > m ? v[j] : m;
          }
          if (__ballot(!ready) != 0ull) break;  // a dependency is pending: come back to it later
          m = wave_max_i32(m);
          smx = m > smx ? m : smx;
          sp += kLongRow;
        }
        if (lane == src) {
          p = sp;
          mx = smx;
        }
      }
      if (pend && e - p <= kLongRow) {  // longer rows advance only through the sweep above
        while (p < e) {
          int32_t v = __hip_atomic_load(lev1 + ci[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (v == 0) break;
          mx = v > mx ? v : mx;
          ++p;
        }
        if (p == e) {
          __hip_atomic_store(lev1 + r, mx + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          pend = false;
        }
      }
      // a wave none of whose rows advanced pauses before it polls again, so
      // that waiting waves do not flood the memory system with coherent loads
      if (__ballot(p != p_in || pend != pend_in) == 0ull) __builtin_amdgcn_s_sleep(4);
      if ((++spins & 63u) == 0u && wall_clock64() - t0 > tlimit) {
        if (lane == 0) atomicOr(err, EB_TIMEOUT);
        return;
      }
    }
  }
}

// Heights (longest path from a row to a row nothing depends on), by a sweep
// over the levels from the last to the first on the level-ordered copy: when
// a level is reached, every row that depends on one of its rows sits in a
// later level and has already raised its height, so the level's heights are
// final; each row then raises the height of every row it depends on. hp is by
// position and starts at zero. A wide level is one launch (kernel boundaries
// order the levels).
__global__ void k_height_level(int32_t pb, int32_t pe, const int32_t *__restrict__ srp,
                               const int32_t *__restrict__ sci, int32_t *hp) {
  for (int64_t p = pb + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pe; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t h = hp[p] + 1;
    // heights only grow, so a value read here (possibly an older copy) that
    // already reaches h makes the atomic redundant: hub columns that thousands
    // of rows of a level depend on then take a few atomics instead of one per
    // row (same-address atomics are serialised)
    for (int32_t q = srp[p]; q < srp[p + 1]; ++q) {
      const int32_t d = sci[q];
      if (hp[d] < h) atomicMax(hp + d, h);
    }
  }
}

// A run of consecutive narrow levels [l0, l1) in one workgroup, last level
// first; the raises of a level complete (s_waitcnt) before the workgroup
// barrier that starts the next one, and heights are read with device-scope
// loads from where the atomics were performed.
__global__ __launch_bounds__(1024) void k_height_run(int32_t l0, int32_t l1, const int32_t *__restrict__ level_ptr,
                                                     const int32_t *__restrict__ srp, const int32_t *__restrict__ sci,
                                                     int32_t *hp) {
  for (int32_t l = l1 - 1; l >= l0; --l) {
    const int32_t pb = level_ptr[l], pe = level_ptr[l + 1];
    for (int32_t p = pb + (int32_t)threadIdx.x; p < pe; p += (int32_t)blockDim.x) {
      const int32_t h = __hip_atomic_load(hp + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
      for (int32_t q = srp[p]; q < srp[p + 1]; ++q) atomicMax(hp + sci[q], h);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
}

// Longest-path membership of every row: level + height = nlev - 1.
__global__ void k_crit_from_heights(int32_t n, int32_t nlev, const int32_t *__restrict__ perm,
                                    const int32_t *__restrict__ row_level, const int32_t *__restrict__ hp,
                                    uint8_t *oncrit) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = perm[p];
    oncrit[r] = (uint8_t)(row_level[r] + hp[p] == nlev - 1 ? 1 : 0);
  }
}

__global__ void k_max(const int32_t *__restrict__ a, int32_t n, int32_t *out) {
  int32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = a[i] > m ? a[i] : m;
  for (int off = 32; off > 0; off >>= 1) {
    int32_t o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// ---------------------------------------------------------------------------
// Exclusive scan of int64 values: 1024 items per block (4 per thread), block
// totals scanned recursively and added back.
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ inline long long block_exclusive_scan(long long v, long long *total) {
  __shared__ long long wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  long long inc = v;
  for (int off = 1; off < 64; off <<= 1) {
    long long o = __shfl_up(inc, off, 64);
    if (lane >= off) inc += o;
  }
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  long long pre = 0, tot = 0;
  for (int i = 0; i < kBlock / 64; ++i) {
    if (i < w) pre += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return pre + inc - v;
}

__global__ void k_scan_block(const long long *__restrict__ in, long long *out, int64_t n, long long *bsum) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  long long v[kScanItems];
  long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    s += v[j];
  }
  long long tot;
  long long ex = block_exclusive_scan(s, &tot);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = ex;
    ex += v[j];
  }
  if (threadIdx.x == 0 && bsum) bsum[blockIdx.x] = tot;
}

__global__ void k_scan_add(long long *out, int64_t n, const long long *__restrict__ boff) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  const long long add = boff[blockIdx.x];
  for (int j = threadIdx.x; j < kScanTile; j += kBlock)
    if (base + j < n) out[base + j] += add;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (key, value) pairs, 8 bits per pass. Within a block
// of 1024 items the rank of an item among equal digits is found wave by wave
// with ballots (lanes in order), then across the block's waves and rounds in
// order, so equal keys keep their input order.
constexpr int kRsItems = 4;
constexpr int kRsTile = kBlock * kRsItems;

__global__ void k_rs_hist(const int32_t *__restrict__ keys, int32_t n, int shift, int32_t *hist, int nblk) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRsTile;
  for (int j = 0; j < kRsItems; ++j) {
    int64_t i = base + j * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_i32_to_i64(const int32_t *__restrict__ a, int64_t n, long long *b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_rs_scatter(const int32_t *__restrict__ kin, const int32_t *__restrict__ vin, int32_t n, int shift,
                             const long long *__restrict__ offs, int nblk, int32_t *kout, int32_t *vout) {
  __shared__ int cnt[kBlock / 64][256];
  __shared__ int woff[kBlock / 64][256];
  __shared__ int run[256];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  run[t] = 0;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int j = 0; j < kRsItems; ++j) {
    const int64_t i = (int64_t)blockIdx.x * kRsTile + j * kBlock + t;
    const bool valid = i < n;
    const int32_t k = valid ? kin[i] : 0;
    const int32_t v = valid ? vin[i] : 0;
    const int d = (k >> shift) & 255;
    unsigned long long m = __ballot(valid);
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1;
      const unsigned long long bb = __ballot(on);
      m &= on ? bb : ~bb;
    }
    const int rank = __popcll(m & lt);
    for (int q = t; q < (kBlock / 64) * 256; q += kBlock) (&cnt[0][0])[q] = 0;
    __syncthreads();
    if (valid && rank == 0) cnt[w][d] = __popcll(m);
    __syncthreads();
    {
      int acc = run[t];
      for (int ww = 0; ww < kBlock / 64; ++ww) {
        woff[ww][t] = acc;
        acc += cnt[ww][t];
      }
      run[t] = acc;
    }
    __syncthreads();
    if (valid) {
      const long long pos = offs[(int64_t)d * nblk + blockIdx.x] + woff[w][d] + rank;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
  }
}

// level_ptr from keys sorted ascending (levels are contiguous: every level
// between 0 and the deepest one holds at least one row).
__global__ void k_level_ptr(const int32_t *__restrict__ skeys, int32_t n, int32_t *level_ptr, int32_t nlev) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = skeys[i] - 1;  // keys are level+1
    const int32_t prev = i == 0 ? -1 : skeys[i - 1] - 1;
    for (int32_t l = prev + 1; l <= k; ++l) level_ptr[l] = (int32_t)i;
    if (i == n - 1) level_ptr[nlev] = n;
  }
}

__global__ void k_iota(int32_t *a, int32_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = (int32_t)i;
}

__global__ void k_invert(const int32_t *__restrict__ perm, int32_t n, int32_t *iperm) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    iperm[perm[i]] = (int32_t)i;
}

__global__ void k_sub1(const int32_t *__restrict__ a, int32_t n, int32_t *out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] - 1;
}

// off-diagonal count of the row at each position
__global__ void k_count_off(const int32_t *__restrict__ perm, const int32_t *__restrict__ rp, int32_t n,
                            long long *cnt) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = perm[p];
    cnt[p] = rp[r + 1] - rp[r] - 1;
  }
}

__global__ void k_ptr_from_scan(const long long *__restrict__ ex, const long long *__restrict__ cnt, int32_t n,
                                int32_t *ptr, int *err) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const long long v = ex[p];
    if (v > 0x7fffffffLL) atomicOr(err, EB_OVERFLOW);
    ptr[p] = (int32_t)v;
    if (p == n - 1) {
      const long long e = v + cnt[p];
      if (e > 0x7fffffffLL) atomicOr(err, EB_OVERFLOW);
      ptr[n] = (int32_t)e;
    }
  }
}

// Level-ordered copy: the row at position p keeps its column order; columns
// become positions so the solve reads its work vectors contiguously per level.
__global__ void k_fill_solve(int32_t n, const int32_t *__restrict__ perm, const int32_t *__restrict__ iperm,
                             const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const double *__restrict__ va, const int32_t *__restrict__ srp, int32_t *sci,
                             double *sva, double *sdg) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = perm[p];
    const int32_t b = rp[r], e = rp[r + 1] - 1;
    int32_t o = srp[p];
    for (int32_t q = b; q < e; ++q, ++o) {
      sci[o] = iperm[ci[q]];
      sva[o] = va[q];
    }
    sdg[p] = va[e];
  }
}

__global__ void k_fill_t(int32_t n, const int32_t *__restrict__ perm, const int32_t *__restrict__ trp,
                         const int32_t *__restrict__ tci, int rev,
                         const double *__restrict__ tva, const int32_t *__restrict__ strp, int32_t *stci,
                         double *stva) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = perm[p];
    const int32_t b = trp[r], e = trp[r + 1] - 1;  // last entry is the unit diagonal
    int32_t o = strp[p];
    for (int32_t q = b; q < e; ++q, ++o) {
      stci[o] = rev ? n - 1 - tci[q] : tci[q];  // columns in the caller's numbering: b is read there
      stva[o] = tva[q];
    }
  }
}

// Cost model per level (Sec. III): cost = 2 * sum(nnz) - rows.
__global__ void k_level_stats(int32_t nlev, const int32_t *__restrict__ lp, const int32_t *__restrict__ srp,
                              int64_t *rows, int64_t *nnz, int64_t *cost, long long *total) {
  long long c = 0;
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nlev; l += (int64_t)gridDim.x * blockDim.x) {
    const int64_t R = lp[l + 1] - lp[l];
    const int64_t z = (int64_t)(srp[lp[l + 1]] - srp[lp[l]]) + R;
    rows[l] = R;
    nnz[l] = z;
    cost[l] = 2 * z - R;
    c += 2 * z - R;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd((unsigned long long *)total, (unsigned long long)c);
}

}  // namespace

// ----------------------------------------------------------------- launchers
hipError_t launch_validate(int32_t n, int32_t nnz, const int32_t *rp, const int32_t *ci, const double *va, int *err,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, nnz, rp, ci, va, err);
  return hipGetLastError();
}

hipError_t launch_levels(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *lev1, unsigned *ticket, int *err,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  const unsigned long long limit = 100000000ull * 20;  // 20 s of the 100 MHz wall clock
  hipLaunchKernelGGL(k_levels, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, s, n, rp, ci, lev1, ticket, err,
                     limit);
  return hipGetLastError();
}

hipError_t launch_heights(int32_t n, int32_t nlev, const int32_t *level_ptr, const int32_t *h_level_ptr,
                          const int32_t *srp, const int32_t *sci, int32_t *hp, hipStream_t s) {
  constexpr int32_t kNarrow = 256;  // levels of at most this many rows share a one-workgroup launch
  int32_t l = nlev - 1;
  while (l >= 0) {
    const int32_t rows = h_level_ptr[l + 1] - h_level_ptr[l];
    if (rows > kNarrow) {
      hipLaunchKernelGGL(k_height_level, dim3(grid_for(rows, kBlock, 4096)), dim3(kBlock), 0, s, h_level_ptr[l],
                         h_level_ptr[l + 1], srp, sci, hp);
      --l;
      continue;
    }
    int32_t l0 = l;
    while (l0 > 0 && h_level_ptr[l0] - h_level_ptr[l0 - 1] <= kNarrow) --l0;
    hipLaunchKernelGGL(k_height_run, dim3(1), dim3(1024), 0, s, l0, l + 1, level_ptr, srp, sci, hp);
    l = l0 - 1;
  }
  return hipGetLastError();
}

hipError_t launch_crit_from_heights(int32_t n, int32_t nlev, const int32_t *perm, const int32_t *row_level,
                                    const int32_t *hp, uint8_t *oncrit, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_crit_from_heights, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, n, nlev, perm,
                     row_level, hp, oncrit);
  return hipGetLastError();
}

hipError_t launch_max(const int32_t *a, int32_t n, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_max, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, s, a, n, out);
  return hipGetLastError();
}

size_t scan_scratch_elems(int64_t n) {
  size_t tot = 0;
  int64_t m = n;
  while (m > kScanTile) {
    m = (m + kScanTile - 1) / kScanTile;
    tot += (size_t)m * 2;
  }
  return tot + 2;
}

hipError_t launch_scan_i64(const long long *in, long long *out, int64_t n, long long *scratch, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(kBlock), 0, s, in, out, n, (long long *)nullptr);
    return hipGetLastError();
  }
  long long *bsum = scratch, *boff = scratch + nb;
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(kBlock), 0, s, in, out, n, bsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_i64(bsum, boff, nb, scratch + 2 * nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kBlock), 0, s, out, n, boff);
  return hipGetLastError();
}

size_t radix_hist_elems(int32_t n) { return (size_t)256 * (size_t)((n + kRsTile - 1) / kRsTile + 1); }

hipError_t launch_radix_by_key(int32_t *keys, int32_t *vals, int32_t *keys_tmp, int32_t *vals_tmp, int32_t n,
                               int bits, int32_t *hist, long long *hist64, long long *scratch, hipStream_t s) {
  if (n <= 1 || bits <= 0) return hipSuccess;
  const int nblk = (n + kRsTile - 1) / kRsTile;
  const int64_t hn = (int64_t)256 * nblk;
  int32_t *ka = keys, *va = vals, *kb = keys_tmp, *vb = vals_tmp;
  int passes = (bits + 7) / 8;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = 8 * ps;
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kBlock), 0, s, ka, n, shift, hist, nblk);
    hipLaunchKernelGGL(k_i32_to_i64, dim3(grid_for(hn, kBlock, 4096)), dim3(kBlock), 0, s, hist, hn, hist64);
    hipError_t e = launch_scan_i64(hist64, hist64, hn, scratch, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kBlock), 0, s, ka, va, n, shift, hist64, nblk, kb, vb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t *t;
    t = ka, ka = kb, kb = t;
    t = va, va = vb, vb = t;
  }
  if (ka != keys) {
    hipError_t e = hipMemcpyAsync(keys, ka, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_level_ptr_from_sorted(const int32_t *sorted_keys, int32_t n, int32_t *level_ptr, int32_t nlev,
                                        hipStream_t s) {
  if (n == 0) return hipMemsetAsync(level_ptr, 0, sizeof(int32_t), s);
  hipLaunchKernelGGL(k_level_ptr, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, sorted_keys, n, level_ptr,
                     nlev);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t *a, int32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, a, n);
  return hipGetLastError();
}

hipError_t launch_invert_perm(const int32_t *perm, int32_t n, int32_t *iperm, hipStream_t s) {
  hipLaunchKernelGGL(k_invert, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, perm, n, iperm);
  return hipGetLastError();
}

hipError_t launch_sub1(const int32_t *a, int32_t n, int32_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sub1, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, a, n, out);
  return hipGetLastError();
}

hipError_t launch_count_off(const int32_t *perm, const int32_t *rp, int32_t n, long long *cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_count_off, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, perm, rp, n, cnt);
  return hipGetLastError();
}

hipError_t launch_ptr_from_scan(const long long *ex, const long long *cnt, int32_t n, int32_t *ptr, int *err,
                                hipStream_t s) {
  if (n == 0) return hipMemsetAsync(ptr, 0, sizeof(int32_t), s);
  hipLaunchKernelGGL(k_ptr_from_scan, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, ex, cnt, n, ptr, err);
  return hipGetLastError();
}

hipError_t launch_fill_solve(int32_t n, const int32_t *perm, const int32_t *iperm, const int32_t *rp,
                             const int32_t *ci, const double *va, const int32_t *srp, int32_t *sci, double *sva,
                             double *sdg, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_solve, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, perm, iperm, rp, ci, va,
                     srp, sci, sva, sdg);
  return hipGetLastError();
}

hipError_t launch_fill_t(int32_t n, const int32_t *perm, const int32_t *trp, const int32_t *tci,
                         const double *tva, const int32_t *strp, int32_t *stci, double *stva, bool rev, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_t, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, perm, trp, tci, rev ? 1 : 0,
                     tva, strp, stci, stva);
  return hipGetLastError();
}

hipError_t launch_level_stats(int32_t nlev, const int32_t *level_ptr, const int32_t *srp, int64_t *rows,
                              int64_t *nnz, int64_t *cost, long long *total, hipStream_t s) {
  hipLaunchKernelGGL(k_level_stats, dim3(grid_for(nlev, kBlock, 1024)), dim3(kBlock), 0, s, nlev, level_ptr, srp,
                     rows, nnz, cost, total);
  return hipGetLastError();
}

namespace {
// Level of every position of the level-ordered numbering (last l with
// level_ptr[l] <= p).
__global__ void k_level_of_pos(int32_t n, const int32_t *__restrict__ level_ptr, int32_t nlev, int32_t *lop) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = nlev - 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (level_ptr[mid] <= (int32_t)p) lo = mid; else hi = mid - 1;
    }
    lop[p] = lo;
  }
}

// Per level, a histogram of the level distance l - level(k) over each row's
// dependencies k except the two at the highest levels (a row keeps two
// in-window dependencies inline; the others need overflow records). Distance
// buckets: 1, 2, 3, 4, 5-8, 9-16, 17-32, 33-64, 65-256, >256.
__global__ void k_extra_hist(int32_t n, const int32_t *__restrict__ srp, const int32_t *__restrict__ sci,
                             const int32_t *__restrict__ lop, int32_t *hist) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t qb = srp[p], qe = srp[p + 1];
    if (qe - qb <= 2) continue;
    const int32_t l = lop[p];
    int32_t m1 = -1, m2 = -1;  // the two highest dependency levels (with multiplicity)
    for (int32_t q = qb; q < qe; ++q) {
      const int32_t a = lop[sci[q]];
      if (a > m1) {
        m2 = m1;
        m1 = a;
      } else if (a > m2) {
        m2 = a;
      }
    }
    bool skip1 = false, skip2 = false;
    for (int32_t q = qb; q < qe; ++q) {
      const int32_t a = lop[sci[q]];
      if (!skip1 && a == m1) {
        skip1 = true;
        continue;
      }
      if (!skip2 && a == m2) {
        skip2 = true;
        continue;
      }
      const int32_t d = l - a;
      const int32_t b = d <= 4 ? d - 1 : d <= 8 ? 4 : d <= 16 ? 5 : d <= 32 ? 6 : d <= 64 ? 7 : d <= 256 ? 8 : 9;
      atomicAdd(hist + (int64_t)l * kExtraBuckets + b, 1);
    }
  }
}
}  // namespace

hipError_t launch_extra_hist(int32_t n, const int32_t *level_ptr, int32_t nlev, const int32_t *srp,
                             const int32_t *sci, int32_t *lop, int32_t *hist, hipStream_t s) {
  if (n == 0 || nlev == 0) return hipSuccess;
  hipLaunchKernelGGL(k_level_of_pos, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, n, level_ptr, nlev, lop);
  hipLaunchKernelGGL(k_extra_hist, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, s, n, srp, sci, lop, hist);
  return hipGetLastError();
}
