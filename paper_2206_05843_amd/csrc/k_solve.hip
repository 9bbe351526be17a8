// Solve kernels: level-by-level forward substitution (Sec. II.A, Algorithm 1)
// over the level-ordered copy of L (or of the rewritten L' with the b-transform
// T applied on the fly, Sec. II.B).
//
// Work vectors are permuted to level order and RHS-interleaved: entry (pos, c)
// of bp/xp is at pos*nrhs + c, so the rows of one level are contiguous and one
// row's right-hand sides share cache lines.
//
// Two schedules per level:
//  * thin runs: consecutive narrow levels inside ONE workgroup; the levels are
//    separated by workgroup barriers (no device-wide synchronisation). Values a
//    run produces are kept in LDS as well, so later levels of the run read
//    them from LDS; the LDS window restarts (after a full barrier that makes the
//    global copies visible) when it is full.
//  * wide levels: one launch over the device per level (kernel boundaries order
//    the levels).
#include "common.h"

namespace {

constexpr int kWinBytes = 150 * 1024;  // LDS of one thin-run window

// Workgroup barrier that orders LDS only: global stores may still be in flight
// (the global copy of x is only read across an LDS-window restart, which uses a
// full barrier).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// x(pos, c) = (b'(pos, c) - sum_k L(pos,k) x(k,c)) / L(pos,pos), with
// b' = b + T_off b when T is present. Columns < lds_base come from global
// memory, columns >= lds_base from the LDS window.
template <bool kUseLds, bool kOne>
__device__ __forceinline__ double row_solve(int32_t pos, int32_t c, int32_t nrhs, const int32_t *__restrict__ srp,
                                            const int32_t *__restrict__ sci, const double *__restrict__ sva,
                                            const double *__restrict__ sdg, const int32_t *__restrict__ trp,
                                            const int32_t *__restrict__ tci, const double *__restrict__ tva,
                                            const double *__restrict__ bp, const double *xp, const double *lds,
                                            int32_t lds_base) {
  const int64_t nr = kOne ? 1 : nrhs;
  double acc = bp[(int64_t)pos * nr + c];
  if (trp) {
    const int32_t tb = trp[pos], te = trp[pos + 1];
    for (int32_t q = tb; q < te; ++q) acc += tva[q] * bp[(int64_t)tci[q] * nr + c];
  }
  const int32_t b = srp[pos], e = srp[pos + 1];
  for (int32_t q = b; q < e; ++q) {
    const int32_t k = sci[q];
    double xv;
    if (kUseLds && k >= lds_base)
      xv = lds[(int64_t)(k - lds_base) * nr + c];
    else
      xv = xp[(int64_t)k * nr + c];
    acc -= sva[q] * xv;
  }
  return acc / sdg[pos];
}

// A thin run is cut into LDS windows (consecutive levels, chosen on the host so
// that the window's rows and dependency records fit in LDS). Per window:
//  phase 1 (all rows in parallel): v = b' - sum of L(pos,k) x(k) over the
//    dependencies k that precede the window (final values, read from global);
//    the dependencies inside the window go to a 32-byte record per row
//    {w0, w1 | slot0, slot1, count, first overflow}; a row's third and later
//    in-window dependencies go to an overflow list of {value, slot} records
//    (its offset is a precomputed prefix sum, ovp);
//  phase 2 (level by level): x = (v - sum over in-window dependencies) * (1/diag),
//    reading and writing LDS only; the global copy of x is written as well.
// When every level of the window has at most one item per thread, phase 2 is
// software-pipelined: the next level's records are requested before the
// current level is computed, and the level bounds are read from registers,
// so a level waits only for the x values it reads. Windows whose levels have
// at most 64 items run phase 2 on one wave without workgroup barriers.
// win[i] = {first level, flags}; the run's last entry holds the end level.
// kTimed (used only to label levels for the learned policy): thread 0 stamps the
// device wall clock around every level and writes per-level times (ns).
struct __align__(16) Dep {
  double w;
  int32_t slot, pad;
};

constexpr int kBatch = 8;

// acc - sum_j w_j x(slot_j, c) over n overflow records starting at d, in order,
// in batches of 8 (tail clamped to a valid record).
template <bool kOne>
__device__ __forceinline__ double ovf_sum(double acc, const Dep *__restrict__ d, int32_t n, const double *v,
                                          int32_t nr, int32_t c) {
  for (int32_t i0 = 0; i0 < n; i0 += kBatch) {
    const int32_t cnt = n - i0;
    double w[kBatch];
    int32_t e[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const Dep dj = d[i0 + (j < cnt ? j : 0)];
      w[j] = dj.w;
      e[j] = dj.slot;
    }
    double xv[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) xv[j] = v[(int64_t)e[j] * (kOne ? 1 : nr) + c];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) acc = j < cnt ? acc - w[j] * xv[j] : acc;
  }
  return acc;
}

// The static inputs of one (row, rhs) item in phase 2.
struct Item {
  double acc, dinv, w0, w1;
  int4 ri;  // slot0, slot1, count, first overflow record
  int32_t s, c, act;
};

template <bool kOne>
__device__ __forceinline__ Item load_item(int32_t pb, int32_t items, int32_t t, int32_t nr, const double *v,
                                          const double *dg, const double2 *rw, const int4 *rix) {
  Item it;
  it.act = t < items;
  it.s = kOne ? pb + t : pb + t / nr;
  it.c = kOne ? 0 : t - (it.s - pb) * nr;
  const int32_t ss = it.act ? it.s : pb;
  const double2 w = rw[ss];
  it.w0 = w.x;
  it.w1 = w.y;
  it.ri = rix[ss];
  it.dinv = dg[ss];
  it.acc = v[(int64_t)ss * nr + (it.act ? it.c : 0)];
  return it;
}

template <bool kOne>
__device__ __forceinline__ double solve_item(const Item &it, int32_t nr, const double *v, const Dep *ovf) {
  const int32_t k = it.ri.z, c = it.c;
  const double xa = v[(int64_t)(k > 0 ? it.ri.x : 0) * nr + c];
  const double xb = v[(int64_t)(k > 1 ? it.ri.y : 0) * nr + c];
  double acc = it.acc;
  acc = k > 0 ? acc - it.w0 * xa : acc;
  acc = k > 1 ? acc - it.w1 * xb : acc;
  if (k > 2) acc = ovf_sum<kOne>(acc, ovf + it.ri.w, k - 2, v, nr, c);
  return acc * it.dinv;
}

// The windows [win, win + nwin) of one thin run, by the calling workgroup.
// Returns the latched error bits; a window that does not fit aborts the run.
template <int WG, bool kOne, bool kTimed>
__device__ __forceinline__ int thin_run_body(double *lds, const int2 *__restrict__ win, int32_t nwin,
                                             const int32_t *__restrict__ level_ptr, int32_t nrhs,
                                             const int32_t *__restrict__ srp, const int32_t *__restrict__ sci,
                                             const double *__restrict__ sva, const double *__restrict__ sdg,
                                             const int32_t *__restrict__ ovp, const int32_t *__restrict__ trp,
                                             const int32_t *__restrict__ tci, const double *__restrict__ tva,
                                             const double *__restrict__ bp, double *xp, float *times,
                                             float ns_per_tick) {
  const int32_t nr = kOne ? 1 : nrhs;
  const int tid = threadIdx.x;
  int bits = 0;
  unsigned long long t_w0 = 0, t_prev = 0;
  float p1_per_row = 0.f;
  for (int32_t w = 0; w < nwin; ++w) {
    if (kTimed && tid == 0) t_w0 = wall_clock64();
    const int32_t lA = win[w].x, lB = win[w + 1].x, flags = win[w].y;
    const int32_t P0 = level_ptr[lA], P1 = level_ptr[lB];
    const int32_t R = P1 - P0;
    const int32_t O0 = ovp[P0], NO = ovp[P1] - O0;
    const int32_t NL = lB - lA;
    const int64_t need = (int64_t)R * (8 * nr + 40) + (int64_t)NO * 16 + 4 * (int64_t)(NL + 1);
    if (need > kWinBytes) return bits | EB_ARG;  // the host sizes windows to fit; never index past LDS
    double2 *rw = reinterpret_cast<double2 *>(lds);          // [R] w0, w1
    int4 *rix = reinterpret_cast<int4 *>(rw + R);             // [R] slot0, slot1, count, overflow
    Dep *ovf = reinterpret_cast<Dep *>(rix + R);              // [NO] third and later dependencies
    double *v = reinterpret_cast<double *>(ovf + NO);         // [R * nr] partial sums, then x
    double *dg = v + (int64_t)R * nr;                         // [R] 1 / diagonal
    int32_t *lv = reinterpret_cast<int32_t *>(dg + R);        // [NL + 1] level bounds, relative to P0
    for (int32_t i = tid; i <= NL; i += WG) lv[i] = level_ptr[lA + i] - P0;
    // phase 1
    for (int32_t it = tid; it < R * nr; it += WG) {
      const int32_t s = kOne ? it : it / nr;
      const int32_t c = kOne ? 0 : it - s * nr;
      const int32_t pos = P0 + s;
      double acc = bp[(int64_t)pos * nr + c];
      if (trp) {
        const int32_t tb = trp[pos], te = trp[pos + 1];
        for (int32_t q = tb; q < te; ++q) acc += tva[q] * bp[(int64_t)tci[q] * nr + c];
      }
      const int32_t qb = srp[pos], qe = srp[pos + 1];
      const int32_t ob = ovp[pos] - O0;
      int32_t kin = 0, s0 = 0, s1 = 0;
      double w0 = 0.0, w1 = 0.0;
      for (int32_t q = qb; q < qe; ++q) {
        const int32_t k = sci[q];
        if (k < P0) {
          acc -= sva[q] * xp[(int64_t)k * nr + c];
        } else {
          if (kin == 0) {
            s0 = k - P0;
            w0 = sva[q];
          } else if (kin == 1) {
            s1 = k - P0;
            w1 = sva[q];
          } else if (c == 0) {
            Dep d;
            d.w = sva[q];
            d.slot = k - P0;
            d.pad = 0;
            ovf[ob + kin - 2] = d;
          }
          ++kin;
        }
      }
      v[(int64_t)s * nr + c] = acc;
      if (c == 0) {
        dg[s] = 1.0 / sdg[pos];  // reciprocal: one multiply on the level chain
        rw[s] = make_double2(w0, w1);
        rix[s] = make_int4(s0, s1, kin, ob);
      }
    }
    __syncthreads();
    if (kTimed && tid == 0) {
      t_prev = wall_clock64();
      p1_per_row = R > 0 ? (float)(t_prev - t_w0) * ns_per_tick / (float)R : 0.f;
    }
    // phase 2
    if (flags & 3) {
      const bool one_wave = flags & 1;
      if (!one_wave || tid < 64) {
        const int lane = tid & 63;
        int32_t lvbase = 0;
        int32_t lvreg = lv[lane <= NL ? lane : NL];
        auto bounds = [&](int32_t l, int32_t &pb, int32_t &items) {
          if (l - lvbase >= 63) {
            lvbase += 63;
            lvreg = lv[lvbase + lane <= NL ? lvbase + lane : NL];
          }
          pb = __builtin_amdgcn_readlane(lvreg, l - lvbase);
          items = (__builtin_amdgcn_readlane(lvreg, l - lvbase + 1) - pb) * nr;
        };
        int32_t pb, items;
        bounds(0, pb, items);
        Item cur = load_item<kOne>(pb, items, tid, nr, v, dg, rw, rix);
        for (int32_t l = 0; l < NL; ++l) {
          Item nxt = cur;
          if (l + 1 < NL) {
            bounds(l + 1, pb, items);
            nxt = load_item<kOne>(pb, items, tid, nr, v, dg, rw, rix);
          }
          if (cur.act) {
            const double x = solve_item<kOne>(cur, nr, v, ovf);
            if (!isfinite(x)) bits |= EB_NONFINITE;
            v[(int64_t)cur.s * nr + cur.c] = x;
            xp[(int64_t)(P0 + cur.s) * nr + cur.c] = x;
          }
          if (one_wave) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
          } else {
            lds_barrier();
          }
          if (kTimed && tid == 0) {
            const unsigned long long now = wall_clock64();
            times[lA + l] = (float)(now - t_prev) * ns_per_tick + p1_per_row * (float)(lv[l + 1] - lv[l]);
            t_prev = now;
          }
          cur = nxt;
        }
      }
    } else {
      for (int32_t l = 0; l < NL; ++l) {
        const int32_t pb = lv[l], items = (lv[l + 1] - pb) * nr;
        for (int32_t t = tid; t < items; t += WG) {
          const Item it = load_item<kOne>(pb, items, t, nr, v, dg, rw, rix);
          const double x = solve_item<kOne>(it, nr, v, ovf);
          if (!isfinite(x)) bits |= EB_NONFINITE;
          v[(int64_t)it.s * nr + it.c] = x;
          xp[(int64_t)(P0 + it.s) * nr + it.c] = x;
        }
        lds_barrier();
        if (kTimed && tid == 0) {
          const unsigned long long now = wall_clock64();
          times[lA + l] = (float)(now - t_prev) * ns_per_tick + p1_per_row * (float)(lv[l + 1] - lv[l]);
          t_prev = now;
        }
      }
    }
    __syncthreads();  // the window's global x is complete before the next phase 1 reads it
  }
  return bits;
}

template <int WG, bool kOne, bool kTimed = false>
__global__ __launch_bounds__(WG) void k_thin_run(const int2 *__restrict__ win, int32_t nwin,
                                                 const int32_t *__restrict__ level_ptr, int32_t nrhs,
                                                 const int32_t *__restrict__ srp, const int32_t *__restrict__ sci,
                                                 const double *__restrict__ sva, const double *__restrict__ sdg,
                                                 const int32_t *__restrict__ ovp, const int32_t *__restrict__ trp,
                                                 const int32_t *__restrict__ tci, const double *__restrict__ tva,
                                                 const double *__restrict__ bp, double *xp, int *err, float *times,
                                                 float ns_per_tick) {
  extern __shared__ double lds[];
  const int bits = thin_run_body<WG, kOne, kTimed>(lds, win, nwin, level_ptr, nrhs, srp, sci, sva, sdg, ovp, trp,
                                                   tci, tva, bp, xp, times, ns_per_tick);
  if (bits) atomicOr(err, bits);
}

// Many independent matrices in one persistent launch: each workgroup takes
// the next matrix from a device queue (matrices are queued largest first) and
// solves all of it with the thin-run windows of that matrix; the levels of a
// matrix are separated by workgroup barriers. The last workgroup to finish
// resets the queue, so the launch can be replayed (graph capture) without a
// host-side reset. q[0] = next ticket, q[1] = finished workgroups.
template <int WG, bool kOne>
__global__ __launch_bounds__(WG) void k_batch_run(int32_t nmat, const int32_t *__restrict__ order,
                                                  const int32_t *__restrict__ mwin, const int2 *__restrict__ win,
                                                  const int32_t *__restrict__ level_ptr, int32_t nrhs,
                                                  const int32_t *__restrict__ srp, const int32_t *__restrict__ sci,
                                                  const double *__restrict__ sva, const double *__restrict__ sdg,
                                                  const int32_t *__restrict__ ovp, const double *__restrict__ bp,
                                                  double *xp, unsigned *q, int *err) {
  extern __shared__ double lds[];
  __shared__ int32_t s_m;
  int bits = 0;
  for (;;) {
    if (threadIdx.x == 0) s_m = (int32_t)atomicAdd(q, 1u);
    __syncthreads();
    const int32_t t = s_m;
    __syncthreads();
    if (t >= nmat) break;
    const int32_t m = order[t];
    bits |= thin_run_body<WG, kOne, false>(lds, win + mwin[m], mwin[m + 1] - mwin[m] - 1, level_ptr, nrhs, srp, sci,
                                           sva, sdg, ovp, nullptr, nullptr, nullptr, bp, xp, nullptr, 0.f);
  }
  if (threadIdx.x == 0) {
    if (bits) atomicOr(err, bits);
    __threadfence();
    if (atomicAdd(q + 1, 1u) == gridDim.x - 1) {
      q[0] = 0;
      q[1] = 0;
      __threadfence();
    }
  }
}

// One wide level, one item (row, rhs) per thread.
template <bool kOne>
__global__ void k_wide_level(int32_t pb, int32_t pe, int32_t nrhs, const int32_t *__restrict__ srp,
                             const int32_t *__restrict__ sci, const double *__restrict__ sva,
                             const double *__restrict__ sdg, const int32_t *__restrict__ trp,
                             const int32_t *__restrict__ tci, const double *__restrict__ tva,
                             const double *__restrict__ bp, double *xp, int *err) {
  const int32_t nr = kOne ? 1 : nrhs;
  const int64_t items = (int64_t)(pe - pb) * nr;
  int bits = 0;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int32_t pos = kOne ? pb + (int32_t)it : pb + (int32_t)(it / nr);
    const int32_t c = kOne ? 0 : (int32_t)(it - (int64_t)(pos - pb) * nr);
    const double xv = row_solve<false, kOne>(pos, c, nr, srp, sci, sva, sdg, trp, tci, tva, bp, xp, nullptr, 0);
    if (!isfinite(xv)) bits |= EB_NONFINITE;
    xp[(int64_t)pos * nr + c] = xv;
  }
  if (bits) atomicOr(err, bits);
}

// One wide level, single RHS, G lanes per row: lanes split the row's products
// and combine them with a fixed butterfly, so the result is deterministic.
template <int G>
__global__ void k_wide_level_group(int32_t pb, int32_t pe, const int32_t *__restrict__ srp,
                                   const int32_t *__restrict__ sci, const double *__restrict__ sva,
                                   const double *__restrict__ sdg, const int32_t *__restrict__ trp,
                                   const int32_t *__restrict__ tci, const double *__restrict__ tva,
                                   const double *__restrict__ bp, double *xp, int *err) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int sub = threadIdx.x & (G - 1);
  int bits = 0;
  const int64_t rows = pe - pb;
  for (int64_t rr = gid / G; rr < (rows + 0); rr += ((int64_t)gridDim.x * blockDim.x) / G) {
    const int32_t pos = pb + (int32_t)rr;
    double acc = 0.0;
    if (trp) {
      const int32_t tb = trp[pos], te = trp[pos + 1];
      for (int32_t q = tb + sub; q < te; q += G) acc += tva[q] * bp[tci[q]];
    }
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

// b (column-major, original rows) -> bp (level order, RHS-interleaved). A tile
// of 64 rows x up to 32 columns is staged in LDS so both sides are coalesced.
__global__ void k_gather(int32_t n, int32_t nrhs, const double *__restrict__ b, int64_t ldb,
                         const int32_t *__restrict__ iperm, double *bp) {
  __shared__ double tile[64][33];
  const int32_t r0 = blockIdx.x * 64;
  for (int32_t c0 = 0; c0 < nrhs; c0 += 32) {
    const int32_t nc = min(32, nrhs - c0);
    for (int idx = threadIdx.x; idx < 64 * nc; idx += blockDim.x) {
      const int c = idx / 64, rr = idx % 64;
      if (r0 + rr < n) tile[rr][c] = b[(int64_t)(c0 + c) * ldb + r0 + rr];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * nc; idx += blockDim.x) {
      const int rr = idx / nc, c = idx % nc;
      if (r0 + rr < n) bp[(int64_t)iperm[r0 + rr] * nrhs + c0 + c] = tile[rr][c];
    }
    __syncthreads();
  }
}

__global__ void k_gather1(int32_t n, const double *__restrict__ b, const int32_t *__restrict__ iperm, double *bp) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    bp[iperm[r]] = b[r];
}

__global__ void k_scatter(int32_t n, int32_t nrhs, const double *__restrict__ xp, const int32_t *__restrict__ iperm,
                          double *x, int64_t ldx) {
  __shared__ double tile[64][33];
  const int32_t r0 = blockIdx.x * 64;
  for (int32_t c0 = 0; c0 < nrhs; c0 += 32) {
    const int32_t nc = min(32, nrhs - c0);
    for (int idx = threadIdx.x; idx < 64 * nc; idx += blockDim.x) {
      const int rr = idx / nc, c = idx % nc;
      if (r0 + rr < n) tile[rr][c] = xp[(int64_t)iperm[r0 + rr] * nrhs + c0 + c];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * nc; idx += blockDim.x) {
      const int c = idx / 64, rr = idx % 64;
      if (r0 + rr < n) x[(int64_t)(c0 + c) * ldx + r0 + rr] = tile[rr][c];
    }
    __syncthreads();
  }
}

__global__ void k_scatter1(int32_t n, const double *__restrict__ xp, const int32_t *__restrict__ iperm, double *x) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    x[r] = xp[iperm[r]];
}

// max_i |(L x - b)[i, c]| per column, original numbering; results as the bit
// patterns of non-negative doubles (monotone as unsigned integers).
__global__ void k_residual(int32_t n, int32_t nrhs, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ va, const double *__restrict__ b, int64_t ldb,
                           const double *__restrict__ x, int64_t ldx, unsigned long long *out) {
  for (int32_t c = 0; c < nrhs; ++c) {
    double m = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
      double s = 0.0;
      for (int32_t q = rp[r]; q < rp[r + 1]; ++q) s += va[q] * x[(int64_t)c * ldx + ci[q]];
      const double d = fabs(s - b[(int64_t)c * ldb + r]);
      m = (d > m || d != d) ? d : m;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(m, off, 64);
      m = (o > m || o != o) ? o : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out + c, (unsigned long long)__double_as_longlong(m));
  }
}

// Batched right-hand sides: matrix m's b and x are n_m x nrhs column-major at
// offset nrhs * row_off[m], ld = n_m. Items run over (global row, column) with
// the row fastest, so each column of each matrix is read/written contiguously.
__global__ void k_batch_gather(int64_t total, int32_t nrhs, const double *__restrict__ b,
                               const int32_t *__restrict__ mat_of_row, const int64_t *__restrict__ row_off,
                               const int32_t *__restrict__ iperm, double *bp) {
  const int64_t items = total * nrhs;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = it / total, r = it - c * total;
    const int32_t m = mat_of_row[r];
    const int64_t ro = row_off[m], nm = row_off[m + 1] - ro;
    bp[(int64_t)iperm[r] * nrhs + c] = b[nrhs * ro + c * nm + (r - ro)];
  }
}

__global__ void k_batch_scatter(int64_t total, int32_t nrhs, const double *__restrict__ xp,
                                const int32_t *__restrict__ mat_of_row, const int64_t *__restrict__ row_off,
                                const int32_t *__restrict__ iperm, double *x) {
  const int64_t items = total * nrhs;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < items;
       it += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = it / total, r = it - c * total;
    const int32_t m = mat_of_row[r];
    const int64_t ro = row_off[m], nm = row_off[m + 1] - ro;
    x[nrhs * ro + c * nm + (r - ro)] = xp[(int64_t)iperm[r] * nrhs + c];
  }
}

inline int grid_for(int64_t items, int threads, int cap) {
  int64_t g = (items + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

template <int WG, bool kOne>
void set_lds_attr() {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_thin_run<WG, kOne>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
}

}  // namespace

int thin_win_bytes() { return kWinBytes; }

void solve_kernels_init() {
  set_lds_attr<256, true>();
  set_lds_attr<256, false>();
  set_lds_attr<512, true>();
  set_lds_attr<512, false>();
  set_lds_attr<1024, true>();
  set_lds_attr<1024, false>();
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_thin_run<512, true, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_thin_run<512, false, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
}

hipError_t launch_gather(int32_t n, int32_t nrhs, const double *b, int64_t ldb, const int32_t *iperm, double *bp,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nrhs == 1)
    hipLaunchKernelGGL(k_gather1, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, b, iperm, bp);
  else
    hipLaunchKernelGGL(k_gather, dim3((n + 63) / 64), dim3(256), 0, s, n, nrhs, b, ldb, iperm, bp);
  return hipGetLastError();
}

hipError_t launch_scatter(int32_t n, int32_t nrhs, const double *xp, const int32_t *iperm, double *x, int64_t ldx,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nrhs == 1)
    hipLaunchKernelGGL(k_scatter1, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, xp, iperm, x);
  else
    hipLaunchKernelGGL(k_scatter, dim3((n + 63) / 64), dim3(256), 0, s, n, nrhs, xp, iperm, x, ldx);
  return hipGetLastError();
}

hipError_t launch_thin_run(int wg, const int2 *win, int32_t nwin, const int32_t *level_ptr, int32_t nrhs,
                           const int32_t *srp, const int32_t *sci, const double *sva, const double *sdg,
                           const int32_t *ovp, const int32_t *trp, const int32_t *tci, const double *tva, const double *bp,
                           double *xp, int *err, hipStream_t s, float *times, float ns_per_tick) {
  const bool one = nrhs == 1;
  if (times) {  // labelling runs only: 512 threads
    if (one)
      hipLaunchKernelGGL((k_thin_run<512, true, true>), dim3(1), dim3(512), kWinBytes, s, win, nwin, level_ptr, nrhs,
                         srp, sci, sva, sdg, ovp, trp, tci, tva, bp, xp, err, times, ns_per_tick);
    else
      hipLaunchKernelGGL((k_thin_run<512, false, true>), dim3(1), dim3(512), kWinBytes, s, win, nwin, level_ptr, nrhs,
                         srp, sci, sva, sdg, ovp, trp, tci, tva, bp, xp, err, times, ns_per_tick);
    return hipGetLastError();
  }
#define THIN(W)                                                                                                   \
  if (one)                                                                                                        \
    hipLaunchKernelGGL((k_thin_run<W, true>), dim3(1), dim3(W), kWinBytes, s, win, nwin, level_ptr, nrhs, srp, sci, \
                       sva, sdg, ovp, trp, tci, tva, bp, xp, err, (float *)nullptr, 0.f);                              \
  else                                                                                                            \
    hipLaunchKernelGGL((k_thin_run<W, false>), dim3(1), dim3(W), kWinBytes, s, win, nwin, level_ptr, nrhs, srp,     \
                       sci, sva, sdg, ovp, trp, tci, tva, bp, xp, err, (float *)nullptr, 0.f);
  if (wg == 256) {
    THIN(256)
  } else if (wg == 1024) {
    THIN(1024)
  } else {
    THIN(512)
  }
#undef THIN
  return hipGetLastError();
}

hipError_t launch_wide_level(int threads, int lanes_per_row, int32_t pb, int32_t pe, int32_t nrhs,
                             const int32_t *srp, const int32_t *sci, const double *sva, const double *sdg,
                             const int32_t *trp, const int32_t *tci, const double *tva, const double *bp,
                             double *xp, int *err, hipStream_t s) {
  const int64_t rows = pe - pb;
  if (rows <= 0) return hipSuccess;
  if (nrhs == 1 && lanes_per_row > 1) {
    const int64_t items = rows * lanes_per_row;
    const int g = grid_for(items, threads, 65536);
#define GRP(G)                                                                                                   \
  hipLaunchKernelGGL((k_wide_level_group<G>), dim3(g), dim3(threads), 0, s, pb, pe, srp, sci, sva, sdg, trp, tci, \
                     tva, bp, xp, err);
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
  const int g = grid_for(items, threads, 65536);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_wide_level<true>), dim3(g), dim3(threads), 0, s, pb, pe, nrhs, srp, sci, sva, sdg, trp,
                       tci, tva, bp, xp, err);
  else
    hipLaunchKernelGGL((k_wide_level<false>), dim3(g), dim3(threads), 0, s, pb, pe, nrhs, srp, sci, sva, sdg, trp,
                       tci, tva, bp, xp, err);
  return hipGetLastError();
}

hipError_t launch_residual(int32_t n, int32_t nrhs, const int32_t *rp, const int32_t *ci, const double *va,
                           const double *b, int64_t ldb, const double *x, int64_t ldx, unsigned long long *out,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n, nrhs, rp, ci, va, b, ldb, x,
                     ldx, out);
  return hipGetLastError();
}

hipError_t launch_batch_run(int32_t nmat, int32_t grid, const int32_t *order, const int32_t *mwin, const int2 *win,
                            const int32_t *level_ptr, int32_t nrhs, const int32_t *srp, const int32_t *sci,
                            const double *sva, const double *sdg, const int32_t *ovp, const double *bp, double *xp,
                            unsigned *q, int *err, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_run<512, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_run<512, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
    attr = true;
  }
  if (nrhs == 1)
    hipLaunchKernelGGL((k_batch_run<512, true>), dim3(grid), dim3(512), kWinBytes, s, nmat, order, mwin, win,
                       level_ptr, nrhs, srp, sci, sva, sdg, ovp, bp, xp, q, err);
  else
    hipLaunchKernelGGL((k_batch_run<512, false>), dim3(grid), dim3(512), kWinBytes, s, nmat, order, mwin, win,
                       level_ptr, nrhs, srp, sci, sva, sdg, ovp, bp, xp, q, err);
  return hipGetLastError();
}

hipError_t launch_batch_gather(int64_t total, int32_t nrhs, const double *b, const int32_t *mat_of_row,
                               const int64_t *row_off, const int32_t *iperm, double *bp, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_gather, dim3(grid_for(total * nrhs, 256, 16384)), dim3(256), 0, s, total, nrhs, b,
                     mat_of_row, row_off, iperm, bp);
  return hipGetLastError();
}

hipError_t launch_batch_scatter(int64_t total, int32_t nrhs, const double *xp, const int32_t *mat_of_row,
                                const int64_t *row_off, const int32_t *iperm, double *x, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_scatter, dim3(grid_for(total * nrhs, 256, 16384)), dim3(256), 0, s, total, nrhs, xp,
                     mat_of_row, row_off, iperm, x);
  return hipGetLastError();
}

int batch_resident_blocks() {
  int dev = 0, cus = 256, occ = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(&k_batch_run<512, false>),
                                                     512, kWinBytes);
  return cus * (occ > 0 ? occ : 1);
}
