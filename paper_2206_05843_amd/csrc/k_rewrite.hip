// Equation rewriting on the device (Sec. II.B, Fig. 2; naive strategy of Sec. III).
//
// Rewriting row r toward target level t substitutes, largest column first,
// every unknown x[j] of the row whose row sits at level >= t (B set) by row j's
// own equation; what is left are unknowns of rows above t (A set). Rearranged,
// the row becomes L'[r] x = T[r] b: L'[r] holds the A coefficients and the
// unchanged diagonal, T[r] holds minus each elimination multiplier and a unit
// diagonal. Fill that cancels to zero stays in the pattern.
//
// One wave computes one row, in a workspace indexed by an open-addressing hash
// on the column: every entry of the row being built is (column, value, state)
// with state 0 = A (kept in L'), 1 = B (still to eliminate), 2 = eliminated
// (its value is the T coefficient). Products and differences are rounded one
// by one (no contraction) and every coefficient receives its updates in the
// same order as the serial definition, so values are reproducible bit for bit.
//
// Decision scan: while the target is t, the B set is fixed (a row moving into t
// stays at or below t), so the candidates of one step are independent; one
// workgroup evaluates a chunk of candidates (one per wave) and its first thread
// accepts them in order until the first refusal.
#include "common.h"

namespace {

constexpr int kWaves = 8;          // waves per workgroup in both kernels
constexpr int kLdsC = 512;         // LDS workspace entries per wave
constexpr int kLdsH = 1024;        // LDS hash slots per wave
// Bytes of a workspace of C entries and H hash slots: val[C], hkey[H],
// hslot[H], col[C], four counters, st[C] (padded to 4 bytes), pend[C]; a
// multiple of 16 so that consecutive workspaces stay aligned.
__host__ __device__ constexpr size_t ws_core_bytes(size_t C, size_t H) {
  return (C * 8 + H * 8 + C * 4 + 16 + ((C + 3) & ~(size_t)3) + C * 4 + 15) & ~(size_t)15;
}
// A scan candidate that outgrows its LDS workspace is evaluated again at once
// by the same wave in a private region of the global workspace of this size
// (cleared per candidate, so kept far below the full workspace); only a row
// that outgrows that too takes the serial path through the full workspace.
constexpr int kTier1C = 1 << 14;
constexpr int kTier1H = 1 << 15;
constexpr size_t kTier1Bytes = ((ws_core_bytes(kTier1C, kTier1H) + 48) + 255) & ~(size_t)255;

enum : int { SUB_OK = 0, SUB_REJECT = 1, SUB_OVERFLOW = 2 };

struct Ws {
  int32_t *hkey;    // [H] column or -1
  int32_t *hslot;   // [H] entry index
  int32_t *col;     // [C]
  double *val;      // [C]
  uint8_t *st;      // [C]
  int32_t *cnt;     // entries used
  int32_t *na;      // entries in state 0
  int32_t *np;      // entries in state 1 (listed in pend)
  int32_t *pend;    // [C] entry indices of the state-1 entries, in no order
  int32_t C, H;
};


__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ long long wave_max_ll(long long v) {
  for (int off = 32; off > 0; off >>= 1) {
    const long long o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Find column k or insert it (keys inserted concurrently by the lanes of a
// wave are distinct). Returns the entry index, or -1 if the workspace is full.
// A failed insert still takes its entry count (cnt becomes larger than C), so
// once one insert has failed every later call returns at once: the row has
// overflowed this workspace and is evaluated again in a larger one, and
// probing a table filled by failed inserts would cost H steps per call.
__device__ __forceinline__ int32_t ws_find_or_insert(Ws &w, int32_t k, bool &isnew) {
  isnew = true;
  if (__hip_atomic_load(w.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > w.C) return -1;
  uint32_t hh = ((uint32_t)k * 2654435761u) & (uint32_t)(w.H - 1);
  for (int32_t probe = 0; probe < w.H; ++probe) {
    const int32_t prev = atomicCAS(w.hkey + hh, -1, k);
    if (prev == -1) {
      const int32_t s = atomicAdd(w.cnt, 1);
      isnew = true;
      if (s >= w.C) {
        w.hslot[hh] = -1;
        return -1;
      }
      w.hslot[hh] = s;
      return s;
    }
    if (prev == k) {
      isnew = false;
      return w.hslot[hh];
    }
    hh = (hh + 1) & (uint32_t)(w.H - 1);
  }
  isnew = true;
  return -1;
}

// Rewrite row r toward target t (B = rows with cur >= t). Stops early with
// SUB_REJECT once more than capA A-columns exist (their number only grows).
// The entries still to substitute (state 1) are also listed in pend, so each
// step finds the largest of them by reading that list, not every entry.
__device__ int subst_row(Ws &w, int32_t r, int32_t t, const int32_t *__restrict__ rp,
                         const int32_t *__restrict__ ci, const double *__restrict__ va, const int32_t *cur,
                         int64_t capA, int32_t *nT_out) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  for (int32_t i = lane; i < w.H; i += 64) w.hkey[i] = -1;
  if (lane == 0) {
    *w.cnt = 0;
    *w.na = 0;
    *w.np = 0;
  }
  wave_sync();
  int overflow = 0;
  {
    const int32_t b = rp[r], e = rp[r + 1] - 1;
    for (int32_t p0 = b; p0 < e; p0 += 64) {  // the wave stops at the first overflow
      const int32_t p = p0 + lane;
      if (p < e) {
        const int32_t k = ci[p];
        bool isnew;
        const int32_t s = ws_find_or_insert(w, k, isnew);
        if (s < 0) {
          overflow = 1;
        } else {
          const bool inB = cur[k] >= t;
          w.col[s] = k;
          w.val[s] = va[p];
          w.st[s] = inB ? 1 : 0;
          if (inB)
            w.pend[atomicAdd(w.np, 1)] = s;
          else
            atomicAdd(w.na, 1);
        }
      }
      if (__ballot(overflow) != 0ull) break;
    }
  }
  wave_sync();
  if (__ballot(overflow) != 0ull) return SUB_OVERFLOW;
  if ((int64_t)*w.na > capA) return SUB_REJECT;
  int32_t nT = 0;
  for (;;) {
    // the largest column still to substitute, from the list of those entries
    const int32_t npend = *w.np;
    long long best = -1;
    for (int32_t i = lane; i < npend; i += 64) {
      const long long key = ((long long)w.col[w.pend[i]] << 32) | (long long)i;
      best = key > best ? key : best;
    }
    best = wave_max_ll(best);
    if (best < 0) break;
    const int32_t j = (int32_t)(best >> 32), ij = (int32_t)(best & 0xffffffffll);
    const int32_t sj = w.pend[ij];
    const double m = w.val[sj] / va[rp[j + 1] - 1];
    wave_sync();
    if (lane == 0) {
      w.st[sj] = 2;
      w.val[sj] = -m;
      w.pend[ij] = w.pend[npend - 1];
      *w.np = npend - 1;
    }
    wave_sync();
    ++nT;
    const int32_t jb = rp[j], je = rp[j + 1] - 1;
    for (int32_t p0 = jb; p0 < je; p0 += 64) {  // the wave stops at the first overflow
      const int32_t p = p0 + lane;
      if (p < je) {
        const int32_t k = ci[p];
        const double v = va[p];
        bool isnew;
        const int32_t s = ws_find_or_insert(w, k, isnew);
        if (s < 0) {
          overflow = 1;
        } else {
          const double prod = m * v;
          if (isnew) {
            const bool inB = cur[k] >= t;
            w.col[s] = k;
            w.val[s] = 0.0 - prod;
            w.st[s] = inB ? 1 : 0;
            if (inB)
              w.pend[atomicAdd(w.np, 1)] = s;
            else
              atomicAdd(w.na, 1);
          } else {
            w.val[s] = w.val[s] - prod;
          }
        }
      }
      if (__ballot(overflow) != 0ull) break;
    }
    wave_sync();
    if (__ballot(overflow) != 0ull) return SUB_OVERFLOW;
    if ((int64_t)*w.na > capA) return SUB_REJECT;
  }
  *nT_out = nT;
  return SUB_OK;
}

// Smallest and largest A column of the row just built in the workspace
// (wave-wide; {INT32_MAX, -1} when it has none).
__device__ __forceinline__ int2 ws_a_span(const Ws &w) {
  wave_sync();
  const int lane = threadIdx.x & 63;
  const int32_t nE = *w.cnt;
  int32_t lo = INT32_MAX, hi = -1;
  for (int32_t s = lane; s < nE; s += 64)
    if (w.st[s] == 0) {
      lo = w.col[s] < lo ? w.col[s] : lo;
      hi = w.col[s] > hi ? w.col[s] : hi;
    }
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t ol = __shfl_xor(lo, off, 64), oh = __shfl_xor(hi, off, 64);
    lo = ol < lo ? ol : lo;
    hi = oh > hi ? oh : hi;
  }
  return make_int2(lo, hi);
}

__device__ __forceinline__ Ws lds_ws(char *base, int wave) {
  // per wave: val[C] hkey[H] hslot[H] col[C] cnt na np - st[C] pend[C]
  constexpr size_t per = ws_core_bytes(kLdsC, kLdsH);
  constexpr size_t per_al = (per + 15) & ~(size_t)15;
  char *p = base + (size_t)wave * per_al;
  Ws w;
  w.val = reinterpret_cast<double *>(p);
  w.hkey = reinterpret_cast<int32_t *>(p + (size_t)kLdsC * 8);
  w.hslot = w.hkey + kLdsH;
  w.col = w.hslot + kLdsH;
  w.cnt = w.col + kLdsC;
  w.na = w.cnt + 1;
  w.np = w.na + 1;
  w.st = reinterpret_cast<uint8_t *>(w.na + 3);
  w.C = kLdsC;
  w.H = kLdsH;
  w.pend = reinterpret_cast<int32_t *>(w.st + ((w.C + 3) & ~3));
  return w;
}
constexpr size_t kLdsWsBytes = ((ws_core_bytes(kLdsC, kLdsH) + 15) & ~(size_t)15) * kWaves;

__device__ __forceinline__ Ws global_ws(char *base, int32_t C, int32_t H) {
  Ws w;
  w.val = reinterpret_cast<double *>(base);
  w.hkey = reinterpret_cast<int32_t *>(base + (size_t)C * 8);
  w.hslot = w.hkey + H;
  w.col = w.hslot + H;
  w.cnt = w.col + C;
  w.na = w.cnt + 1;
  w.np = w.na + 1;
  w.st = reinterpret_cast<uint8_t *>(w.na + 3);
  w.C = C;
  w.H = H;
  w.pend = reinterpret_cast<int32_t *>(w.st + ((w.C + 3) & ~3));
  return w;
}

struct ScanArgs {
  int32_t n, nlev;
  const int32_t *rp, *ci;
  const double *va;
  const int32_t *level_ptr, *level_rows;
  const int64_t *lv_rows, *lv_cost;
  const uint8_t *mask;
  int32_t metric;
  double W, fill_cap;
  const int32_t *lv_budget;  // optional per source level: row budget (THIN_ROWS), <= 0 = W
  const float *lv_cap;       // optional per source level: fill cap, <= 0 = fill_cap
  double Wmax;               // the largest row budget of any level (THIN_ROWS)
  int32_t max_dist;
  // row constraints (Sec. III.A): alpha, beta, and critical-path membership
  // of the original rows (null: no such constraint)
  int32_t max_indeg;
  int64_t max_spread;
  const uint8_t *oncrit;
  int32_t *skipped;  // rows a row constraint left in place
  int32_t *cur, *target, *cntL, *cntT;
  const int32_t *seg;            // first level of each segment, then nlev
  unsigned long long *claim;     // (next segment from the front) << 32 | (end of those left)
  size_t big_stride;             // bytes of global workspace per workgroup
  char *big;        // global workspace for candidates that overflow LDS
  int32_t bigC, bigH;
  int32_t *out;     // [0] rows moved [1] max distance [2] target steps [3] error bits
};

// Row budget (THIN_ROWS) and fill cap of the rows of source level lvl: the
// level's own where one is given and positive, else the options'.
__device__ __forceinline__ double level_budget(const ScanArgs &a, int32_t lvl) {
  return a.lv_budget && a.lv_budget[lvl] > 0 ? (double)a.lv_budget[lvl] : a.W;
}
__device__ __forceinline__ double level_cap(const ScanArgs &a, int32_t lvl) {
  return a.lv_cap && a.lv_cap[lvl] > 0.0f ? (double)a.lv_cap[lvl] : a.fill_cap;
}

// Whether a row constraint leaves candidate r (already within budget, fill
// and distance) where it is: na A columns spanning [lo, hi].
__device__ __forceinline__ bool row_held(const ScanArgs &a, int32_t r, int32_t na, int32_t lo, int32_t hi) {
  if (a.max_indeg > 0 && na >= a.max_indeg) return true;
  if (a.max_spread > 0 && na > 0 && (int64_t)hi - (int64_t)lo >= a.max_spread) return true;
  if (a.oncrit && !a.oncrit[r]) return true;
  return false;
}

// Size and cost of level lvl counting only its rows still there (the target a
// refusal creates keeps the rows skipped or not yet tried).
__device__ __forceinline__ void level_left(const ScanArgs &a, int32_t lvl, int64_t &size, int64_t &cost) {
  size = 0;
  cost = 0;
  for (int32_t p = a.level_ptr[lvl]; p < a.level_ptr[lvl + 1]; ++p) {
    const int32_t rr = a.level_rows[p];
    if (a.cur[rr] != lvl) continue;
    size += 1;
    cost += 2 * (int64_t)(a.rp[rr + 1] - a.rp[rr]) - 1;
  }
}

__device__ __forceinline__ bool is_source(const ScanArgs &a, int32_t lvl) {
  if (lvl == 0) return false;
  if (a.mask) return a.mask[lvl] != 0;
  if (a.metric == SPTRSV_THIN_ROWS) return (double)a.lv_rows[lvl] < a.W;
  return (double)a.lv_cost[lvl] < a.W;
}

// The segments of the scan: level 0 and every level that is not a source
// start one, and each runs to the next. A segment's scan reads nothing another
// segment decides: its rows move only to levels inside it, and a substitution
// expands only unknowns at or below the current target, while every row of an
// earlier segment, moved or not, sits below the segment's first level. One
// workgroup lists their first levels in order (ballot compaction) and sets the
// claim word to all of them.
__global__ __launch_bounds__(1024) void k_scan_segments(ScanArgs a, int32_t *seg) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t base;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) base = 0;
  __syncthreads();
  for (int32_t l0 = 0; l0 < a.nlev; l0 += 1024) {
    const int32_t l = l0 + tid;
    const bool f = l < a.nlev && !is_source(a, l);
    const unsigned long long m = __ballot(f);
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int32_t off = base;
    for (int w2 = 0; w2 < wave; ++w2) off += wsum[w2];
    if (f) seg[off + __popcll(m & ((1ull << lane) - 1ull))] = l;
    __syncthreads();
    if (tid == 0) {
      int32_t tot = 0;
      for (int w2 = 0; w2 < 16; ++w2) tot += wsum[w2];
      base += tot;
    }
    __syncthreads();
  }
  if (tid == 0) {
    seg[base] = a.nlev;
    *a.claim = (unsigned long long)(uint32_t)base;  // front 0, end base
  }
}

// Next segment for a workgroup taking them from the front (ascending) or from
// the end (descending); -1 when none is left. Two workgroups are the scan
// started at the beginning and at the end of the graph at once.
__device__ int32_t claim_segment(unsigned long long *claim, bool front) {
  unsigned long long old = __hip_atomic_load(claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const uint32_t lo = (uint32_t)(old >> 32), hi = (uint32_t)old;
    if (lo >= hi) return -1;
    const unsigned long long nw = front ? old + (1ull << 32) : old - 1ull;
    const unsigned long long prev = atomicCAS(claim, old, nw);
    if (prev == old) return front ? (int32_t)lo : (int32_t)(hi - 1);
    old = prev;
  }
}

// The decision scan: each workgroup takes segments (even-numbered workgroups
// from the front, odd ones from the end) and scans each in level order
// (targets only move forward). Thread 0 owns the scan state; waves evaluate
// candidates. The result does not depend on the number of workgroups.
__global__ __launch_bounds__(64 * kWaves) void k_rewrite_scan(ScanArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ int32_t c_row[kWaves], c_lvl[kWaves], c_q[kWaves], c_st[kWaves], c_na[kWaves], c_nt[kWaves];
  __shared__ int32_t c_lo[kWaves], c_hi[kWaves];
  __shared__ int32_t s_nc, s_done, s_redo, s_t;
  __shared__ int64_t s_capA_cost;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  Ws w = lds_ws(lds_raw, wave);
  char *const big = a.big + (size_t)blockIdx.x * a.big_stride;
  const bool front = (blockIdx.x & 1u) == 0u;
  // scan state (thread 0); the first chunk claims a segment
  int32_t t = 0, l = 0, q = 0, seg_end = 0, moved = 0, maxd = 0, steps = 0, held = 0;
  int64_t size = 0, cost = 0;
  int bits = 0;
  const int64_t guard = (int64_t)a.n + 2 * (int64_t)a.nlev + 16;
  for (int64_t iter = 0;; ++iter) {
    if (tid == 0) {
      // next chunk of candidates: rows of consecutive source levels of the
      // current segment, or of the next segment claimed
      int32_t nc = 0;
      for (;;) {
        int32_t limit = kWaves;
        if (a.metric == SPTRSV_THIN_ROWS) {
          const double room = a.Wmax - (double)size;  // rows the target can still take (at most)
          if (room < (double)kWaves) limit = room < 0.0 ? 1 : (int32_t)room + 1;
        }
        while (l < seg_end && nc < limit) {
          const int32_t lb = a.level_ptr[l], lr = a.level_ptr[l + 1] - lb;
          while (q < lr && nc < limit) {
            c_row[nc] = a.level_rows[lb + q];
            c_lvl[nc] = l;
            c_q[nc] = q;
            ++nc;
            ++q;
          }
          if (q == lr) {
            ++l;
            q = 0;
          }
        }
        if (nc > 0) break;
        const int32_t k = claim_segment(a.claim, front);
        if (k < 0) break;
        t = a.seg[k];
        seg_end = a.seg[k + 1];
        size = a.lv_rows[t];
        cost = a.lv_cost[t];
        ++steps;
        l = t + 1;
        q = 0;
      }
      s_nc = nc;
      s_t = t;
      s_done = (nc == 0) || iter > guard;
      if (iter > guard) bits |= EB_TIMEOUT;
      // bound on A columns: fill cap, and for a cost budget the room left
      int64_t capA = INT64_MAX;
      s_capA_cost = capA;
      if (a.metric == SPTRSV_THIN_COST) {
        // cost_t + 2*(nA+1) - 1 <= W  =>  nA <= (W - cost_t - 1) / 2
        const double room = a.W - (double)cost - 1.0;
        s_capA_cost = room < 0.0 ? -1 : (int64_t)(room / 2.0);
      }
    }
    __syncthreads();
    if (s_done) break;
    const int32_t nc = s_nc, tt = s_t;
    if (wave < nc) {
      const int32_t r = c_row[wave];
      const int64_t nnz_old = a.rp[r + 1] - a.rp[r];
      int64_t capA = s_capA_cost;
      const double capl = level_cap(a, c_lvl[wave]);
      if (capl > 0.0) {
        // nA + 1 <= fill_cap * nnz_old
        const double lim = capl * (double)nnz_old - 1.0;
        const int64_t c2 = lim < 0.0 ? -1 : (int64_t)lim;
        capA = c2 < capA ? c2 : capA;
      }
      int32_t nT = 0;
      int stt = subst_row(w, r, tt, a.rp, a.ci, a.va, a.cur, capA, &nT);
      Ws used = w;
      if (stt == SUB_OVERFLOW) {
        used = global_ws(big + (size_t)wave * kTier1Bytes, kTier1C, kTier1H);
        nT = 0;
        stt = subst_row(used, r, tt, a.rp, a.ci, a.va, a.cur, capA, &nT);
      }
      const int2 span = stt == SUB_OK && a.max_spread > 0 ? ws_a_span(used) : make_int2(0, 0);
      if (lane == 0) {
        c_st[wave] = stt;
        c_na[wave] = *used.na;
        c_nt[wave] = nT;
        c_lo[wave] = span.x;
        c_hi[wave] = span.y;
      }
    }
    __syncthreads();
    if (tid == 0) {
      s_redo = -1;
      for (int32_t i = 0; i < nc; ++i) {
        if (c_st[i] == SUB_OVERFLOW) {
          s_redo = i;
          break;
        }
        const int32_t r = c_row[i], lvl = c_lvl[i];
        const int64_t nnz_old = a.rp[r + 1] - a.rp[r];
        const int64_t nnz_new = (int64_t)c_na[i] + 1;
        bool ok = c_st[i] == SUB_OK;
        if (ok) {
          if (a.metric == SPTRSV_THIN_ROWS)
            ok = (double)(size + 1) <= level_budget(a, lvl);
          else
            ok = (double)(cost + 2 * nnz_new - 1) <= a.W;
          const double capl = level_cap(a, lvl);
          if (capl > 0.0) ok = ok && (double)nnz_new <= capl * (double)nnz_old;
          if (a.max_dist > 0) ok = ok && (lvl - t) <= a.max_dist;
        }
        if (ok && row_held(a, r, c_na[i], c_lo[i], c_hi[i])) {
          ++held;  // stays in its level; the scan position is already past it
          continue;
        }
        if (ok) {
          a.cur[r] = t;
          a.target[r] = t;
          a.cntL[r] = (int32_t)nnz_new;
          a.cntT[r] = c_nt[i] + 1;
          size += 1;
          cost += 2 * nnz_new - 1;
          ++moved;
          if (lvl - t > maxd) maxd = lvl - t;
          // the scan position is already past this candidate
        } else {
          // its level becomes the target with the rows not moved
          t = lvl;
          ++steps;
          level_left(a, lvl, size, cost);
          l = lvl + 1;
          q = 0;
          break;
        }
      }
      if (s_redo >= 0) {  // resume right at the overflowing candidate
        l = c_lvl[s_redo];
        q = c_q[s_redo];
      }
    }
    __syncthreads();
    if (s_redo >= 0) {
      // evaluate that candidate alone with the large global workspace
      if (wave == 0) {
        const int32_t i = s_redo, r = c_row[i];
        Ws g = global_ws(big, a.bigC, a.bigH);
        int32_t nT = 0;
        const int stt = subst_row(g, r, s_t, a.rp, a.ci, a.va, a.cur, INT64_MAX, &nT);
        const int2 span = stt == SUB_OK && a.max_spread > 0 ? ws_a_span(g) : make_int2(0, 0);
        if (lane == 0) {
          c_st[0] = stt;
          c_na[0] = *g.na;
          c_nt[0] = nT;
          c_lo[0] = span.x;
          c_hi[0] = span.y;
        }
      }
      __syncthreads();
      if (tid == 0) {
        const int32_t i = s_redo, r = c_row[i], lvl = c_lvl[i];
        if (c_st[0] == SUB_OVERFLOW) {
          bits |= EB_OVERFLOW;
          s_done = 1;
        } else {
          const int64_t nnz_old = a.rp[r + 1] - a.rp[r];
          const int64_t nnz_new = (int64_t)c_na[0] + 1;
          bool ok;
          if (a.metric == SPTRSV_THIN_ROWS)
            ok = (double)(size + 1) <= level_budget(a, lvl);
          else
            ok = (double)(cost + 2 * nnz_new - 1) <= a.W;
          const double capl = level_cap(a, lvl);
          if (capl > 0.0) ok = ok && (double)nnz_new <= capl * (double)nnz_old;
          if (a.max_dist > 0) ok = ok && (lvl - t) <= a.max_dist;
          const bool keep = ok && row_held(a, r, c_na[0], c_lo[0], c_hi[0]);
          if (keep) ++held;
          if (ok && !keep) {
            a.cur[r] = t;
            a.target[r] = t;
            a.cntL[r] = (int32_t)nnz_new;
            a.cntT[r] = c_nt[0] + 1;
            size += 1;
            cost += 2 * nnz_new - 1;
            ++moved;
            if (lvl - t > maxd) maxd = lvl - t;
          }
          if (ok) {  // moved or held: advance past it
            q = c_q[i] + 1;
            l = lvl;
            if (q == a.level_ptr[lvl + 1] - a.level_ptr[lvl]) {
              ++l;
              q = 0;
            }
          } else {
            t = lvl;
            ++steps;
            level_left(a, lvl, size, cost);
            l = lvl + 1;
            q = 0;
          }
        }
      }
      __syncthreads();
      if (s_done) break;
    }
  }
  if (tid == 0) {  // the outputs start at zero; every workgroup adds its part
    atomicAdd(a.out + 0, moved);
    atomicMax(a.out + 1, maxd);
    atomicAdd(a.out + 2, steps);
    if (bits) atomicOr(a.out + 3, bits);
    atomicAdd(a.skipped, held);
  }
}

// Rows not rewritten: copied; their T row is the unit row.
__global__ void k_copy_unmoved(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const double *__restrict__ va, const int32_t *__restrict__ target,
                               const int32_t *__restrict__ lrp, int32_t *lci, double *lva,
                               const int32_t *__restrict__ trp, int32_t *tci, double *tva) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    if (target[r] >= 0) continue;
    const int32_t b = rp[r], e = rp[r + 1];
    int32_t o = lrp[r];
    for (int32_t p = b; p < e; ++p, ++o) {
      lci[o] = ci[p];
      lva[o] = va[p];
    }
    tci[trp[r]] = (int32_t)r;
    tva[trp[r]] = 1.0;
  }
}

// Rows rewritten: recomputed with their final target (the B set of a row's
// step is exactly the rows whose final level is >= its target), then written
// in ascending column order with the diagonal last.
__global__ __launch_bounds__(64 * kWaves) void k_rewrite_rows(
    int32_t nrows, const int32_t *__restrict__ rows, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const double *__restrict__ va, const int32_t *__restrict__ cur, const int32_t *__restrict__ target,
    const int32_t *__restrict__ lrp, int32_t *lci, double *lva, const int32_t *__restrict__ trp, int32_t *tci,
    double *tva, char *big, int32_t bigC, int32_t bigH, int use_big, int *err) {
  extern __shared__ __align__(16) char lds_raw[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  Ws w = use_big ? global_ws(big + (size_t)(blockIdx.x * kWaves + wave) *
                                       (ws_core_bytes(bigC, bigH) + 48),
                             bigC, bigH)
                 : lds_ws(lds_raw, wave);
  const int64_t gw = (int64_t)blockIdx.x * kWaves + wave, nw = (int64_t)gridDim.x * kWaves;
  for (int64_t i = gw; i < nrows; i += nw) {
    const int32_t r = rows[i];
    const int32_t t = target[r];
    int32_t nT = 0;
    const int stt = subst_row(w, r, t, rp, ci, va, cur, INT64_MAX, &nT);
    if (stt != SUB_OK) {
      if (lane == 0) atomicOr(err, EB_OVERFLOW);
      continue;
    }
    const int32_t nA = *w.na, nE = *w.cnt;
    const int32_t lb = lrp[r], tb = trp[r];
    if (lrp[r + 1] - lb != nA + 1 || trp[r + 1] - tb != nT + 1) {
      if (lane == 0) atomicOr(err, EB_ARG);  // disagrees with the scan's counts
      continue;
    }
    for (int32_t s = lane; s < nE; s += 64) {
      const uint8_t cls = w.st[s];
      const int32_t c = w.col[s];
      int32_t rank = 0;
      for (int32_t s2 = 0; s2 < nE; ++s2) rank += (w.st[s2] == cls && w.col[s2] < c) ? 1 : 0;
      if (cls == 0) {
        lci[lb + rank] = c;
        lva[lb + rank] = w.val[s];
      } else {
        tci[tb + rank] = c;
        tva[tb + rank] = w.val[s];
      }
    }
    if (lane == 0) {
      lci[lb + nA] = r;
      lva[lb + nA] = va[rp[r + 1] - 1];
      tci[tb + nT] = r;
      tva[tb + nT] = 1.0;
    }
    wave_sync();
  }
}

// Row counts of L' and T (unmoved rows keep theirs), as int64 for the scan.
__global__ void k_row_counts(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ target,
                             const int32_t *__restrict__ cntL, const int32_t *__restrict__ cntT, long long *cl,
                             long long *ct) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const bool mv = target[r] >= 0;
    cl[r] = mv ? cntL[r] : rp[r + 1] - rp[r];
    ct[r] = mv ? cntT[r] : 1;
  }
}

// Compact the rewritten rows, split by the size of the workspace they need.
__global__ void k_collect_moved(int32_t n, const int32_t *__restrict__ target, const int32_t *__restrict__ cntL,
                                const int32_t *__restrict__ cntT, int32_t small_cap, int32_t *small_rows,
                                int32_t *nsmall, int32_t *big_rows, int32_t *nbig, int32_t *max_entries) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    if (target[r] < 0) continue;
    const int32_t ent = (cntL[r] - 1) + (cntT[r] - 1);
    if (ent <= small_cap) {
      small_rows[atomicAdd(nsmall, 1)] = (int32_t)r;
    } else {
      big_rows[atomicAdd(nbig, 1)] = (int32_t)r;
      atomicMax(max_entries, ent);
    }
  }
}

// Per-row inputs of the learned policy's level features: the row's
// off-diagonal count bin, the sizes of L'[r] and T[r] if its level alone were
// rewritten into the level before it (every other row in place: the B set is
// the rows at level >= lev(r) - 1 of the original levels), and the row
// constraints of Sec. III.A on that moved form (dependencies, column span) and
// on the row (longest-path membership). Level-0 rows count as they are. Rows
// whose rewrite outgrows the LDS workspace are listed for a second pass with a
// global workspace.
__global__ __launch_bounds__(64 * kWaves) void k_feat_rows(int32_t n, const int32_t *__restrict__ rows,
                                                           int32_t nrows, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const double *__restrict__ va,
                                                           const int32_t *__restrict__ lev, FeatAcc acc,
                                                           int32_t *redo, int32_t *nredo, char *big, int32_t bigC,
                                                           int32_t bigH, int *err) {
  extern __shared__ __align__(16) char lds_raw[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool use_big = big != nullptr;
  Ws w = use_big ? global_ws(big + (size_t)(blockIdx.x * kWaves + wave) * (ws_core_bytes(bigC, bigH) + 48),
                             bigC, bigH)
                 : lds_ws(lds_raw, wave);
  const int64_t total = rows ? nrows : n;
  const int64_t gw = (int64_t)blockIdx.x * kWaves + wave, nw = (int64_t)gridDim.x * kWaves;
  for (int64_t i = gw; i < total; i += nw) {
    const int32_t r = rows ? rows[i] : (int32_t)i;
    const int32_t l = lev[r];
    const int32_t off = rp[r + 1] - rp[r] - 1;
    int32_t lp = off + 1, tn = 1, na = off;
    int2 span = off > 0 ? make_int2(ci[rp[r]], ci[rp[r + 1] - 2]) : make_int2(INT32_MAX, -1);
    if (l > 0) {
      int32_t nT = 0;
      const int stt = subst_row(w, r, l - 1, rp, ci, va, lev, INT64_MAX, &nT);
      if (stt == SUB_OVERFLOW) {
        if (lane == 0) {
          if (use_big)
            atomicOr(err, EB_OVERFLOW);
          else
            redo[atomicAdd(nredo, 1)] = r;
        }
        wave_sync();
        continue;
      }
      na = *w.na;
      lp = na + 1;
      tn = nT + 1;
      span = ws_a_span(w);
    }
    if (lane == 0) {
      atomicAdd((unsigned long long *)(acc.sum_lp + l), (unsigned long long)lp);
      atomicAdd((unsigned long long *)(acc.sum_t + l), (unsigned long long)tn);
      const int64_t sp = span.y >= 0 ? (int64_t)span.y - span.x : 0;
      atomicAdd((unsigned long long *)(acc.sum_span + l), (unsigned long long)sp);
      // counted once per row: rows sent to the second pass skipped this block
      const int bin = off == 0 ? 0 : off == 1 ? 1 : off == 2 ? 2 : off <= 4 ? 3 : off <= 8 ? 4 : 5;
      int32_t *hl = acc.hist + (int64_t)l * kFeatHist;
      atomicAdd(hl + bin, 1);
      if (na < 4) atomicAdd(hl + 6, 1);
      if (acc.oncrit[r]) atomicAdd(hl + 7, 1);
      if (sp < 1024) atomicAdd(hl + 8, 1);
    }
    wave_sync();
  }
}

// Critical-path membership of the rows of L from two level numberings:
// row_level[r] (longest path from a source to r) and levr[n - 1 - r], the
// 1-based level of row n - 1 - r in J L^T J, whose rows are the dependents of
// the rows of L in reverse order, so that levr[n - 1 - r] - 1 is the height of
// r (longest path from r to a row nothing depends on).
// oncrit[r] = level(r) + height(r) == nlev - 1.

}  // namespace


size_t rewrite_big_ws_bytes(int32_t C, int32_t H) { return ws_core_bytes(C, H) + 48; }

hipError_t launch_rewrite_scan(int32_t n, int32_t nlev, const int32_t *rp, const int32_t *ci, const double *va,
                               const int32_t *level_ptr, const int32_t *level_rows, const int64_t *lv_rows,
                               const int64_t *lv_cost, const uint8_t *mask, int32_t metric, double W, double fill_cap,
                               const int32_t *lv_budget, const float *lv_cap, double Wmax,
                               int32_t max_dist, int32_t max_indeg, int64_t max_spread, const uint8_t *oncrit,
                               int32_t *skipped, int32_t *cur, int32_t *target, int32_t *cntL, int32_t *cntT,
                               int32_t workers, int32_t *seg, unsigned long long *claim, char *big, int32_t bigC,
                               int32_t bigH, int32_t *out, hipStream_t s) {
  if (workers < 1) return hipErrorInvalidValue;
  ScanArgs a;
  a.n = n;
  a.nlev = nlev;
  a.rp = rp;
  a.ci = ci;
  a.va = va;
  a.level_ptr = level_ptr;
  a.level_rows = level_rows;
  a.lv_rows = lv_rows;
  a.lv_cost = lv_cost;
  a.mask = mask;
  a.metric = metric;
  a.W = W;
  a.fill_cap = fill_cap;
  a.lv_budget = lv_budget;
  a.lv_cap = lv_cap;
  a.Wmax = Wmax > W ? Wmax : W;
  a.max_dist = max_dist;
  a.max_indeg = max_indeg;
  a.max_spread = max_spread;
  a.oncrit = oncrit;
  a.skipped = skipped;
  a.cur = cur;
  a.target = target;
  a.cntL = cntL;
  a.cntT = cntT;
  a.seg = seg;
  a.claim = claim;
  a.big = big;
  a.bigC = bigC;
  a.bigH = bigH;
  a.big_stride = rewrite_big_ws_bytes(bigC, bigH);  // one full workspace per workgroup
  // the full workspace also holds the waves' first-retry regions
  if (a.big_stride < (size_t)kWaves * kTier1Bytes) return hipErrorInvalidValue;
  a.out = out;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rewrite_scan),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsWsBytes);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rewrite_rows),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsWsBytes);
    attr = true;
  }
  hipLaunchKernelGGL(k_scan_segments, dim3(1), dim3(1024), 0, s, a, seg);
  hipLaunchKernelGGL(k_rewrite_scan, dim3(workers), dim3(64 * kWaves), kLdsWsBytes, s, a);
  return hipGetLastError();
}

int32_t rewrite_lds_capacity() { return kLdsC; }

hipError_t launch_row_counts(int32_t n, const int32_t *rp, const int32_t *target, const int32_t *cntL,
                             const int32_t *cntT, long long *cl, long long *ct, hipStream_t s) {
  hipLaunchKernelGGL(k_row_counts, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, rp, target, cntL, cntT, cl, ct);
  return hipGetLastError();
}

hipError_t launch_collect_moved(int32_t n, const int32_t *target, const int32_t *cntL, const int32_t *cntT,
                                int32_t *small_rows, int32_t *nsmall, int32_t *big_rows, int32_t *nbig,
                                int32_t *max_entries, hipStream_t s) {
  hipLaunchKernelGGL(k_collect_moved, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, target, cntL, cntT, kLdsC,
                     small_rows, nsmall, big_rows, nbig, max_entries);
  return hipGetLastError();
}

hipError_t launch_copy_unmoved(int32_t n, const int32_t *rp, const int32_t *ci, const double *va,
                               const int32_t *target, const int32_t *lrp, int32_t *lci, double *lva,
                               const int32_t *trp, int32_t *tci, double *tva, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_unmoved, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, rp, ci, va, target, lrp, lci,
                     lva, trp, tci, tva);
  return hipGetLastError();
}

hipError_t launch_rewrite_rows(int32_t nrows, const int32_t *rows, const int32_t *rp, const int32_t *ci,
                               const double *va, const int32_t *cur, const int32_t *target, const int32_t *lrp,
                               int32_t *lci, double *lva, const int32_t *trp, int32_t *tci, double *tva, char *big,
                               int32_t bigC, int32_t bigH, int32_t big_blocks, int *err, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const bool use_big = big != nullptr;
  const int blocks = use_big ? big_blocks : grid_for(nrows, kWaves, 2048);
  hipLaunchKernelGGL(k_rewrite_rows, dim3(blocks), dim3(64 * kWaves), use_big ? 0 : kLdsWsBytes, s, nrows, rows, rp,
                     ci, va, cur, target, lrp, lci, lva, trp, tci, tva, big, bigC, bigH, use_big ? 1 : 0, err);
  return hipGetLastError();
}

int32_t rewrite_waves_per_block() { return kWaves; }

hipError_t launch_feat_rows(int32_t n, const int32_t *rows, int32_t nrows, const int32_t *rp, const int32_t *ci,
                            const double *va, const int32_t *lev, FeatAcc acc, int32_t *redo, int32_t *nredo,
                            char *big, int32_t bigC, int32_t bigH, int32_t big_blocks, int *err, hipStream_t s) {
  const int64_t total = rows ? nrows : n;
  if (total <= 0) return hipSuccess;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_feat_rows),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsWsBytes);
    attr = true;
  }
  const bool use_big = big != nullptr;
  const int blocks = use_big ? big_blocks : grid_for(total, kWaves, 4096);
  hipLaunchKernelGGL(k_feat_rows, dim3(blocks), dim3(64 * kWaves), use_big ? 0 : kLdsWsBytes, s, n, rows, nrows, rp,
                     ci, va, lev, acc, redo, nredo, big, bigC, bigH, err);
  return hipGetLastError();
}
