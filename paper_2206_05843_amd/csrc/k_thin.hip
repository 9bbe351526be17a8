// Thin-run solve kernels: level-by-level forward substitution (Sec. II.A,
// Algorithm 1) over the level-ordered copy of L, or of the rewritten L'
// (Sec. II.B) after the b-transform b' = T b (applied before the level chain
// starts, since it does not depend on x). Wide levels are in k_wide.hip.
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
#include "sync.h"

namespace {

constexpr int kWinBytes = 159 * 1024;  // dynamic LDS of a thin-run workgroup (of the CU's 160 KB)
// Its first 16 bytes hold control words (no static LDS in these kernels: it
// would offset the dynamic region and misalign its 16-byte records); the
// window layout starts after them.
constexpr int kCtlBytes = 16;
struct Ctl {
  int32_t next;  // batched launch: the workgroup's next queue ticket
  int32_t pad[3];
};


// A thin run is cut into LDS windows (consecutive levels, chosen on the host so
// that the window's rows and dependency records fit in LDS). Per window:
//  phase 1 (all rows in parallel): the window's static image, built once per
//    schedule, is streamed into LDS: per row an inline record {w0, w1 | slot0,
//    slot1, count, first overflow} of its first two in-window dependencies
//    (weights scaled by 1/L(pos,pos); absent ones point to a zero entry with
//    weight 0, so phase 2 needs no predication) and a list of {weight, slot}
//    records for its third and later ones. Meanwhile each thread loads, for
//    several rows at once, b', the diagonal and the row's range of
//    dependencies on earlier windows, then forms
//    v = (b' - sum of L(pos,k) x(k)) / L(pos,pos) over those (final values,
//    read from global memory, in the row's column order);
//  phase 2 (level by level): x = v - sum over in-window dependencies of w x,
//    in LDS only;
//  then the window's x goes to global memory in one coalesced pass (where the
//    finiteness check happens too), before the next window reads it.
// When every level of the window has at most one item per thread, phase 2 is
// software-pipelined: the next level's records are requested before the
// current level is computed, and the level bounds are read from registers,
// so a level waits only for the x values it reads. Windows whose levels have
// at most 64 items run phase 2 on one wave without workgroup barriers.
// win[i] = {first level, flags}; the run's last entry holds the end level.
// kTimed (used only to label levels for the learned policy): thread 0 stamps the
// device wall clock around every level and writes per-level times (ns).
constexpr int kBatch = 4;

// acc - sum_j w_j x(slot_j, c) over n overflow records starting at d, in order,
// in batches of 4 (tail clamped to a valid record).
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
  double acc, w0, w1;
  uint2 r;  // packed slots/count/offset, unpacked where used (a prefetch never waits for it)
  int32_t s, c, act;
};

template <bool kOne>
__device__ __forceinline__ Item load_item(int32_t pb, int32_t items, int32_t t, int32_t nr, const double *v,
                                          const double2 *rw, const uint2 *rix) {
  Item it;
  it.act = t < items;
  it.s = kOne ? pb + t : pb + t / nr;
  it.c = kOne ? 0 : t - (it.s - pb) * nr;
  const int32_t ss = it.act ? it.s : pb;
  const double2 w = rw[ss];
  it.w0 = w.x;
  it.w1 = w.y;
  it.r = rix[ss];
  it.acc = v[(int64_t)ss * nr + (it.act ? it.c : 0)];
  return it;
}

template <bool kOne>
__device__ __forceinline__ double solve_item(const Item &it, int32_t nr, const double *v, const Dep *ovf) {
  const int32_t c = it.c;
  const int32_t s0 = (int32_t)(it.r.x & 0xffffu), s1 = (int32_t)(it.r.x >> 16);
  const int32_t cnt = (int32_t)(it.r.y & 0xffffu), ob = (int32_t)(it.r.y >> 16);
  const double xa = v[(int64_t)s0 * (kOne ? 1 : nr) + c];
  const double xb = v[(int64_t)s1 * (kOne ? 1 : nr) + c];
  double acc = it.acc - it.w0 * xa;
  acc = acc - it.w1 * xb;
  if (cnt > 2) acc = ovf_sum<kOne>(acc, ovf + ob, cnt - 2, v, nr, c);
  return acc;
}

// Phase 1: (row, rhs) items per thread whose loads are in flight together,
// and 16-byte image units per thread per copy round.
template <int WG, bool kOne>
constexpr int p1_items() {
  return WG >= 1024 ? 5 : WG >= 512 ? 6 : 8;
}
template <int WG>
constexpr int p1_copy() {
  return WG >= 1024 ? 8 : 12;
}

// The windows [win, win + nwin) of one thin run, by the calling workgroup,
// for the ng right-hand sides c0 .. c0 + ng - 1 of the nrhs (kOne: ng = 1).
// The columns are independent, so a run can be split over several
// workgroups by columns; LDS holds ng values per row (windows are cut for ng
// columns). Returns the latched error bits; a window that does not fit aborts
// the run.
// kSplit: the run is split over workgroups by columns (ng < nrhs); without it
// the strides and the first column are compile-time where they can be.
template <int WG, bool kOne, bool kTimed, bool kSplit = false>
__device__ __forceinline__ int thin_run_body(char *lds_raw, const int4 *__restrict__ win, int32_t nwin, int32_t nrhs,
                                             int32_t ng, int32_t c0_arg, const ThinArgs &A, float *times,
                                             float ns_per_tick, unsigned *prog = nullptr, unsigned ptag = 0) {
  double *lds = reinterpret_cast<double *>(lds_raw + kCtlBytes);
  const int32_t nr = kOne && !kSplit ? 1 : nrhs;  // stride of the global vectors
  const int32_t gw = kOne ? 1 : ng;               // columns in LDS and per row of items
  const int32_t c0 = kSplit ? c0_arg : 0;         // the first of those columns
  const int tid = threadIdx.x;
  const int32_t *__restrict__ level_ptr = A.level_ptr;
  const double *__restrict__ sdg = A.sdg;
  const int32_t *__restrict__ ext_ptr = A.ext_ptr;
  const ExtDep *__restrict__ ext = A.ext;
  const double *__restrict__ bp = A.bp;
  double *xp = A.xp;
  const double *xs = A.rio.x ? A.rio.x : xp;  // where the x of earlier windows is read
  int bits = 0;
  unsigned long long t_w0 = 0, t_prev = 0;
  float p1_per_row = 0.f;
  for (int32_t w = 0; w < nwin; ++w) {
    if (prog && tid == 0) __hip_atomic_store(prog, ptag | (unsigned)w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (kTimed && tid == 0) t_w0 = wall_clock64();
    const int4 W = win[w];
    const int32_t lA = W.x, lB = win[w + 1].x, flags = W.y;
    const int32_t P0 = level_ptr[lA], P1 = level_ptr[lB];
    const int32_t R = P1 - P0;
    const int32_t NO = W.z;  // the window's overflow records
    const int32_t NL = lB - lA;
    // the host sizes windows to fit, and 16-bit slots and offsets must hold R and NO
    if (thin_window_bytes(R, NO, NL, gw) > kWinBytes - kCtlBytes || R >= 65536 || NO >= 65536) return bits | EB_ARG;
    double2 *rw = reinterpret_cast<double2 *>(lds);          // [R] w0, w1 (scaled by 1/diagonal)
    Dep *ovf = reinterpret_cast<Dep *>(rw + R);               // [NO] third and later dependencies
    uint2 *rix = reinterpret_cast<uint2 *>(ovf + NO);         // [R, padded to even] slot0, slot1, count, overflow
    double *v = reinterpret_cast<double *>(rix + ((R + 1) & ~1));  // [(R + 1) * gw] partial sums, then x; zero row R
    int32_t *lv = reinterpret_cast<int32_t *>(v + (int64_t)(R + 1) * gw);  // [NL + 1] level bounds from P0
    // phase 1. Each thread requests its items' right-hand side, diagonal and
    // range of dependencies before the window; in the first round it streams
    // the window's static image into LDS while those are in flight; then it
    // subtracts the dependencies before the window (in the row's column order).
    const int32_t nitems = R * gw;
    constexpr int kI = p1_items<WG, kOne>();
    for (int32_t base = 0; base < nitems; base += WG * kI) {
      double acc[kI], dg[kI];
      int32_t e0[kI], e1[kI];
#pragma unroll
      for (int j = 0; j < kI; ++j) {
        const int32_t it = base + j * WG + tid;
        const int32_t itc = it < nitems ? it : nitems - 1;
        const int32_t sj = kOne ? itc : itc / gw;
        const int32_t pos = P0 + sj;
        const int32_t cj = c0 + (kOne ? 0 : itc - sj * gw);
        // right-hand sides stored by rows: the caller's b through the level
        // order, except rows of T with off-diagonals (b' in bp)
        if (A.rio.b && !(A.rio.tflag && A.rio.tflag[pos]))
          acc[j] = A.rio.b[(int64_t)A.rio.perm[pos] * nr + cj];
        else
          acc[j] = bp[(int64_t)pos * nr + cj];
        dg[j] = sdg[pos];
        e0[j] = ext_ptr[pos];
        e1[j] = it < nitems ? ext_ptr[pos + 1] : e0[j];
      }
      if (base == 0) {
        for (int32_t i = tid; i <= NL; i += WG) lv[i] = level_ptr[lA + i] - P0;
        for (int32_t i = tid; i < gw; i += WG) v[(int64_t)R * gw + i] = 0.0;
        const uint4 *__restrict__ im = A.img + W.w;
        uint4 *dst = reinterpret_cast<uint4 *>(lds);
        const int32_t nu = (int32_t)window_image_units(R, NO);
        constexpr int kC = p1_copy<WG>();
        for (int32_t u0 = 0; u0 < nu; u0 += WG * kC) {
          uint4 t[kC];
#pragma unroll
          for (int j = 0; j < kC; ++j) {
            const int32_t u = u0 + j * WG + tid;
            t[j] = im[u < nu ? u : nu - 1];
          }
#pragma unroll
          for (int j = 0; j < kC; ++j) {
            const int32_t u = u0 + j * WG + tid;
            if (u < nu) dst[u] = t[j];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kI; ++j) {
        const int32_t it = base + j * WG + tid;
        if (it >= nitems) continue;
        const int32_t c = c0 + (kOne ? 0 : it - (it / gw) * gw);
        double a = acc[j];
        for (int32_t e = e0[j]; e < e1[j]; e += kBatch) {
          double wv[kBatch], xv[kBatch];
          int32_t k[kBatch];
#pragma unroll
          for (int d = 0; d < kBatch; ++d) {
            const ExtDep x = ext[e + d < e1[j] ? e + d : e];
            wv[d] = x.w;
            k[d] = A.rio.x ? x.row : x.col;
          }
          // by rows the caller's x is the work vector, read by caller row
#pragma unroll
          for (int d = 0; d < kBatch; ++d) xv[d] = xs[(int64_t)k[d] * nr + c];
#pragma unroll
          for (int d = 0; d < kBatch; ++d)
            if (e + d < e1[j]) a -= wv[d] * xv[d];
        }
        v[(int64_t)it] = a * (1.0 / dg[j]);
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
        // levels in chunks of 63: lane i holds the bound of level c0 + i, read
        // once per chunk, so a level's bounds come from registers
        for (int32_t c0 = 0; c0 < NL; c0 += 63) {
          const int32_t nlc = NL - c0 < 63 ? NL - c0 : 63;
          const int32_t lvreg = lv[c0 + lane <= NL ? c0 + lane : NL];
          int32_t pb = __builtin_amdgcn_readlane(lvreg, 0);
          int32_t items = (__builtin_amdgcn_readlane(lvreg, 1) - pb) * gw;
          Item cur = load_item<kOne>(pb, items, tid, gw, v, rw, rix);
          for (int32_t l = 0; l < nlc; ++l) {
            Item nxt = cur;
            if (l + 1 < nlc) {
              pb = __builtin_amdgcn_readlane(lvreg, l + 1);
              items = (__builtin_amdgcn_readlane(lvreg, l + 2) - pb) * gw;
              nxt = load_item<kOne>(pb, items, tid, gw, v, rw, rix);
            }
            if (cur.act) v[(int64_t)cur.s * gw + cur.c] = solve_item<kOne>(cur, gw, v, ovf);
            if (one_wave)
              wave_lds_barrier();
            else
              lds_barrier();  // LDS only: the global x is read only across a window restart
            if (kTimed && tid == 0) {
              const int32_t lg = c0 + l;
              const unsigned long long now = wall_clock64();
              times[lA + lg] = (float)(now - t_prev) * ns_per_tick + p1_per_row * (float)(lv[lg + 1] - lv[lg]);
              t_prev = now;
            }
            cur = nxt;
          }
        }
      }
    } else {
      for (int32_t l = 0; l < NL; ++l) {
        const int32_t pb = lv[l], items = (lv[l + 1] - pb) * gw;
        for (int32_t t = tid; t < items; t += WG) {
          const Item it = load_item<kOne>(pb, items, t, gw, v, rw, rix);
          v[(int64_t)it.s * gw + it.c] = solve_item<kOne>(it, gw, v, ovf);
        }
        lds_barrier();
        if (kTimed && tid == 0) {
          const unsigned long long now = wall_clock64();
          times[lA + l] = (float)(now - t_prev) * ns_per_tick + p1_per_row * (float)(lv[l + 1] - lv[l]);
          t_prev = now;
        }
      }
    }
    __syncthreads();  // every x of the window is in LDS
    for (int32_t i = tid; i < nitems; i += WG) {
      const double x = v[i];
      if (!isfinite(x)) bits |= EB_NONFINITE;
      if (!A.rio.x && gw == nr) {  // all columns in this workgroup: the window is one contiguous block
        xp[(int64_t)P0 * nr + i] = x;
        continue;
      }
      const int32_t sj = kOne ? i : i / gw;
      const int32_t cj = c0 + (kOne ? 0 : i - sj * gw);
      if (A.rio.x)  // by rows: the caller's x only
        A.rio.x[(int64_t)A.rio.perm[P0 + sj] * nr + cj] = x;
      else
        xp[(int64_t)(P0 + sj) * nr + cj] = x;
    }
    __syncthreads();  // the window's global x is complete before the next phase 1 reads it
  }
  return bits;
}

// L2 prefetch helpers of a single thin run. One workgroup solves; a few more
// workgroups on the same XCD (workgroups are dispatched to the 8 XCDs in turn,
// so workgroup 8 h shares workgroup 0's L2) touch one word of every cache line
// of the next windows' images, b', diagonals and outside-dependency lists, so
// the solver's phase 1 finds them in L2. They keep at most kAhead windows ahead
// of the solver, which publishes (epoch tag | window) in tp[1] as it starts
// each window and advances the epoch tp[0] when it ends; launches on a stream
// do not overlap, so the epoch read at the start names this launch. The solver
// never waits for a helper; a helper stops when the epoch moves on, when it
// has done its windows, or when one wait exceeds kWaitTicks of the device
// wall clock, so every helper finishes.
constexpr int kXcd = 8;
constexpr int kHelp = 4;            // helpers per launch
constexpr int kAhead = 4;           // windows a helper may run ahead of the solver
constexpr int kHelpMinWin = 8;      // runs with fewer windows launch no helpers
constexpr unsigned long long kWaitTicks = 5000;  // 50 us at the 100 MHz wall clock
constexpr int kTagShift = 20;       // progress word: (epoch mod 2^12) << 20 | window

__device__ __forceinline__ unsigned epoch_tag(unsigned ep) { return (ep & 0xfffu) << kTagShift; }

template <int WG>
__device__ void prefetch_windows(char *lds_raw, const int4 *__restrict__ win, int32_t nwin, int32_t nrhs,
                                 const ThinArgs &A, int hh) {
  int32_t &s_go = reinterpret_cast<Ctl *>(lds_raw)->next;
  unsigned *tp = A.tp;
  const int tid = threadIdx.x;
  const unsigned ep = __hip_atomic_load(tp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned sink = 0;
  for (int32_t j = hh; j < nwin; j += kHelp) {
    if (tid == 0) {
      int go = 1;
      const unsigned long long t0 = wall_clock64();
      for (;;) {
        if (__hip_atomic_load(tp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ep) {
          go = 0;  // the solver has finished
          break;
        }
        const unsigned p = __hip_atomic_load(tp + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t at = (p >> kTagShift) == (ep & 0xfffu) ? (int32_t)(p & ((1u << kTagShift) - 1)) : 0;
        if (j <= at + kAhead) break;
        if (wall_clock64() - t0 > kWaitTicks) {
          go = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      s_go = go;
    }
    __syncthreads();
    if (!s_go) break;
    const int4 W = win[j];
    const int32_t P0 = A.level_ptr[W.x], P1 = A.level_ptr[win[j + 1].x], R = P1 - P0;
    const int32_t nu = (int32_t)window_image_units(R, W.z);
    const uint4 *im = A.img + W.w;
    for (int32_t u = tid * 8; u < nu; u += WG * 8) sink ^= im[u].x;
    const double *bw = A.bp + (int64_t)P0 * nrhs;
    for (int32_t u = tid * 16; u < R * nrhs; u += WG * 16) sink ^= (unsigned)__double_as_longlong(bw[u]);
    for (int32_t u = tid * 16; u < R; u += WG * 16) sink ^= (unsigned)__double_as_longlong(A.sdg[P0 + u]);
    for (int32_t u = tid * 32; u <= R; u += WG * 32) sink ^= (unsigned)A.ext_ptr[P0 + u];
    const int32_t e0 = A.ext_ptr[P0], e1 = A.ext_ptr[P1];
    for (int32_t e = e0 + tid * 8; e < e1; e += WG * 8) sink ^= (unsigned)A.ext[e].col;
    __syncthreads();  // s_go is rewritten only after every thread has read it
  }
  if (sink == 0x9e3779b9u) tp[2] = sink;  // keeps the loads; the value is never read
}

// One thin run: workgroup g < nrhs / ng solves columns g*ng .. g*ng + ng - 1;
// with one solver (ng = nrhs) the launcher may add prefetch helpers after it.
template <int WG, bool kOne, bool kTimed = false, bool kSplit = false>
__global__ __launch_bounds__(WG) void k_thin_run(const int4 *__restrict__ win, int32_t nwin, int32_t nrhs, int32_t ng,
                                                 ThinArgs A, int *err, float *times, float ns_per_tick) {
  extern __shared__ __align__(16) char lds_raw[];
  const int32_t nsolver = nrhs / ng;
  if ((int32_t)blockIdx.x >= nsolver) {  // helpers exist only when the launcher gave the grid room for them
    if (blockIdx.x % kXcd == 0) prefetch_windows<WG>(lds_raw, win, nwin, nrhs, A, (int)(blockIdx.x / kXcd) - 1);
    return;
  }
  unsigned ep = 0;
  if (A.tp) ep = __hip_atomic_load(A.tp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int bits = thin_run_body<WG, kOne, kTimed, kSplit>(lds_raw, win, nwin, nrhs, ng, (int32_t)blockIdx.x * ng, A,
                                                           times, ns_per_tick, A.tp ? A.tp + 1 : nullptr,
                                                           epoch_tag(ep));
  if (threadIdx.x == 0) {
    if (bits) atomicOr(err, bits);
    if (A.tp) __hip_atomic_store(A.tp, ep + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// A row's first four off-diagonals (column position, value), -1 / 0 padded.
__global__ void k_fill_ell(int32_t n, const int32_t *__restrict__ srp, const int32_t *__restrict__ sci,
                           const double *__restrict__ sva, int4 *ell_c, double2 *ell_v) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t qb = srp[p], deg = srp[p + 1] - qb;
    int32_t c[4];
    double v[4];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      c[d] = d < deg ? sci[qb + d] : -1;
      v[d] = d < deg ? sva[qb + d] : 0.0;
    }
    ell_c[p] = make_int4(c[0], c[1], c[2], c[3]);
    ell_v[2 * p] = make_double2(v[0], v[1]);
    ell_v[2 * p + 1] = make_double2(v[2], v[3]);
  }
}

// Many independent matrices in one persistent launch: each workgroup takes
// the next matrix from a device queue (matrices are queued largest first) and
// solves all of it with the thin-run windows of that matrix; the levels of a
// matrix are separated by workgroup barriers. The last workgroup to finish
// resets the queue, so the launch can be replayed (graph capture) without a
// host-side reset. q[0] = next ticket, q[1] = finished workgroups.
template <int WG, bool kOne>
__global__ __launch_bounds__(WG) void k_batch_run(int32_t nmat, const int32_t *__restrict__ order,
                                                  const int32_t *__restrict__ mwin, const int4 *__restrict__ win,
                                                  int32_t nrhs, ThinArgs A, unsigned *q, int *err) {
  extern __shared__ __align__(16) char lds_raw[];
  int32_t &s_m = reinterpret_cast<Ctl *>(lds_raw)->next;
  int bits = 0;
  for (;;) {
    if (threadIdx.x == 0) s_m = (int32_t)atomicAdd(q, 1u);
    __syncthreads();
    const int32_t t = s_m;
    __syncthreads();
    if (t >= nmat) break;
    const int32_t m = order[t];
    bits |= thin_run_body<WG, kOne, false>(lds_raw, win + mwin[m], mwin[m + 1] - mwin[m] - 1, nrhs, nrhs, 0, A,
                                           nullptr, 0.f);
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

template <int WG, bool kOne>
void set_lds_attr() {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_thin_run<WG, kOne>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_thin_run<WG, kOne, false, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
}

}  // namespace

int thin_win_bytes() { return kWinBytes - kCtlBytes; }

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

hipError_t launch_thin_run(int wg, const int4 *win, int32_t nwin, int32_t nrhs, const ThinArgs &a, int *err,
                           hipStream_t s, float *times, float ns_per_tick, int32_t ng) {
  if (ng <= 0 || ng > nrhs || nrhs % ng || times) ng = nrhs;  // labelling runs are never split
  const bool one = ng == 1;
  const bool split = ng < nrhs;
  ThinArgs aa = a;
  unsigned grid = (unsigned)(nrhs / ng);  // one solver per group of ng columns
  if (grid == 1) {
    // the solver, plus kHelp prefetch helpers on its XCD for runs long enough
    // to use them (windows are numbered below 2^20 in the progress word)
    if (a.tp && nwin >= kHelpMinWin && nwin < (1 << kTagShift)) grid = 1 + kXcd * kHelp;
  } else {
    aa.tp = nullptr;  // several solvers: no helpers, no progress words
  }
  if (times) {  // labelling runs only: 512 threads
    if (one)
      hipLaunchKernelGGL((k_thin_run<512, true, true>), dim3(grid), dim3(512), kWinBytes, s, win, nwin, nrhs, ng, aa,
                         err, times, ns_per_tick);
    else
      hipLaunchKernelGGL((k_thin_run<512, false, true>), dim3(grid), dim3(512), kWinBytes, s, win, nwin, nrhs, ng,
                         aa, err, times, ns_per_tick);
    return hipGetLastError();
  }
#define THIN(W)                                                                                              \
  if (split && one)                                                                                          \
    hipLaunchKernelGGL((k_thin_run<W, true, false, true>), dim3(grid), dim3(W), kWinBytes, s, win, nwin, nrhs,  \
                       ng, aa, err, (float *)nullptr, 0.f);                                                  \
  else if (split)                                                                                            \
    hipLaunchKernelGGL((k_thin_run<W, false, false, true>), dim3(grid), dim3(W), kWinBytes, s, win, nwin, nrhs, \
                       ng, aa, err, (float *)nullptr, 0.f);                                                  \
  else if (one)                                                                                              \
    hipLaunchKernelGGL((k_thin_run<W, true>), dim3(grid), dim3(W), kWinBytes, s, win, nwin, nrhs, ng, aa, err,  \
                       (float *)nullptr, 0.f);                                                               \
  else                                                                                                       \
    hipLaunchKernelGGL((k_thin_run<W, false>), dim3(grid), dim3(W), kWinBytes, s, win, nwin, nrhs, ng, aa, err, \
                       (float *)nullptr, 0.f);
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

hipError_t launch_fill_ell(int32_t n, const int32_t *srp, const int32_t *sci, const double *sva, int4 *ell_c,
                           double2 *ell_v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_ell, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, n, srp, sci, sva, ell_c, ell_v);
  return hipGetLastError();
}

template <int WG>
void batch_attr() {
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_run<WG, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch_run<WG, false>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, kWinBytes);
}

hipError_t launch_batch_run(int wg, int32_t nmat, int32_t grid, const int32_t *order, const int32_t *mwin,
                            const int4 *win, int32_t nrhs, const ThinArgs &a, unsigned *q, int *err, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    batch_attr<256>();
    batch_attr<512>();
    batch_attr<1024>();
    attr = true;
  }
#define BATCH(W)                                                                                                \
  if (nrhs == 1)                                                                                                \
    hipLaunchKernelGGL((k_batch_run<W, true>), dim3(grid), dim3(W), kWinBytes, s, nmat, order, mwin, win, nrhs, a, \
                       q, err);                                                                                 \
  else                                                                                                          \
    hipLaunchKernelGGL((k_batch_run<W, false>), dim3(grid), dim3(W), kWinBytes, s, nmat, order, mwin, win, nrhs,   \
                       a, q, err);
  if (wg == 256) {
    BATCH(256)
  } else if (wg == 1024) {
    BATCH(1024)
  } else {
    BATCH(512)
  }
#undef BATCH
  return hipGetLastError();
}

int batch_resident_blocks(int wg) {
  int dev = 0, cus = 256, occ = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void *f = wg == 256    ? reinterpret_cast<const void *>(&k_batch_run<256, false>)
                  : wg == 1024 ? reinterpret_cast<const void *>(&k_batch_run<1024, false>)
                               : reinterpret_cast<const void *>(&k_batch_run<512, false>);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, wg, kWinBytes);
  return cus * (occ > 0 ? occ : 1);
}
