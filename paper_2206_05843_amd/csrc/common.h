// Internal declarations of libsptrsv: device buffers, the handle, plans and
// the host-side launchers of every kernel. Nothing here is part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "sptrsv.h"

// Error bits latched on the device (atomicOr into a handle-owned int).
enum : int {
  EB_ARG = 1 << 0,
  EB_NOT_LOWER = 1 << 1,
  EB_UNSORTED = 1 << 2,
  EB_MISSING_DIAG = 1 << 3,
  EB_ZERO_PIVOT = 1 << 4,
  EB_NONFINITE = 1 << 5,
  EB_OVERFLOW = 1 << 6,
  EB_TIMEOUT = 1 << 7,
};
sptrsv_status_t status_from_bits(int bits);

// Owned device array (hipMalloc'd, freed on destruction or re-allocation).
template <class T>
struct DArr {
  T *p = nullptr;
  size_t n = 0;
  DArr() = default;
  DArr(const DArr &) = delete;
  DArr &operator=(const DArr &) = delete;
  DArr(DArr &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr, o.n = 0; }
  DArr &operator=(DArr &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p, n = o.n, o.p = nullptr, o.n = 0;
    }
    return *this;
  }
  ~DArr() { release(); }
  hipError_t alloc(size_t count) {
    release();
    if (count == 0) count = 1;  // keep a valid pointer for empty arrays
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = count;
    return hipSuccess;
  }
  // grow-only allocation
  hipError_t reserve(size_t count) { return count <= n && p ? hipSuccess : alloc(count); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// One in-window dependency beyond a row's two inline ones: weight scaled by
// 1/diagonal and the slot (row of the window) it reads.
struct __align__(16) Dep {
  double w;
  int32_t slot, pad;
};

// One dependency on a row before the row's LDS window: the unscaled weight,
// the position whose final x it reads, and that position's row in the
// caller's numbering (where a solve by rows reads it).
struct __align__(16) ExtDep {
  double w;
  int32_t col, row;
};

// One run of the solve schedule: a range of levels done inside one workgroup
// (thin) or a single level spread over the device (wide).
struct Run {
  int32_t l0, l1;  // levels [l0, l1)
  bool thin;
  int32_t wi = 0, nw = 0;  // thin: its LDS windows in Plan::win [wi, wi + nw], entry wi + nw = end
  bool flow = false;       // a dataflow run (schedule mode 4) of wide levels
  int32_t nchunk = 0;      // flow: its chunks, chunk_pos [cp, cp + nchunk], dptr [cp, cp + nchunk], flags [fl, ...)
  int32_t cp = 0, fl = 0;
  int32_t lc = 0;          // flow: level_chunk [lc, lc + l1 - l0]: first chunk of each level of the run
  int32_t max_chunks = 0;  // flow: chunks of its widest level
  bool longr = false;      // one wide level of long rows, several right-hand sides: a workgroup per row
};

// What a dataflow run reads (pointers already offset to the run's chunks):
// chunk c holds positions [chunk_pos[c], chunk_pos[c + 1]) and waits for the
// chunks dlist[dptr[c] .. dptr[c + 1]) of the same run; level l of the run
// holds chunks [level_chunk[l], level_chunk[l + 1]); flags[c] holds the tag of
// the launch that finished it; ctl = {unused, workgroups done, epoch}.
struct FlowArgs {
  const int32_t *chunk_pos, *dptr, *dlist, *level_chunk;
  unsigned *flags, *ctl;
  const int32_t *srp, *sci;
  const double *sva, *sdg;
  const int4 *ell_c;
  const double2 *ell_v;
  const double *bp;
  double *xp;
};

// Everything needed to solve one lower-triangular matrix level by level:
// its level sets, a level-ordered copy with columns renumbered to positions,
// the optional b-transform T (off-diagonals, same numbering) and work vectors.
struct Plan {
  bool ready = false;
  int32_t n = 0, nlev = 0;
  int64_t nnz = 0;                     // nonzeros including the diagonal
  DArr<int32_t> level_ptr;             // [nlev+1] positions
  DArr<int32_t> perm;                  // [n] position -> row (= level_rows)
  DArr<int32_t> iperm;                 // [n] row -> position
  // reversed systems (U x = b, L^T x = b): the caller's numbering is the
  // reverse of the lower form's; these maps replace perm/iperm for b and x
  bool rev_io = false;
  DArr<int32_t> perm_io, iperm_io;
  DArr<int32_t> row_level;             // [n]
  std::vector<int32_t> h_level_ptr;    // host copy for scheduling
  DArr<int32_t> srp, sci;              // level-ordered off-diagonal CSR
  DArr<double> sva, sdg;               // values, diagonal per position
  bool has_t = false;
  int64_t nnz_t_off = 0;
  DArr<int32_t> trp, tci;              // T off-diagonals per position (columns: caller's rows)
  DArr<double> tva;
  DArr<int32_t> tpos;                  // positions whose row of T has off-diagonals
  DArr<uint8_t> tflag;                 // 1 at those positions (solves by rows; built on demand)
  DArr<int4> ell_r;                    // [n] ell_c in the caller's rows (solves by rows; built on demand)
  DArr<int32_t> sci_r;                 // [nnz - n] sci in the caller's rows (the same)
  bool rows_ready = false;
  int32_t n_tpos = 0;
  int32_t t_lanes = 1;                 // lanes per row of T in the b-transform
  DArr<int64_t> lv_rows, lv_nnz, lv_cost;
  std::vector<int64_t> h_lv_nnz;       // per level: nnz incl. diagonal (host copy)
  std::vector<int64_t> h_lv_tnnz;      // per level: off-diagonal nnz of T
  DArr<int4> ell_c;                    // [n] first four off-diagonal columns per position (-1: none)
  DArr<double2> ell_v;                 // [2n] their values
  std::vector<int32_t> h_xh;           // [nlev * kExtraBuckets] level-distance histogram of dependencies
                                       // that need overflow records when inside an LDS window
  int64_t total_cost = 0;
  double avg_cost = 0.0;
  sptrsv_schedule_t sched{};           // knobs in force (mode 0 = automatic)
  std::map<int32_t, sptrsv_schedule_t> tuned;  // per nrhs
  std::vector<Run> runs;
  // LDS windows of all thin runs {first level, flags, overflow records, image
  // offset in 16-byte units}; each run's list ends with {end level, -1, 0, 0}
  std::vector<int4> h_win;
  DArr<int4> win;
  DArr<uint4> img;                     // static window images, back to back
  DArr<int32_t> ext_ptr;               // [n+1] dependencies before the row's window (CSR over positions)
  DArr<ExtDep> ext;
  int32_t runs_nrhs = -1;
  sptrsv_schedule_t runs_sched{};
  // Overlap of the layout transposes with the level chain (large solves): the
  // chain's runs are cut into segments at levels seg_lvl[k]; gather group k
  // (the caller-row tiles of 64 rows whose first position lies in segment k)
  // and the b-transform of segment k's rows run on the handle's side stream
  // before segment k starts, and scatter group k (tiles whose last position
  // lies in segment k) after it ends, while later segments run.
  bool ovl = false;
  std::vector<int32_t> seg_run;        // [K+1] first run of each segment
  std::vector<int32_t> g_off, s_off;   // [K+1] offsets of each group in g_tiles / s_tiles
  std::vector<int32_t> t_off;          // [K+1] offsets of each segment's rows of T in tpos
  DArr<int32_t> g_tiles, s_tiles;
  std::vector<int32_t> h_tpos;         // host copy of tpos
  // dataflow runs (mode 4): chunk tables of all flow runs, back to back
  DArr<int32_t> flow_pos, flow_dptr, flow_dlist, flow_lc;
  DArr<unsigned> flow_flags, flow_ctl;
  std::vector<int32_t> h_srp, h_sci;   // host copy of the level-ordered pattern (built on first use)
  DArr<double> bp, xp;                 // [n * nrhs] permuted, RHS-interleaved
  DArr<unsigned> tp;                   // [4] thin-run launches: epoch, progress, helper sink
  DArr<unsigned long long> sf_ticket;  // [1] ticket counter of the synchronisation-free solve
  DArr<unsigned> wbar;                 // [2] barrier counters of persistent wide runs (zero between launches)
  int32_t work_nrhs = 0;
};

// Index maps between positions and the caller's rows.
inline const int32_t *io_perm(const Plan &P) { return P.rev_io ? P.perm_io.p : P.perm.p; }
inline const int32_t *io_iperm(const Plan &P) { return P.rev_io ? P.iperm_io.p : P.iperm.p; }

struct BatchMat {
  int32_t n;
  int64_t row_off, nnz_off;
};

// A batched matrix with a level too wide for an LDS window at the cached
// nrhs: solved level by level beside the persistent launch.
struct BatchWide {
  int32_t m = 0;
  std::vector<Run> runs;
};

struct Graph {
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
};

struct sptrsv_ctx {
  int dev = 0;
  std::string last_error;
  DArr<int32_t> d_err;     // latched error bits of solves
  DArr<int32_t> d_aux;     // small scratch: counters, tickets, maxima
  // the matrix in lower-triangular form (owned; for the other triangular forms
  // its conversion, see form)
  int32_t form = SPTRSV_LOWER;
  int32_t n = 0;
  int64_t nnz = 0;
  DArr<int32_t> rp, ci;
  DArr<double> va;
  Plan orig, rew;
  // rewritten matrix in original numbering
  bool has_rewrite = false;
  DArr<int32_t> lp_rp, lp_ci, t_rp, t_ci, target;
  DArr<double> lp_va, t_va;
  sptrsv_rewrite_stats_t rstats{};
  DArr<char> rw_big;       // global workspace of the decision scan
  // batched matrices
  // batched matrices: one plan over the block-diagonal union whose positions
  // are grouped by matrix, then by level (levels of matrix m are
  // [b_lvl_off[m], b_lvl_off[m+1]) of the plan)
  int32_t b_nmat = 0;
  bool b_ready = false;
  Plan bat;
  std::vector<int32_t> b_n, b_nlev;
  std::vector<int64_t> b_row_off, b_lvl_off;
  DArr<int32_t> b_rp, b_ci, b_mat_of_row, b_order, b_mwin;
  DArr<double> b_va;
  DArr<int64_t> b_row_off_d;           // [nmat+1]
  DArr<unsigned> b_q;                  // persistent-launch queue counters
  std::vector<int32_t> b_h_mwin;       // window index of each matrix's run, for the cached nrhs
  std::vector<int32_t> b_h_order;      // longest-processing-time order of all matrices
  int32_t b_nq = 0;                    // matrices in the persistent queue (b_order) for the cached nrhs
  std::vector<BatchWide> b_wide;       // the others
  int32_t b_win_nrhs = -1, b_win_wg = -1;
  std::vector<Graph> graphs;
  // live profile of solve launches
  bool prof = false;
  std::vector<hipEvent_t> prof_ev;   // 2 per recorded launch
  std::vector<int> prof_cls;
  std::vector<double> prof_bytes;
  size_t prof_used = 0;
  // scan scratch
  DArr<long long> scan_tmp;
  // bounded device-side waits of solves (synchronisation-free and persistent
  // launches), in ticks of the 100 MHz wall clock; 0 = the default 10 s. The
  // autotuner lowers it per candidate.
  unsigned long long wait_ticks = 0;
  sptrsv_tune_info_t tune_info{};
  // side stream (default priority) and events of the overlapped transposes
  hipStream_t side = nullptr;
  std::vector<hipEvent_t> ovl_ev;
};

// Per-device address of the static work area of sptrsv_solve_noalloc
// (api_noalloc.hip), looked up once per device.
hipError_t noalloc_init(int dev);

// Wait limit of a solve launch in wall-clock ticks.
inline unsigned long long wait_limit(const sptrsv_ctx *h) {
  return h->wait_ticks ? h->wait_ticks : 100000000ull * 10;
}

// Status plumbing ------------------------------------------------------------
sptrsv_status_t set_err(sptrsv_ctx *h, sptrsv_status_t st, const char *fmt, ...);
#define HIPCHK(h, expr)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_err((h), e_ == hipErrorOutOfMemory ? SPTRSV_ERR_ALLOC : SPTRSV_ERR_HIP,     \
                     "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)
#define STCHK(expr)                          \
  do {                                       \
    sptrsv_status_t st_ = (expr);            \
    if (st_ != SPTRSV_OK) return st_;        \
  } while (0)

// Launchers (k_analyze.hip) ----------------------------------------------------
hipError_t launch_validate(int32_t n, int32_t nnz, const int32_t *rp, const int32_t *ci, const double *va, int *err,
                           hipStream_t s);
hipError_t launch_levels(int32_t n, const int32_t *rp, const int32_t *ci, int32_t *lev1, unsigned *ticket, int *err,
                         hipStream_t s);
hipError_t launch_max(const int32_t *a, int32_t n, int32_t *out, hipStream_t s);
// Heights by position (hp zeroed by the caller) from the plan's level-ordered
// copy, last level first; then the longest-path flags of the rows.
hipError_t launch_heights(int32_t n, int32_t nlev, const int32_t *level_ptr, const int32_t *h_level_ptr,
                          const int32_t *srp, const int32_t *sci, int32_t *hp, hipStream_t s);
hipError_t launch_crit_from_heights(int32_t n, int32_t nlev, const int32_t *perm, const int32_t *row_level,
                                    const int32_t *hp, uint8_t *oncrit, hipStream_t s);
// exclusive scan of int64 values in place-compatible form: out may equal in
size_t scan_scratch_elems(int64_t n);
hipError_t launch_scan_i64(const long long *in, long long *out, int64_t n, long long *scratch, hipStream_t s);
hipError_t launch_radix_by_key(int32_t *keys, int32_t *vals, int32_t *keys_tmp, int32_t *vals_tmp, int32_t n,
                               int bits, int32_t *hist, long long *hist64, long long *scratch, hipStream_t s);
size_t radix_hist_elems(int32_t n);
hipError_t launch_level_ptr_from_sorted(const int32_t *sorted_keys, int32_t n, int32_t *level_ptr, int32_t nlev,
                                        hipStream_t s);
hipError_t launch_iota(int32_t *a, int32_t n, hipStream_t s);
hipError_t launch_invert_perm(const int32_t *perm, int32_t n, int32_t *iperm, hipStream_t s);
hipError_t launch_sub1(const int32_t *a, int32_t n, int32_t *out, hipStream_t s);
hipError_t launch_count_off(const int32_t *perm, const int32_t *rp, int32_t n, long long *cnt, hipStream_t s);
hipError_t launch_ptr_from_scan(const long long *ex, const long long *cnt, int32_t n, int32_t *ptr, int *err,
                                hipStream_t s);
hipError_t launch_fill_solve(int32_t n, const int32_t *perm, const int32_t *iperm, const int32_t *rp,
                             const int32_t *ci, const double *va, const int32_t *srp, int32_t *sci, double *sva,
                             double *sdg, hipStream_t s);
// rev: T's columns go to the caller's numbering of a reversed system (n-1-c)
hipError_t launch_fill_t(int32_t n, const int32_t *perm, const int32_t *trp, const int32_t *tci,
                         const double *tva, const int32_t *strp, int32_t *stci, double *stva, bool rev, hipStream_t s);
hipError_t launch_level_stats(int32_t nlev, const int32_t *level_ptr, const int32_t *srp, int64_t *rows,
                              int64_t *nnz, int64_t *cost, long long *total, hipStream_t s);

// LDS bytes of a thin-run window of `rows` rows, `ovf` overflow dependency
// records and `nl` levels: per row the partial sum or x of every RHS (8 nrhs),
// two inline weights (16) and packed slots/count/offset (8); one zero entry
// per RHS that absent dependencies point to; 16 per overflow record; the level
// bounds; 16 for aligning the window's sections.
__host__ __device__ inline int64_t thin_window_bytes(int64_t rows, int64_t ovf, int64_t nl, int32_t nrhs) {
  return rows * (8 * (int64_t)nrhs + 24) + 8 * (int64_t)nrhs + ovf * 16 + 4 * (nl + 1) + 16;
}

// Inline record of a row: slots, in-window dependency count and first
// overflow record, 16 bits each (a window holds far fewer than 65536 rows or
// records).
__host__ __device__ inline uint2 pack_rix(int32_t s0, int32_t s1, int32_t cnt, int32_t ob) {
  return make_uint2((uint32_t)s0 | ((uint32_t)s1 << 16), (uint32_t)cnt | ((uint32_t)ob << 16));
}

// 16-byte units of a window's static image: weights (one unit per row),
// overflow records (one each), packed records (two rows per unit).
__host__ __device__ inline int64_t window_image_units(int64_t rows, int64_t ovf) {
  return rows + ovf + ((rows + 1) >> 1);
}

// Level-distance buckets of the overflow-record histogram: lower bounds of
// the distances 1, 2, 3, 4, 5-8, 9-16, 17-32, 33-64, 65-256, >256.
constexpr int kExtraBuckets = 10;
constexpr int32_t kExtraLo[kExtraBuckets] = {1, 2, 3, 4, 5, 9, 17, 33, 65, 257};

// Workgroups for a grid-stride launch over `items` items, at most `cap`.
inline int grid_for(int64_t items, int threads, int cap = 1 << 20) {
  int64_t g = (items + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Device arrays a thin run reads: level bounds, diagonal, the static window
// images and each position's dependencies before its window (CSR), and the
// work vectors.
// Right-hand sides stored by rows (b null: the work vectors only): b is read
// at b[perm[pos] * nrhs + c] except where tflag[pos] marks a row of T with
// off-diagonals (b' already in the work vector), and x is written to
// x[perm[pos] * nrhs + c] only: the caller's x is the work vector, and
// dependencies are read from it through caller rows (ell_r: a position's
// first four dependencies as caller rows, -1 padded; sci_r: every column).
struct RowsIO {
  const double *b;
  double *x;
  const int32_t *perm;
  const uint8_t *tflag;
  const int4 *ell_r;
  const int32_t *sci_r;  // the level-ordered copy's columns as caller rows
};

struct ThinArgs {
  const int32_t *level_ptr;
  const double *sdg;
  const uint4 *img;
  const int32_t *ext_ptr;
  const ExtDep *ext;
  const double *bp;
  double *xp;
  unsigned *tp;  // pacing words of the L2 prefetch helpers of a single-run launch (null: no helpers)
  RowsIO rio;
};

// Launchers (k_solve.hip) ------------------------------------------------------
hipError_t launch_gather(int32_t n, int32_t nrhs, const double *b, int64_t ldb, const int32_t *iperm, double *bp,
                         hipStream_t s);
// lanes: 1 (a thread per row and column of b) or 4, 16, 64 (a group per row)
// b's entry (row, c) at b[row * rs + c * cs]: rs = 1, cs = ldb column-major;
// rs = nrhs, cs = 1 by rows.
hipError_t launch_apply_t(int32_t nt, int32_t nrhs, int32_t lanes, const int32_t *tpos, const int32_t *perm,
                          const int32_t *trp, const int32_t *tcol, const double *tva, const double *b, int64_t rs,
                          int64_t cs, double *bp, hipStream_t s);
// Right-hand sides stored by rows: bp[pos * nrhs + c] = b[perm[pos] * nrhs + c],
// x[perm[pos] * nrhs + c] = xp[pos * nrhs + c]; tflag[tpos[i]] = 1 (zeroed first).
hipError_t launch_gather_rows(int32_t n, int32_t nrhs, const double *b, const int32_t *perm, double *bp,
                              hipStream_t s);
hipError_t launch_scatter_rows(int32_t n, int32_t nrhs, const double *xp, const int32_t *perm, double *x,
                               hipStream_t s);
hipError_t launch_tflag(int32_t n, int32_t nt, const int32_t *tpos, uint8_t *tflag, hipStream_t s);
// ell_r[p] = ell_c[p] with every position k >= 0 replaced by perm[k]
hipError_t launch_map_ell(int32_t n, const int4 *ell_c, const int32_t *perm, int4 *ell_r, hipStream_t s);
// out[q] = perm[col[q]]
hipError_t launch_map_cols(int64_t nnz, const int32_t *col, const int32_t *perm, int32_t *out, hipStream_t s);
hipError_t launch_scatter(int32_t n, int32_t nrhs, const double *xp, const int32_t *iperm, double *x, int64_t ldx,
                          hipStream_t s);
// The same over a list of caller-row tiles of 64 rows.
hipError_t launch_gather_tiles(int32_t n, int32_t nrhs, const double *b, int64_t ldb, const int32_t *iperm,
                               const int32_t *tiles, int32_t ntiles, double *bp, hipStream_t s);
hipError_t launch_scatter_tiles(int32_t n, int32_t nrhs, const double *xp, const int32_t *iperm,
                                const int32_t *tiles, int32_t ntiles, double *x, int64_t ldx, hipStream_t s);
// Row sums b = A 1, and out[0..1] = bits of max |x1 - x0| and max |x0|
// (out zeroed by the caller; NaN counts as infinite).
hipError_t launch_row_sums(int32_t n, const int32_t *rp, const double *va, double *b, hipStream_t s);
hipError_t launch_max_abs_diff(int32_t n, const double *x0, const double *x1, unsigned long long *out,
                               hipStream_t s);
// First and last position of the rows of every caller-row tile of 64 rows.
hipError_t launch_tile_span(int32_t n, const int32_t *iperm, int32_t *first, int32_t *last, hipStream_t s);
int thin_win_bytes();
hipError_t launch_extra_hist(int32_t n, const int32_t *level_ptr, int32_t nlev, const int32_t *srp,
                             const int32_t *sci, int32_t *lop, int32_t *hist, hipStream_t s);
// ng: right-hand sides per solver workgroup (a divisor of nrhs; 0 = all)
hipError_t launch_thin_run(int wg, const int4 *win, int32_t nwin, int32_t nrhs, const ThinArgs &a, int *err,
                           hipStream_t s, float *times = nullptr, float ns_per_tick = 0.f, int32_t ng = 0);
hipError_t launch_fill_ell(int32_t n, const int32_t *srp, const int32_t *sci, const double *sva, int4 *ell_c,
                           double2 *ell_v, hipStream_t s);
hipError_t launch_wide_level(int threads, int lanes_per_row, int32_t pb, int32_t pe, int32_t nrhs,
                             const int32_t *srp, const int32_t *sci, const double *sva, const double *sdg,
                             const int4 *ell_c, const double2 *ell_v, const double *bp, double *xp, int *err,
                             hipStream_t s, RowsIO rio = RowsIO{});
// One wide level [pb, pe) with a workgroup per row (long rows, 2 <= nrhs <= 256;
// avg_deg: the level's off-diagonals per row, which sizes the workgroup).
hipError_t launch_wide_long(int32_t pb, int32_t pe, int32_t nrhs, int32_t avg_deg, const int32_t *srp,
                            const int32_t *sci, const double *sva, const double *sdg, const double *bp, double *xp,
                            int *err, hipStream_t s, RowsIO rio = RowsIO{});
hipError_t launch_wide_run(int grid, int threads, int32_t l0, int32_t l1, const int32_t *level_ptr, int32_t nrhs,
                           const int32_t *srp, const int32_t *sci, const double *sva, const double *sdg,
                           const int4 *ell_c, const double2 *ell_v, const double *bp, double *xp, unsigned *bar,
                           int *err, unsigned long long tlimit, hipStream_t s, RowsIO rio = RowsIO{});
int wide_run_resident_blocks(int threads);
// rev: b and x in the reversed (caller's) numbering of the lower form
hipError_t launch_residual(int32_t n, int32_t nrhs, const int32_t *rp, const int32_t *ci, const double *va,
                           const double *b, int64_t ldb, const double *x, int64_t ldx, unsigned long long *out,
                           bool rev, hipStream_t s);
void solve_kernels_init();

// Launchers (k_rewrite.hip) ----------------------------------------------------
size_t rewrite_big_ws_bytes(int32_t C, int32_t H);
int32_t rewrite_lds_capacity();
int32_t rewrite_waves_per_block();
hipError_t launch_rewrite_scan(int32_t n, int32_t nlev, const int32_t *rp, const int32_t *ci, const double *va,
                               const int32_t *level_ptr, const int32_t *level_rows, const int64_t *lv_rows,
                               const int64_t *lv_cost, const uint8_t *mask, int32_t metric, double W, double fill_cap,
                               const int32_t *lv_budget, const float *lv_cap, double Wmax,
                               int32_t max_dist, int32_t max_indeg, int64_t max_spread, const uint8_t *oncrit,
                               int32_t *skipped, int32_t *cur, int32_t *target, int32_t *cntL, int32_t *cntT,
                               int32_t workers, int32_t *seg, unsigned long long *claim, char *big, int32_t bigC,
                               int32_t bigH, int32_t *out, hipStream_t s);
hipError_t launch_row_counts(int32_t n, const int32_t *rp, const int32_t *target, const int32_t *cntL,
                             const int32_t *cntT, long long *cl, long long *ct, hipStream_t s);
hipError_t launch_collect_moved(int32_t n, const int32_t *target, const int32_t *cntL, const int32_t *cntT,
                                int32_t *small_rows, int32_t *nsmall, int32_t *big_rows, int32_t *nbig,
                                int32_t *max_entries, hipStream_t s);
hipError_t launch_copy_unmoved(int32_t n, const int32_t *rp, const int32_t *ci, const double *va,
                               const int32_t *target, const int32_t *lrp, int32_t *lci, double *lva,
                               const int32_t *trp, int32_t *tci, double *tva, hipStream_t s);
hipError_t launch_rewrite_rows(int32_t nrows, const int32_t *rows, const int32_t *rp, const int32_t *ci,
                               const double *va, const int32_t *cur, const int32_t *target, const int32_t *lrp,
                               int32_t *lci, double *lva, const int32_t *trp, int32_t *tci, double *tva, char *big,
                               int32_t bigC, int32_t bigH, int32_t big_blocks, int *err, hipStream_t s);

// Launchers (k_mlp.hip, k_rewrite.hip features) -----------------------------------
int mlp_backward_parts();
hipError_t launch_mlp_forward(const float *P, const float *feat, const float *norm, int32_t B, float *prob,
                              hipStream_t s);
hipError_t launch_mlp_backward(const float *P, const float *feat, const float *norm, const float *label,
                               const float *weight, int32_t B, float *part, float *part_loss, float *grad,
                               float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *P, const float *g, float *m, float *v, float lr, float c1, float c2,
                           hipStream_t s);
hipError_t launch_mlp_mask(const float *prob, int32_t nlev, float thr, uint8_t *mask, hipStream_t s);
struct MlpTiers {
  int32_t n;
  float thr[4];
  int32_t budget[4];
  float cap[4];
};
hipError_t launch_mlp_actions(const float *prob, int32_t nlev, const MlpTiers &t, uint8_t *mask, int32_t *budget,
                              float *cap, hipStream_t s);
// Per-level sums behind the learned policy's level features, filled row by row:
// hist[l * kFeatHist + b] holds the off-diagonal count bins (b < 6) and the
// counts of rows passing the row-constraint tests (6: fewer than 4 dependencies
// after the move, 7: on a longest path, 8: span under 1024 columns).
constexpr int kFeatHist = 9;
struct FeatAcc {
  long long *sum_lp, *sum_t, *sum_span;
  int32_t *hist;
  const uint8_t *oncrit;  // longest-path membership per row
};
hipError_t launch_feat_finalize(int32_t nlev, const int64_t *rows, const int64_t *nnz, const int64_t *cost,
                                double avg, FeatAcc acc, float *feat, hipStream_t s);
hipError_t launch_feat_rows(int32_t n, const int32_t *rows, int32_t nrows, const int32_t *rp, const int32_t *ci,
                            const double *va, const int32_t *lev, FeatAcc acc, int32_t *redo, int32_t *nredo,
                            char *big, int32_t bigC, int32_t bigH, int32_t big_blocks, int *err, hipStream_t s);
// Window images (k_image.hip) ------------------------------------------------------
// Per position: overflow records and dependencies before its window (zero for
// positions outside thin windows); lvl_win maps a level to its window in win
// (-1: not in a thin run).
hipError_t launch_img_count(int32_t n, const int32_t *level_ptr, int32_t nlev, const int32_t *lvl_win,
                            const int4 *win, const int32_t *srp, const int32_t *sci, long long *ovf_cnt,
                            long long *ext_cnt, hipStream_t s);
// Per window-table entry e: the overflow prefix at the entry's first position.
hipError_t launch_win_prefix(int32_t nent, const int4 *win, const int32_t *level_ptr, int32_t n,
                             const long long *ovf_ex, const long long *ovf_cnt, long long *out, hipStream_t s);
hipError_t launch_img_fill(int32_t n, const int32_t *level_ptr, int32_t nlev, const int32_t *lvl_win, const int4 *win,
                           const int32_t *srp, const int32_t *sci, const double *sva, const double *sdg,
                           const long long *ovf_ex, const int32_t *ext_ptr, uint4 *img, ExtDep *ext,
                           const int32_t *perm, hipStream_t s);
// Batched launchers (k_solve.hip) -------------------------------------------------
hipError_t launch_batch_run(int wg, int32_t nmat, int32_t grid, const int32_t *order, const int32_t *mwin,
                            const int4 *win, int32_t nrhs, const ThinArgs &a, unsigned *q, int *err, hipStream_t s);
hipError_t launch_batch_gather(int64_t total, int32_t nrhs, const double *b, const int32_t *mat_of_row,
                               const int64_t *row_off, const int32_t *iperm, double *bp, hipStream_t s);
hipError_t launch_batch_scatter(int64_t total, int32_t nrhs, const double *xp, const int32_t *mat_of_row,
                                const int64_t *row_off, const int32_t *iperm, double *x, hipStream_t s);
int batch_resident_blocks(int wg);
sptrsv_schedule_t effective_sched(const Plan &P, int32_t nrhs);
Plan *plan_of(sptrsv_ctx *h, int which);
Plan *sched_plan_of(sptrsv_ctx *h, int which);
sptrsv_schedule_t default_schedule();
// Schedule helpers (api.hip) -----------------------------------------------------
bool level_fits_window(const Plan &P, int32_t l, int32_t nrhs);
int32_t cut_windows(const Plan &P, int32_t l0, int32_t l1, int32_t nrhs, int32_t wg, std::vector<int4> &out);
sptrsv_status_t build_extra_hist(sptrsv_ctx *h, Plan &P, hipStream_t s);
sptrsv_status_t make_runs(sptrsv_ctx *h, Plan &P, int32_t nrhs, const sptrsv_schedule_t &sc, hipStream_t s);
sptrsv_status_t build_images(sptrsv_ctx *h, Plan &P, hipStream_t s);
sptrsv_status_t ensure_work(sptrsv_ctx *h, Plan &P, int32_t nrhs);

// Plan building (api.hip) --------------------------------------------------------
// Longest-path membership flags of the rows of the handle's lower matrix
// (plan P of it): oncrit[r] = level(r) + height(r) == nlev - 1. Synchronous.
sptrsv_status_t crit_rows(sptrsv_ctx *h, const Plan &P, uint8_t *oncrit, hipStream_t s);
sptrsv_status_t build_plan(sptrsv_ctx *h, Plan &P, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                           const double *va, const int32_t *trp, const int32_t *tci, const double *tva,
                           hipStream_t s, bool rev_io = false);
// Dataflow run (k_flow.hip): workgroups of wg threads (128, 256 or 512), grid
// 0 = as many as are resident.
int flow_items_per_thread();
hipError_t launch_flow_run(int wg, int grid, const FlowArgs &a, int32_t nlev, int32_t max_chunks, int32_t nrhs,
                           int *err, unsigned long long tlimit, hipStream_t s);
// Synchronisation-free solve of the whole plan (k_syncfree.hip): bp -> xp.
// blocks: workgroups of 256 threads (0: 512). stamp (optional, n * nrhs):
// the device wall clock when each item's value was written.
hipError_t launch_syncfree(int32_t n, int32_t nrhs, const int32_t *srp, const int32_t *sci, const double *sva,
                           const double *sdg, const double *bp, double *xp, unsigned long long *ticket, int *err,
                           int32_t blocks, unsigned long long tlimit, hipStream_t s,
                           unsigned long long *stamp = nullptr);
// times[l] = (latest stamp of level l - earliest stamp of all) * ns_per_tick;
// lmax has nlev entries, *gmin must hold ~0 before the call.
hipError_t launch_stamp_levels(int32_t nlev, int32_t nrhs, const int32_t *level_ptr, const unsigned long long *stamp,
                               unsigned long long *lmax, unsigned long long *gmin, float ns_per_tick, float *times,
                               hipStream_t s);
// Triangular forms (k_form.hip) ---------------------------------------------------
hipError_t launch_rev_entries(int32_t n, int32_t nnz, const int32_t *rp, const int32_t *ci, const double *va,
                              int32_t *orp, int32_t *oci, double *ova, hipStream_t s);
hipError_t launch_row_of_entry(int32_t n, const int32_t *rp, int32_t *row_of, hipStream_t s);
hipError_t launch_ptr_from_sorted(const int32_t *keys, int32_t nnz, int32_t n, int32_t *ptr, hipStream_t s);
hipError_t launch_take_entries(int32_t nnz, const int32_t *order, const int32_t *row_of, const double *va,
                               int32_t *oci, double *ova, hipStream_t s);
hipError_t launch_rev_io(int32_t n, const int32_t *perm, const int32_t *iperm, int32_t *perm_io, int32_t *iperm_io,
                         hipStream_t s);
ThinArgs thin_args(const Plan &P);
ThinArgs thin_args(const Plan &P, double *bp, double *xp);
sptrsv_status_t gather_b(sptrsv_ctx *h, Plan &P, int32_t nrhs, const double *b, int64_t ldb, double *bp,
                         hipStream_t s);
// The plan a solve entry point addresses after checking its arguments (null
// with *st set on failure).
Plan *solve_plan(sptrsv_ctx *h, int which, int32_t nrhs, const double *d_b, int64_t ldb, const double *d_x,
                 int64_t ldx, sptrsv_status_t *st);
// Whether the plan's runs and images are built for nrhs and the schedule in force.
bool runs_ready(const Plan &P, int32_t nrhs);
sptrsv_status_t solve_runs(sptrsv_ctx *h, Plan &P, int32_t nrhs, const double *b, int64_t ldb, double *x,
                           int64_t ldx, double *bp, double *xp, hipStream_t s);
sptrsv_status_t plan_solve(sptrsv_ctx *h, Plan &P, int32_t nrhs, const double *b, int64_t ldb, double *x,
                           int64_t ldx, hipStream_t s);
