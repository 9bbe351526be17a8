/*
 * sptrsv.h -- C ABI of libsptrsv.so: level-scheduled sparse lower-triangular
 * solves on MI355X (gfx950), with the equation-rewriting graph transformation of
 * "A Graph Transformation Strategy for Optimizing SpTRSV" (Yilmaz and Yildiz,
 * arXiv 2206.05843).
 *
 * Problem (Sec. II.A): given a sparse lower-triangular L in CSR and dense right-
 * hand sides b, find x with L x = b. Rows are grouped into levels (no row depends
 * on another row of its level) and levels are solved in order.
 * Transformation (Sec. II.B, Sec. III): rows of thin levels are rewritten by
 * substituting the equations of the rows they read, then rearranged back into
 * L'x = b' form, with b' = T b; the rewritten rows move to earlier levels and
 * the dependency graph becomes shorter and wider.
 *
 * Conventions for every call:
 *   - Indices are 0-based int32. A CSR matrix has n+1 row pointers starting at 0,
 *     column indices strictly ascending within a row, every column <= the row,
 *     and the diagonal stored LAST in its row (the layout Algorithm 1 reads).
 *   - Pointers named d_* are device pointers owned by the caller; h_* are host
 *     pointers owned by the caller. Inputs are only read during the call.
 *   - Dense right-hand sides and solutions are column-major: column c of b starts
 *     at d_b + c*ldb (ld >= n). b and x must not overlap.
 *   - hipStream_t may be NULL (the null stream). Calls marked ASYNC enqueue work
 *     on the stream and return; the rest return after the stream has completed.
 *   - Every call returns a status; nothing throws or aborts across this ABI. The
 *     handle keeps a message for the last failure (sptrsv_last_error).
 *   - A handle is used by one host thread at a time. All handle-owned device
 *     memory lives until sptrsv_destroy (or the next analyze, which replaces it).
 */
#ifndef SPTRSV_H
#define SPTRSV_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sptrsv_ctx *sptrsv_handle_t;

typedef enum {
  SPTRSV_OK = 0,
  SPTRSV_ERR_ARG = 1,          /* bad argument or malformed row pointers       */
  SPTRSV_ERR_STATE = 2,        /* call out of order (e.g. solve before analyze) */
  SPTRSV_ERR_NOT_LOWER = 3,    /* a column index outside [0, row]              */
  SPTRSV_ERR_UNSORTED = 4,     /* columns not strictly ascending in a row      */
  SPTRSV_ERR_MISSING_DIAG = 5, /* empty row or last column != row              */
  SPTRSV_ERR_ZERO_PIVOT = 6,   /* diagonal value 0                             */
  SPTRSV_ERR_NONFINITE = 7,    /* NaN/Inf in values, or a non-finite solution  */
  SPTRSV_ERR_OVERFLOW = 8,     /* a rewritten size exceeds int32 / a capacity  */
  SPTRSV_ERR_ALLOC = 9,        /* device allocation failed                     */
  SPTRSV_ERR_HIP = 10,         /* a HIP runtime call failed                    */
  SPTRSV_ERR_TIMEOUT = 11      /* a bounded device-side wait expired           */
} sptrsv_status_t;

/* Which plan: the analysed matrix, its rewrite, or (schedule and autotuner
 * only) the batched matrices of sptrsv_batch_analyze, whose persistent launch
 * uses the wg_threads knob (256, 512 or 1024). */
enum { SPTRSV_ORIGINAL = 0, SPTRSV_REWRITTEN = 1, SPTRSV_BATCH = 2 };
enum { SPTRSV_THIN_ROWS = 0, SPTRSV_THIN_COST = 1 };
/* Triangular forms a handle can solve (sptrsv_analyze_form). */
enum { SPTRSV_LOWER = 0, SPTRSV_UPPER = 1, SPTRSV_LOWER_TRANS = 2, SPTRSV_UPPER_TRANS = 3 };

/* Handle lifetime. create: makes a handle bound to the current HIP device.
 * destroy: frees every handle-owned buffer (NULL is accepted). */
sptrsv_status_t sptrsv_create(sptrsv_handle_t *h);
sptrsv_status_t sptrsv_destroy(sptrsv_handle_t h);
/* Message of the handle's last failure ("" if none). Valid until the next call. */
const char *sptrsv_last_error(sptrsv_handle_t h);
/* Name of a status code, e.g. "SPTRSV_ERR_ZERO_PIVOT". */
const char *sptrsv_status_name(sptrsv_status_t s);

/* ---------------------------------------------------------------------------
 * sptrsv_analyze -- validate L and build its level sets (Sec. II.A).
 * The level of a row is the length of the longest dependency path that ends at
 * it (0 for a row with no off-diagonal); the rows of a level are independent.
 * Also builds the handle-owned level-ordered copy of L the solve streams.
 *   n, nnz        : dimensions (nnz = d_row_ptr[n]); n >= 0
 *   d_row_ptr     : int32[n+1], d_col: int32[nnz], d_val: double[nnz] (device)
 *   nlevels_out   : host pointer, receives the number of levels
 * Errors: ARG/NOT_LOWER/UNSORTED/MISSING_DIAG/ZERO_PIVOT/NONFINITE for malformed
 * input (first in that priority order), TIMEOUT, ALLOC, HIP. The caller's arrays
 * may be freed after the call returns (the handle keeps a copy). Synchronous.
 * Replaces any previous analysis and rewrite held by the handle.
 * ------------------------------------------------------------------------- */
sptrsv_status_t sptrsv_analyze(sptrsv_handle_t h, int32_t n, int32_t nnz, const int32_t *d_row_ptr,
                               const int32_t *d_col, const double *d_val, hipStream_t s,
                               int32_t *nlevels_out);

/* ---------------------------------------------------------------------------
 * sptrsv_analyze_form -- sptrsv_analyze for the other triangular systems a
 * preconditioner application needs (the solve of Sec. II.A run the other way):
 *   SPTRSV_LOWER        L x = b, the CSR is lower-triangular (= sptrsv_analyze)
 *   SPTRSV_UPPER        U x = b, the CSR is upper-triangular with the diagonal
 *                       first in each row and columns ascending
 *   SPTRSV_LOWER_TRANS  L^T x = b, the CSR is lower-triangular (as above)
 *   SPTRSV_UPPER_TRANS  U^T x = b, the CSR is upper-triangular (as above)
 * The handle keeps the system in lower-triangular form: L; J U J and J L^T J
 * (J reverses the order of rows and columns); U^T. Levels, statistics, the
 * rewrite (Sec. II.B, Sec. III: for U and L^T it runs in reverse row order)
 * and the getters refer to that form and its row numbering; sptrsv_solve and
 * sptrsv_residual take b and return x in the caller's numbering of the
 * original system. Arguments and errors as sptrsv_analyze (the input is
 * checked in its own triangular form; an entry on the wrong side of the
 * diagonal is NOT_LOWER), plus ARG for an unknown form. Synchronous. Replaces
 * any previous analysis and rewrite held by the handle.
 * ------------------------------------------------------------------------- */
sptrsv_status_t sptrsv_analyze_form(sptrsv_handle_t h, int32_t form, int32_t n, int32_t nnz, const int32_t *d_row_ptr,
                                    const int32_t *d_col, const double *d_val, hipStream_t s, int32_t *nlevels_out);

/* Copy the level sets of the ORIGINAL matrix or of the REWRITTEN matrix L'
 * into caller buffers (device): level_ptr int32[nlev+1], level_rows int32[n]
 * (rows of each level in ascending order), row_level int32[n]. Any pointer may
 * be NULL to skip it. ERR_STATE if that matrix has not been analysed. ASYNC. */
sptrsv_status_t sptrsv_get_levels(sptrsv_handle_t h, int which, int32_t *d_level_ptr, int32_t *d_level_rows,
                                  int32_t *d_row_level, hipStream_t s);

/* Per-level statistics of the cost model (Sec. III): rows, sum of nnz (diagonal
 * included) and cost = 2*sum(nnz) - rows of every level, as int64[nlev] device
 * arrays, plus (host) the total cost and avgLevelCost = total / nlev.
 * Any pointer may be NULL. Synchronous. */
sptrsv_status_t sptrsv_level_stats(sptrsv_handle_t h, int which, int64_t *d_rows, int64_t *d_nnz, int64_t *d_cost,
                                   int64_t *h_total_cost, double *h_avg_level_cost, hipStream_t s);

/* ---------------------------------------------------------------------------
 * sptrsv_rewrite -- the naive strategy of Sec. III applied on the device.
 * Sources are the thin levels (THIN_COST: level cost < thin_threshold, or
 * < avgLevelCost when thin_threshold <= 0; THIN_ROWS: fewer than thin_threshold
 * rows), or the levels a mask marks. Level 0 starts as the target; a non-source
 * level becomes the target; the rows of each source level, in ascending order,
 * are rewritten toward the current target while it stays within budget
 * (THIN_COST: target cost, each row costing 2*nnz'-1, <= the threshold;
 * THIN_ROWS: target rows <= thin_threshold), optionally while nnz(L'[r]) <=
 * fill_cap * nnz(L[r]) and the distance is <= max_distance. The first refusal
 * makes its level the next target with every row of it not moved (rows already
 * moved stay moved).
 * Row constraints (the refinements Sec. III.A lists): a row that passes the
 * tests above is left in place, and the run goes on, when its rewritten form
 * has max_indegree or more off-diagonals (indegree < alpha), when its
 * off-diagonal columns span max_spread or more (distance between dependencies
 * < beta, the locality limit), or, with critical_only, when it is not on a
 * longest path of the original DAG (level + longest path to a row nothing
 * depends on = nlev - 1). Zero disables each.
 * A row is rewritten by substituting, largest column first, every unknown whose
 * row currently sits at or below the target level (Sec. II.B, Fig. 2) and
 * rearranging (Sec. II.B): L'[r] keeps its diagonal; T[r] collects the b terms
 * with a unit diagonal; explicit zeros from cancellation stay in the pattern.
 * L' is then re-levelled (empty levels vanish) and prepared for solving.
 * The scan splits into segments, each starting at level 0 or at a non-source
 * level and running to the next: a segment's decisions depend on nothing
 * outside it (its rows move only within it, and every row of an earlier
 * segment stays below its first level), so scan_workers workgroups can take
 * segments at once, from the beginning and from the end of the level order
 * (the parallel sketch of Sec. III: empty levels are removed only at the end,
 * so level numbers stay valid while both scans run). Each worker holds a
 * ~34 MB global workspace.
 * ------------------------------------------------------------------------- */
#define SPTRSV_MAX_SCAN_WORKERS 16
typedef struct {
  int32_t thin_metric;          /* SPTRSV_THIN_ROWS or SPTRSV_THIN_COST                         */
  double thin_threshold;        /* ROWS: W (e.g. 32). COST: <= 0 means avgLevelCost              */
  double fill_cap;              /* accept iff nnz(L'[r]) <= fill_cap * nnz(L[r]); <= 0 disables  */
  int32_t max_distance;         /* 0 = unlimited                                                 */
  const uint8_t *d_level_mask;  /* optional device uint8[nlev]: 1 = source; NULL = thin test     */
  int32_t max_indegree;         /* alpha: 0 = no limit                                           */
  int32_t critical_only;        /* 1: only rows on a longest path are rewritten                  */
  int64_t max_spread;           /* beta, in columns: 0 = no limit                                */
  int32_t scan_workers;         /* workgroups running the scan at once, 0..SPTRSV_MAX_SCAN_WORKERS:
                                   0 or 1 = one, from level 0 on; 2 = from both ends of the level
                                   order at once; more = half from each end. Same result for all. */
  const int32_t *d_level_budget; /* optional device int32[nlev]: for the rows of source level l, a
                                   positive entry replaces thin_threshold as the row budget of the
                                   target (THIN_ROWS only): the learned policy's per-level action  */
  const float *d_level_fill_cap; /* optional device float[nlev]: a positive entry replaces fill_cap
                                   for the rows of source level l                                */
  double self_check;            /* > 0: after rewriting, solve L x = L 1 with the original and the
                                   rewritten system; if their solutions differ by more than this
                                   (relative, max norm) or are not finite, the rewrite is replaced by
                                   the original system (L' = L, T = I) and the stats say so (the
                                   precision risk of long substitution chains, Sec. III.A). 0 = off */
} sptrsv_rewrite_opts_t;

typedef struct {
  int32_t nlev_before, nlev_after, rows_rewritten, max_distance, target_steps;
  int64_t nnz_L, nnz_Lp, nnz_T, total_cost_before, total_cost_after;
  double avg_level_cost_before, avg_level_cost_after; /* Table I metrics (Sec. IV) */
  int32_t rows_skipped;         /* rows a row constraint left in place                           */
  int32_t self_check_failed;    /* 1: the self-check failed and the original system is in use    */
  double self_check_err;        /* the self-check's relative difference (0 when it did not run)  */
} sptrsv_rewrite_stats_t;

/* Errors: STATE (no analysis), ARG (bad opts), OVERFLOW (rewritten sizes beyond
 * int32 or the device work capacity), TIMEOUT, ALLOC, HIP. st may be NULL.
 * Synchronous. Replaces any previous rewrite held by the handle. */
sptrsv_status_t sptrsv_rewrite(sptrsv_handle_t h, const sptrsv_rewrite_opts_t *o, hipStream_t s,
                               sptrsv_rewrite_stats_t *st);

/* Copy L' and T (CSR over the ORIGINAL row numbering, both lower-triangular,
 * diagonal last) into caller device buffers sized from the stats: row_ptr
 * int32[n+1], col int32[nnz], val double[nnz]. Any pointer may be NULL. ASYNC.
 * Also the per-row targets: int32[n], -1 for rows that were not rewritten. */
sptrsv_status_t sptrsv_get_rewritten(sptrsv_handle_t h, int32_t *d_Lp_row_ptr, int32_t *d_Lp_col, double *d_Lp_val,
                                     int32_t *d_T_row_ptr, int32_t *d_T_col, double *d_T_val, hipStream_t s);
sptrsv_status_t sptrsv_get_targets(sptrsv_handle_t h, int32_t *d_target, hipStream_t s);

/* ---------------------------------------------------------------------------
 * sptrsv_solve -- x = L^{-1} b for nrhs >= 1 columns (Sec. II.A, Algorithm 1,
 * level by level). which = ORIGINAL solves L; which = REWRITTEN computes
 * b' = T b on the fly and solves L' x = b', which gives the same x.
 *   d_b : double, column-major n x nrhs, ld ldb >= n;  d_x : same for x.
 * ASYNC and capture-safe (no allocation, no host synchronisation) once a solve
 * of the same (which, nrhs) has run or sptrsv_prepare has been called.
 * A non-finite solution entry latches SPTRSV_ERR_NONFINITE on the device,
 * reported by sptrsv_check. Errors: STATE, ARG (nrhs < 1, ld < n, overlap).
 * ------------------------------------------------------------------------- */
sptrsv_status_t sptrsv_solve(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, int64_t ldb,
                             double *d_x, int64_t ldx, hipStream_t s);

/* sptrsv_solve_noalloc -- sptrsv_solve for callers that cannot allocate device
 * memory: code under hipGraph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments, kernels and result (bit for bit) as
 * sptrsv_solve; its two work vectors (n * nrhs doubles each) live in a static
 * 64 MiB device array that every GPU the library runs on holds until the
 * process ends, so n * nrhs must be at most 4,194,304 (else ERR_ARG).
 * It calls no allocating routine: the schedule for (which, nrhs) must already
 * be built (sptrsv_prepare, or an earlier sptrsv_solve with the same nrhs and
 * schedule), else ERR_STATE. The work area is shared by every call on the same
 * GPU (all handles): calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller. Nothing in it needs to
 * start at any value. ASYNC; errors as sptrsv_solve. */
sptrsv_status_t sptrsv_solve_noalloc(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, int64_t ldb,
                                     double *d_x, int64_t ldx, hipStream_t s);

/* sptrsv_solve_rows -- sptrsv_solve with the right-hand sides stored by rows:
 * d_b, d_x: n x nrhs, entry (i, c) at i * nrhs + c (the layout of one row's
 * right-hand sides together that the solve kernels work in), no leading
 * dimension. Same x as sptrsv_solve bit for bit (the same kernels and order).
 * With thin runs, wide launches and persistent wide runs (modes 0, 1, 2) the
 * solve kernels read b and write x through the level order themselves, with
 * no transposes, and d_x serves as the solve's work vector: a dependency's
 * value is read from it through the caller's row (so d_x must not be read or
 * written by anything else while the solve runs); the b-transform writes only
 * the rows of T with off-diagonals into the handle's work vector. The
 * synchronisation-free and dataflow executors (modes 3, 4) copy b in and x out
 * by rows. The first solve by rows of a plan maps its columns to caller rows
 * (about 4 bytes per nonzero and 17 per row of device memory, kept with the
 * plan). nrhs = 1 is sptrsv_solve with ld = n. ASYNC and capture-safe once a
 * solve of the same (which, nrhs) has run or sptrsv_prepare has been called.
 * Errors as sptrsv_solve (ARG: nrhs < 1, b and x overlapping). */
sptrsv_status_t sptrsv_solve_rows(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, double *d_x,
                                  hipStream_t s);

/* Allocate the work vectors for (which, nrhs) so later solves allocate nothing. */
sptrsv_status_t sptrsv_prepare(sptrsv_handle_t h, int which, int32_t nrhs, hipStream_t s);

/* Synchronise s and report (then clear) the errors latched on the device. */
sptrsv_status_t sptrsv_check(sptrsv_handle_t h, hipStream_t s);

/* Schedule knobs of the solve (see the autotuner): a level with at most
 * thin_rows rows runs inside one workgroup of wg_threads threads, together with
 * its thin neighbours; wider levels get one multi-workgroup launch each with
 * wide_threads threads per workgroup. mode: 0 = split at thin_rows,
 * 1 = every level as a wide launch, 2 = every level inside one workgroup,
 * 3 = no level barriers at all: one synchronisation-free launch in which each
 * (row, right-hand side) waits only for the values it reads (the comparison
 * executor; wide_grid gives its workgroups of 256 threads, 0 = 512, at most
 * 2048; the other knobs are ignored),
 * 4 = levels with at most thin_rows rows in thin runs as in mode 0, and each
 * run of consecutive wider levels as one dataflow launch: every level is cut
 * into chunks of 2 * wide_threads items (wide_threads = 128, 256 or 512) and
 * a chunk waits only for the chunks of the run holding the rows it reads, not
 * for whole levels (wide_grid: workgroups in flight, 0 = as many as fit).
 * overlap = 1: when the work vectors are large (n * nrhs >= 2^22) and the
 * chain has at least four runs, the transposes between the caller's b, x and
 * the work vectors run in 64-row tile groups on a handle-owned side stream
 * beside the level chain (up to 16 segments, at most two ahead of it); 0 (the
 * default, and what the autotuner keeps): before and after the chain. On the
 * 3D stencil with 32 right-hand sides the side stream's memory traffic slowed
 * the chain by more than it hid, in graph replays.
 * set_schedule replaces the schedules sptrsv_autotune picked for this matrix;
 * get_schedule reports the schedule a solve with nrhs right-hand sides uses
 * (the tuned one for that nrhs if there is one, else the one set). */
typedef struct {
  int32_t mode;
  int32_t thin_rows;
  int32_t wg_threads;     /* 256, 512 or 1024 */
  int32_t wide_threads;   /* 64 .. 1024, multiple of 64 */
  int32_t lanes_per_row;  /* wide levels, nrhs == 1: 1, 2, 4, 8, 16 or 32 lanes per row */
  int32_t wide_grid;      /* 0: one launch per wide level; > 0: consecutive wide levels in one persistent launch
                             of up to wide_grid workgroups (capped to what is resident at once) with a
                             device-wide barrier between levels, each workgroup fetching the next level's
                             indices, weights and b between its arrival and its wait (lanes_per_row is
                             then 1) */
  int32_t overlap;        /* 0 or 1: transposes beside the chain (see above) */
  int32_t thin_cols;      /* right-hand sides per thin-run workgroup: 0 = all; c, a divisor of nrhs smaller than
                             it = nrhs / c workgroups each solve c columns of every thin run (columns are
                             independent), with LDS windows cut for c columns; otherwise all. The batched
                             launch (SPTRSV_BATCH) solves every column of a matrix in one workgroup */
} sptrsv_schedule_t;
sptrsv_status_t sptrsv_set_schedule(sptrsv_handle_t h, int which, const sptrsv_schedule_t *sched);
sptrsv_status_t sptrsv_get_schedule(sptrsv_handle_t h, int which, int32_t nrhs, sptrsv_schedule_t *sched);

/* Autotuner: times candidate schedules with HIP events on s (inputs b = 1) and
 * keeps the fastest for (which, nrhs), then tries the wide launches of a best
 * split schedule (mode 0) with 64, 128 and 512 threads per workgroup, and,
 * with several right-hand sides, the other splits of the best schedule's thin
 * runs over workgroups by columns (the candidates split them one column per
 * workgroup; then thin_cols 2, 4, ... dividing nrhs, and all columns); for
 * SPTRSV_BATCH the candidates are the
 * workgroup sizes of the persistent launch. best_ms (host, may be NULL) receives the
 * best solve time. Synchronous.
 * Candidates whose launches wait on the device (the synchronisation-free
 * executor, persistent wide runs) run with a wait limit of 8x the best time so
 * far (at least 2 ms) instead of the solve's 10 s: a candidate that reaches it
 * is dropped, and counted in sptrsv_get_tune_info. */
sptrsv_status_t sptrsv_autotune(sptrsv_handle_t h, int which, int32_t nrhs, hipStream_t s, float *best_ms);
/* The same, timing solves with the right-hand sides stored by rows
 * (sptrsv_solve_rows), where thin-run and per-level wide schedules skip the
 * copies the other executors keep. The pick is stored for (which, nrhs) as
 * sptrsv_autotune's is: the layout tuned last sets the schedule both layouts
 * use. which = SPTRSV_BATCH is an ARG error. */
sptrsv_status_t sptrsv_autotune_rows(sptrsv_handle_t h, int which, int32_t nrhs, hipStream_t s, float *best_ms);

/* What the handle's last sptrsv_autotune call did: candidates timed,
 * candidates dropped because a device-side wait reached its limit, the best
 * time, and the largest wait limit given to a candidate (ms). */
typedef struct {
  int32_t candidates;
  int32_t timed_out;
  float best_ms;
  float max_wait_limit_ms;
} sptrsv_tune_info_t;
sptrsv_status_t sptrsv_get_tune_info(sptrsv_handle_t h, sptrsv_tune_info_t *out);

/* hipGraph capture of one solve with fixed buffers; replays are ASYNC. The graph
 * belongs to the handle (at most 16); graph_id receives its index. */
sptrsv_status_t sptrsv_graph_create(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, int64_t ldb,
                                    double *d_x, int64_t ldx, hipStream_t s, int32_t *graph_id);
/* The same for sptrsv_solve_rows. */
sptrsv_status_t sptrsv_graph_create_rows(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, double *d_x,
                                         hipStream_t s, int32_t *graph_id);
sptrsv_status_t sptrsv_graph_launch(sptrsv_handle_t h, int32_t graph_id, hipStream_t s);

/* Live kernel profile of solves: enable = 1 clears the counters and starts
 * bracketing every solve launch on its stream with HIP events (at most 65536
 * launches are recorded); enable = 0 stops, synchronises s and fills out[4]
 * for the launch classes {gather b, thin runs, wide levels, scatter x}: number
 * of launches, summed device time (ms), and algorithmic bytes (index, value,
 * diagonal and right-hand-side bytes the launches must move at least once). */
typedef struct {
  int64_t launches;
  double ms;
  double bytes;
} sptrsv_kernel_profile_t;
sptrsv_status_t sptrsv_profile(sptrsv_handle_t h, int enable, sptrsv_kernel_profile_t *out, hipStream_t s);

/* Level floor: what one level costs when it holds no work, for each way a
 * solve separates consecutive levels (Sec. II.A: levels run in order, so a
 * solve costs at least the sum of these over its levels). Measured on the
 * device with the solve kernels' own synchronisation (ns per level):
 *   thin_level_ns       a level of a thin-run window spread over several waves:
 *                       an LDS-only workgroup barrier and one dependent LDS read
 *   thin_wave_level_ns  the same in a window run by one wave (no barrier)
 *   launch_ns           a kernel launch per level on a stream
 *   graph_node_ns       a kernel node per level of a replayed hipGraph
 *   grid_barrier_ns     a device-wide barrier of a persistent launch
 *   flag_hop_ns         a value handed from one workgroup to the next through
 *                       a device-coherent store and load (the least a
 *                       dependency costs the synchronisation-free executor)
 * Synchronous; allocates a few bytes of device memory. */
typedef struct {
  double thin_level_ns;
  double thin_wave_level_ns;
  double launch_ns;
  double graph_node_ns;
  double grid_barrier_ns;
  double flag_hop_ns;
} sptrsv_level_costs_t;
sptrsv_status_t sptrsv_measure_level_costs(sptrsv_handle_t h, hipStream_t s, sptrsv_level_costs_t *out);
/* The level floor of one solve of (which, nrhs) under the schedule it uses
 * (built if needed): the costs above summed over the plan's levels as its
 * runs separate them (thin-run levels by window kind, one launch or graph node
 * per wide level and per launch of a run, device-wide barriers inside
 * persistent runs, one hop per level for the synchronisation-free executor),
 * plus the launches of the gather, b-transform and scatter. flags:
 * SPTRSV_FLOOR_GRAPH prices launches as graph nodes; SPTRSV_FLOOR_ROWS prices a
 * solve with the right-hand sides by rows (sptrsv_solve_rows), which has no
 * gather or scatter launch under modes 0, 1 and 2; other
 * bits are an ARG error. floor_us receives microseconds. Synchronous. */
#define SPTRSV_FLOOR_GRAPH 1
#define SPTRSV_FLOOR_ROWS 2
sptrsv_status_t sptrsv_level_floor(sptrsv_handle_t h, int which, int32_t nrhs, int32_t flags,
                                   const sptrsv_level_costs_t *c, double *floor_us);

/* Residual check: h_out[c] = max_i |(L x - b)[i,c]| for the ORIGINAL L, host
 * double[nrhs]. Synchronous. */
sptrsv_status_t sptrsv_residual(sptrsv_handle_t h, int32_t nrhs, const double *d_b, int64_t ldb, const double *d_x,
                                int64_t ldx, double *h_out, hipStream_t s);

/* ---------------------------------------------------------------------------
 * Batched solves: many independent matrices, concatenated. Matrix i has n_i =
 * h_n[i] rows starting at global row h_row_off[i] and nonzeros starting at
 * h_nnz_off[i] of the concatenated arrays; its row pointers (d_row_ptr_cat
 * segment of n_i+1 entries at h_row_off[i] + i) are LOCAL (start at 0) and its
 * column indices local. Each matrix is level-scheduled as in sptrsv_analyze.
 * batch_solve solves all matrices in one persistent launch; matrix i's b and x
 * are n_i x nrhs column-major at offset nrhs*h_row_off[i], ld = n_i. ASYNC.
 * A matrix with a level too wide for one workgroup's LDS window at this nrhs
 * (about 1,000 rows at 16 right-hand sides) is taken out of the persistent
 * launch and solved level by level (thin runs, one device-wide launch per
 * wide level) in the same call, with the same result.
 * ------------------------------------------------------------------------- */
sptrsv_status_t sptrsv_batch_analyze(sptrsv_handle_t h, int32_t nmat, const int32_t *h_n, const int64_t *h_row_off,
                                     const int64_t *h_nnz_off, const int32_t *d_row_ptr_cat, const int32_t *d_col_cat,
                                     const double *d_val_cat, hipStream_t s);
sptrsv_status_t sptrsv_batch_solve(sptrsv_handle_t h, int32_t nrhs, const double *d_b_cat, double *d_x_cat,
                                   hipStream_t s);
/* The per-matrix solve the batched launch replaces: one plain solve per matrix,
 * looped on the stream (ASYNC). */
sptrsv_status_t sptrsv_batch_solve_looped(sptrsv_handle_t h, int32_t nrhs, const double *d_b_cat, double *d_x_cat,
                                          hipStream_t s);
/* Levels of batched matrix i (ERR_ARG if out of range). Synchronous. */
sptrsv_status_t sptrsv_batch_levels(sptrsv_handle_t h, int32_t i, int32_t *nlev, int32_t *d_level_ptr,
                                    int32_t *d_level_rows, hipStream_t s);

/* ---------------------------------------------------------------------------
 * Plan files: rewriting is a preprocessing step whose result later solves use
 * (Sec. II.B, Sec. III), so a handle's analysis and rewrite can be kept in a
 * file and loaded into another handle (or process) that then solves without
 * analysing, rewriting or tuning again.
 * plan_save writes the matrix in its lower-triangular form, the level sets and
 * level-ordered copy of L, the rewritten L', T, targets and statistics (if a
 * rewrite was made) with their level sets, and the schedules in force and
 * tuned per nrhs, to the host file `path` (created or truncated). Synchronous
 * (waits for the device). Errors: STATE (nothing analysed), ARG (the file
 * cannot be written), HIP.
 * plan_load replaces the handle's analysis and rewrite by the file's (it
 * destroys the handle's graphs, which captured the old buffers). Solves after
 * it give the same x, bit for bit, as solves with the handle that saved it.
 * The file is checked before the handle changes: a file that is not a plan,
 * of another version, truncated or altered (an FNV-1a-64 hash over its bytes
 * is stored at its end) returns ERR_ARG and leaves the handle as it was; a
 * file that passes the checks but fails while loading leaves it unanalysed.
 * Window images and work vectors are rebuilt by the first solve or
 * sptrsv_prepare. Synchronous. */
sptrsv_status_t sptrsv_plan_save(sptrsv_handle_t h, const char *path);
sptrsv_status_t sptrsv_plan_load(sptrsv_handle_t h, const char *path);

/* What a handle holds (after analyze, rewrite or plan_load): its triangular
 * form, n, nnz and number of levels of the analysed matrix, whether a rewrite
 * is held, and (st, may be NULL) that rewrite's statistics. ERR_STATE if
 * nothing is analysed. */
typedef struct {
  int32_t form, n, nlev, has_rewrite;
  int64_t nnz;
} sptrsv_info_t;
sptrsv_status_t sptrsv_get_info(sptrsv_handle_t h, sptrsv_info_t *out, sptrsv_rewrite_stats_t *st);

/* ---------------------------------------------------------------------------
 * Learned rewrite policy (not in the paper; replaces the thin-level test of
 * Sec. III with a small network). Parameters are float32[SPTRSV_MLP_NPARAM]:
 * W1[64,20] b1[64] W2[64,64] b2[64] W3[64] b3[1], row-major.
 * ------------------------------------------------------------------------- */
#define SPTRSV_MLP_NIN 20
#define SPTRSV_MLP_HID 64
#define SPTRSV_MLP_NPARAM 5569

/* 20 float features per level of the ORIGINAL matrix (layout float[nlev][20]):
 * log1p(rows), log1p(sum nnz), log1p(cost), cost/avgLevelCost, rows/32,
 * sum nnz/rows, fractions of rows with 0,1,2,3-4,5-8,>=9 off-diagonals,
 * sum nnz(L'[r])/sum nnz(L[r]) and log1p(sum nnz(T[r])) if the level alone were
 * rewritten into the level before it, level/nlev, log1p(rows of previous level),
 * then the row constraints of Sec. III.A on that same move: the fraction of
 * rows left with fewer than 4 off-diagonals (indegree < alpha), the fraction on
 * a longest path of the DAG (level + height = nlev - 1), log1p of the mean
 * column span (largest minus smallest off-diagonal column) and the fraction of
 * rows spanning fewer than 1024 columns (spread < beta). Level 0 counts its rows
 * as they are. Synchronous (host reads of overflow counts). */
sptrsv_status_t sptrsv_level_features(sptrsv_handle_t h, float *d_feat, hipStream_t s);
/* p[i] = sigmoid(MLP(f[i])) for the batch rows, f = (feat - mean) * inv_std
 * when d_norm (float[40]: mean[20], inv_std[20]) is given, else f = feat.
 * d_feat float[batch][20], d_prob float[batch]. ASYNC. */
sptrsv_status_t sptrsv_mlp_forward(const float *d_params, const float *d_feat, const float *d_norm, int32_t batch,
                                   float *d_prob, hipStream_t s);
/* Gradient of the mean binary cross-entropy, (1/batch) sum_i w_i BCE(p_i, y_i),
 * w.r.t. every parameter (d_grad float[NPARAM], overwritten) and that loss
 * (d_loss float[1]); d_label float[batch] in {0,1}; d_weight (optional,
 * float[batch], default 1); d_norm as in forward. The batch reduction has a
 * fixed order (deterministic). ASYNC. */
sptrsv_status_t sptrsv_mlp_backward(const float *d_params, const float *d_feat, const float *d_norm,
                                    const float *d_label, const float *d_weight, int32_t batch, float *d_grad,
                                    float *d_loss, hipStream_t s);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step >= 1). ASYNC. */
sptrsv_status_t sptrsv_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step, float lr,
                                hipStream_t s);
/* Measured per-level device time of one solve of the ORIGINAL or REWRITTEN
 * matrix with every level run inside one workgroup where it fits (levels too
 * wide for one workgroup report 0): ns per level into d_times float[nlev], from
 * the device wall clock; the bulk phase of an LDS window is shared among its
 * levels in proportion to their rows. b as in sptrsv_solve (nrhs columns, ld =
 * n); the solution is discarded. Synchronous. These times label levels when the
 * policy is trained (the change in solve time a rewrite causes). */
sptrsv_status_t sptrsv_level_times(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, float *d_times,
                                   hipStream_t s);
/* mask[l] = (p[l] >= threshold) for l >= 1, mask[0] = 0: the rewrite mask of
 * the learned policy from probabilities (ASYNC). */
sptrsv_status_t sptrsv_mlp_mask(const float *d_prob, int32_t nlev, float threshold, uint8_t *d_mask, hipStream_t s);
/* Per-level finish times under the synchronisation-free executor (the
 * schedule the autotuner picks on power-law matrices; with its tuned grid when
 * the handle holds a tuned mode-3 schedule for this nrhs): one solve in which
 * every item records the device wall clock when its value is written, then
 * d_times[l] (device, nlev floats) = latest stamp of level l - earliest stamp
 * of the solve, in ns. A level's share of the solve is the growth of the
 * running maximum of these times across it. b as in sptrsv_solve (ld = n); the
 * solution is discarded. Allocates 8 n nrhs bytes for the stamps.
 * Synchronous. These times label levels when the policy is trained on the
 * executor it will run under (Sec. III.A: a rewrite pays only where it shortens
 * the solve). */
sptrsv_status_t sptrsv_level_finish_times(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b,
                                          float *d_times, hipStream_t s);

/* Tiered actions of the learned policy (Sec. III.A: which rows to rewrite, and
 * how far). Tier j (0 <= j < ntiers <= SPTRSV_MAX_TIERS) has a probability
 * threshold (host array, ascending), a target budget in rows and a fill cap
 * (host arrays; 0 = the rewrite's own value). A level l >= 1 takes the highest
 * tier whose threshold p[l] reaches: d_mask[l] = 1, d_budget[l], d_cap[l] =
 * that tier's; otherwise, and at level 0, d_mask[l] = 0 and d_budget[l] =
 * d_cap[l] = 0. The three device arrays (nlev entries each) go to
 * sptrsv_rewrite as mask, d_level_budget and d_level_fill_cap. ERR_ARG for
 * thresholds out of order or NaN, a negative budget or cap, or ntiers out of
 * range. ASYNC. */
#define SPTRSV_MAX_TIERS 4
sptrsv_status_t sptrsv_mlp_actions(const float *d_prob, int32_t nlev, int32_t ntiers, const float *thresholds,
                                   const int32_t *budgets, const float *caps, uint8_t *d_mask, int32_t *d_budget,
                                   float *d_cap, hipStream_t s);

#ifdef __cplusplus
}
#endif
#endif /* SPTRSV_H */
