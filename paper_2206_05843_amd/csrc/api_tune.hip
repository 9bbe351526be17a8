// Autotuner and hipGraph capture of solves.
#include <algorithm>
#include <cstring>

#include "common.h"

namespace {

__global__ void k_fill(double *a, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// Candidate schedules: all-wide, all-in-one-workgroup, and thin/wide splits at
// several widths, workgroup sizes and (one RHS) lanes per row. With several
// right-hand sides the thin runs start split one column per workgroup (their
// windows cut for one column); other splits are tried around the best.
std::vector<sptrsv_schedule_t> candidates(int32_t nrhs) {
  std::vector<sptrsv_schedule_t> c;
  const int thin_list[] = {64, 256, 1024, 4096, 16384};
  const int wg_list[] = {256, 512, 1024};
  const int lpr1[] = {1, 4};
  const int32_t tc = nrhs > 1 ? 1 : 0;  // thin_cols of the first round
  const int32_t gw = nrhs > 1 ? 1 : nrhs;
  for (int wg : wg_list) c.push_back(sptrsv_schedule_t{2, 0, wg, 256, 1, 0, 0, tc});
  for (int lpr : lpr1) {
    if (nrhs > 1 && lpr > 1) continue;
    c.push_back(sptrsv_schedule_t{1, 0, 512, 256, lpr, 0, 0, 0});
    for (int thr : thin_list) {
      if (thin_window_bytes(thr, 0, 1, gw) > thin_win_bytes()) continue;
      for (int wg : wg_list) c.push_back(sptrsv_schedule_t{0, thr, wg, 256, lpr, 0, 0, tc});
    }
  }
  // the synchronisation-free executor at a few grid sizes (workgroups in flight)
  for (int g : {128, 256, 512}) c.push_back(sptrsv_schedule_t{3, 0, 512, 256, 1, g});
  // dataflow runs of the wide levels (chunk sizes from the workgroup size), thin runs below
  for (int wt : {128, 256, 512})
    for (int thr : {0, 64, 1024}) {
      if (thin_window_bytes(thr, 0, 1, gw) > thin_win_bytes()) continue;
      c.push_back(sptrsv_schedule_t{4, thr, 1024, wt, 1, 0, 0, thr > 0 ? tc : 0});
    }
  // consecutive wide levels in one persistent launch (one lane per item; 4096
  // is capped to the workgroups that fit on the device at once)
  const int grids[] = {32, 256, 4096};
  for (int g : grids) {
    c.push_back(sptrsv_schedule_t{1, 0, 512, 256, 1, g});
    for (int thr : thin_list) {
      if (thin_window_bytes(thr, 0, 1, gw) > thin_win_bytes()) continue;
      c.push_back(sptrsv_schedule_t{0, thr, 1024, 256, 1, g, 0, tc});
    }
  }
  return c;
}

// rows: time solves with the right-hand sides stored by rows (solve_rows)
sptrsv_status_t autotune(sptrsv_ctx *h, int which, int32_t nrhs, bool rows, hipStream_t s, float *best_ms) {
  if (!h) return SPTRSV_ERR_ARG;
  Plan *P = sched_plan_of(h, which);
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  if (rows && which == SPTRSV_BATCH) return set_err(h, SPTRSV_ERR_ARG, "right-hand sides by rows: one matrix only");
  if (!P->ready) return set_err(h, SPTRSV_ERR_STATE, "matrix not analysed/rewritten");
  if (nrhs < 1) return set_err(h, SPTRSV_ERR_ARG, "nrhs=%d", nrhs);
  const int64_t n = P->n;
  if (n == 0) {
    if (best_ms) *best_ms = 0.f;
    return SPTRSV_OK;
  }
  DArr<double> b, x;
  HIPCHK(h, b.alloc((size_t)(n * nrhs)));
  HIPCHK(h, x.alloc((size_t)(n * nrhs)));
  hipLaunchKernelGGL(k_fill, dim3(1024), dim3(256), 0, s, b.p, n * nrhs, 1.0);
  HIPCHK(h, hipGetLastError());
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  const sptrsv_schedule_t keep = P->sched;
  float best = 1e30f;
  sptrsv_schedule_t best_s = keep;
  sptrsv_status_t st = SPTRSV_OK;
  // the batched matrices: workgroup size of the persistent launch
  const bool batch = which == SPTRSV_BATCH;
  std::vector<sptrsv_schedule_t> cands;
  if (batch) {
    for (int wg : {256, 512, 1024}) cands.push_back(sptrsv_schedule_t{2, 0, wg, 256, 1, 0});
  } else {
    cands = candidates(nrhs);
  }
  auto run = [&]() {
    if (batch) return sptrsv_batch_solve(h, nrhs, b.p, x.p, s);
    return rows ? sptrsv_solve_rows(h, which, nrhs, b.p, x.p, s) : plan_solve(h, *P, nrhs, b.p, n, x.p, n, s);
  };
  // a candidate whose device-side wait reaches its limit on this matrix is
  // dropped (its timeout bit cleared) and counted in the tuning report
  auto drop_timeout = [&]() -> bool {
    int32_t bits = 0;
    if (hipMemcpyAsync(&bits, h->d_err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess || !(bits & EB_TIMEOUT))
      return false;
    const int32_t rest = bits & ~EB_TIMEOUT;
    (void)hipMemcpyAsync(h->d_err.p, &rest, sizeof(int32_t), hipMemcpyHostToDevice, s);
    (void)hipStreamSynchronize(s);
    return true;
  };
  sptrsv_tune_info_t info{};
  // one candidate: a warm-up and the median of three timed solves; false
  // when it was dropped at its wait limit or a solve failed (st says which)
  auto time_cand = [&](const sptrsv_schedule_t &cand, float *ms) -> bool {
    P->sched = cand;
    P->runs_nrhs = -1;
    P->tuned.erase(nrhs);
    // launches that wait on the device get a limit tied to the best time so far
    const bool waits = !batch && (cand.mode == 3 || cand.mode == 4 || cand.wide_grid > 0);
    h->wait_ticks = 0;
    if (waits && best < 1e29f) {
      const double lim_ms = std::max(2.0, 8.0 * (double)best);
      h->wait_ticks = (unsigned long long)(lim_ms * 1e5);  // 100 MHz wall clock
      info.max_wait_limit_ms = std::max(info.max_wait_limit_ms, (float)lim_ms);
    }
    ++info.candidates;
    float t[3];
    st = run();  // warm-up
    if (st != SPTRSV_OK) return false;
    if (waits && drop_timeout()) {
      ++info.timed_out;
      return false;
    }
    for (int rep = 0; rep < 3 && st == SPTRSV_OK; ++rep) {
      (void)hipEventRecord(e0, s);
      st = run();
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      (void)hipEventElapsedTime(&t[rep], e0, e1);
    }
    if (st != SPTRSV_OK) return false;
    if (waits && drop_timeout()) {
      ++info.timed_out;
      return false;
    }
    std::sort(t, t + 3);
    *ms = t[1];
    return true;
  };
  for (const sptrsv_schedule_t &cand : cands) {
    float ms = 0.f;
    if (time_cand(cand, &ms) && ms < best) {
      best = ms;
      best_s = cand;
    }
    if (st != SPTRSV_OK) break;
  }
  // the workgroup size of the wide-level launches, around the best split
  // schedule (smaller workgroups spread a level over more CUs)
  if (st == SPTRSV_OK && !batch && best_s.mode == 0 && best < 1e29f) {
    const sptrsv_schedule_t base = best_s;
    for (int wt : {64, 128, 512}) {
      if (wt == base.wide_threads) continue;
      sptrsv_schedule_t cand = base;
      cand.wide_threads = wt;
      float ms = 0.f;
      if (time_cand(cand, &ms) && ms < best) {
        best = ms;
        best_s = cand;
      }
      if (st != SPTRSV_OK) break;
    }
  }
  // several right-hand sides: the other splits of the thin runs over
  // workgroups by columns (thin_cols 2, 4, ... and all columns in one
  // workgroup), around the best schedule with thin runs
  if (st == SPTRSV_OK && !batch && nrhs > 1 && best < 1e29f &&
      (best_s.mode == 2 || ((best_s.mode == 0 || best_s.mode == 4) && best_s.thin_rows > 0))) {
    const sptrsv_schedule_t base = best_s;
    std::vector<int32_t> splits;
    for (int32_t tc = 1; tc < nrhs; tc *= 2)
      if (nrhs % tc == 0) splits.push_back(tc);
    splits.push_back(0);  // all columns in one workgroup
    for (int32_t tc : splits) {
      if (tc == base.thin_cols) continue;
      sptrsv_schedule_t cand = base;
      cand.thin_cols = tc;
      float ms = 0.f;
      if (time_cand(cand, &ms) && ms < best) {
        best = ms;
        best_s = cand;
      }
      if (st != SPTRSV_OK) break;
    }
  }
  h->wait_ticks = 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->sched = keep;
  P->runs_nrhs = -1;
  if (st != SPTRSV_OK) return st;
  HIPCHK(h, hipStreamSynchronize(s));
  P->tuned[nrhs] = best_s;
  info.best_ms = best;
  h->tune_info = info;
  if (best_ms) *best_ms = best;
  return sptrsv_check(h, s);
}

}  // namespace

extern "C" {

sptrsv_status_t sptrsv_autotune(sptrsv_handle_t h, int which, int32_t nrhs, hipStream_t s, float *best_ms) {
  return autotune(h, which, nrhs, false, s, best_ms);
}

sptrsv_status_t sptrsv_autotune_rows(sptrsv_handle_t h, int which, int32_t nrhs, hipStream_t s, float *best_ms) {
  return autotune(h, which, nrhs, true, s, best_ms);
}

sptrsv_status_t sptrsv_get_tune_info(sptrsv_handle_t h, sptrsv_tune_info_t *out) {
  if (!h || !out) return SPTRSV_ERR_ARG;
  *out = h->tune_info;
  return SPTRSV_OK;
}

// One solve captured in a hipGraph: by columns (ldb, ldx) or, with rows, by rows.
static sptrsv_status_t graph_create(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, int64_t ldb,
                                    double *d_x, int64_t ldx, bool rows, hipStream_t s, int32_t *graph_id) {
  if (!h || !graph_id) return SPTRSV_ERR_ARG;
  if (!s) return set_err(h, SPTRSV_ERR_ARG, "graph capture needs a non-null stream");
  if (h->graphs.size() >= 16) return set_err(h, SPTRSV_ERR_ARG, "at most 16 graphs per handle");
  STCHK(sptrsv_prepare(h, which, nrhs, s));
  Graph g;
  const bool prof = h->prof;  // no event records inside a captured graph
  h->prof = false;
  HIPCHK(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  sptrsv_status_t st = rows ? sptrsv_solve_rows(h, which, nrhs, d_b, d_x, s)
                            : sptrsv_solve(h, which, nrhs, d_b, ldb, d_x, ldx, s);
  hipError_t e = hipStreamEndCapture(s, &g.g);
  h->prof = prof;
  if (st != SPTRSV_OK) {
    if (g.g) (void)hipGraphDestroy(g.g);
    return st;
  }
  if (e != hipSuccess) return set_err(h, SPTRSV_ERR_HIP, "capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&g.ge, g.g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g.g);
    return set_err(h, SPTRSV_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
  }
  h->graphs.push_back(g);
  *graph_id = (int32_t)h->graphs.size() - 1;
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_graph_create(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, int64_t ldb,
                                    double *d_x, int64_t ldx, hipStream_t s, int32_t *graph_id) {
  return graph_create(h, which, nrhs, d_b, ldb, d_x, ldx, false, s, graph_id);
}

sptrsv_status_t sptrsv_graph_create_rows(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, double *d_x,
                                         hipStream_t s, int32_t *graph_id) {
  return graph_create(h, which, nrhs, d_b, 0, d_x, 0, true, s, graph_id);
}

sptrsv_status_t sptrsv_graph_launch(sptrsv_handle_t h, int32_t graph_id, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  if (graph_id < 0 || graph_id >= (int32_t)h->graphs.size()) return set_err(h, SPTRSV_ERR_ARG, "graph id");
  HIPCHK(h, hipGraphLaunch(h->graphs[(size_t)graph_id].ge, s));
  return SPTRSV_OK;
}

}  // extern "C"
