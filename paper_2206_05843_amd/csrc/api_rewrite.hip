// sptrsv_rewrite: decision scan, row pointers, rewritten rows, re-levelling.
#include <algorithm>
#include <cstring>
#include <vector>

#include "common.h"

namespace {

constexpr int32_t kScanBigC = 1 << 20;  // entries of the scan's global workspace
constexpr int32_t kScanBigH = 1 << 21;

__global__ void k_fill_value(double *a, int64_t n, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

int32_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return (int32_t)p;
}

// The rewrite's self-check: b = L 1 solved with the original and with the
// rewritten system; a relative difference above tol, or a non-finite one,
// replaces the rewrite by the original system (L' = L, T = I, no row moved),
// so later rewritten solves give the original solve's result. A non-finite
// value the check itself produced is not left latched on the device.
sptrsv_status_t self_check(sptrsv_ctx *h, double tol, sptrsv_rewrite_stats_t &r, hipStream_t s) {
  const int32_t n = h->n;
  DArr<double> b, x0, x1;
  HIPCHK(h, b.alloc((size_t)n));
  HIPCHK(h, x0.alloc((size_t)n));
  HIPCHK(h, x1.alloc((size_t)n));
  int32_t bits_before = 0;
  HIPCHK(h, hipMemcpyAsync(&bits_before, h->d_err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, launch_row_sums(n, h->rp.p, h->va.p, b.p, s));
  STCHK(plan_solve(h, h->orig, 1, b.p, n, x0.p, n, s));
  STCHK(plan_solve(h, h->rew, 1, b.p, n, x1.p, n, s));
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(h->d_aux.p + 256);
  HIPCHK(h, hipMemsetAsync(acc, 0, 2 * sizeof(unsigned long long), s));
  HIPCHK(h, launch_max_abs_diff(n, x0.p, x1.p, acc, s));
  unsigned long long hv[2];
  HIPCHK(h, hipMemcpyAsync(hv, acc, sizeof(hv), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(h->d_err.p, &bits_before, sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIPCHK(h, hipStreamSynchronize(s));
  double d, m;
  std::memcpy(&d, &hv[0], sizeof(double));
  std::memcpy(&m, &hv[1], sizeof(double));
  const double err = m > 0.0 ? d / m : d;
  r.self_check_err = err;
  r.self_check_failed = 0;
  if (err <= tol) return SPTRSV_OK;
  // fall back to the original system
  const int64_t nnz = h->nnz;
  r.self_check_failed = 1;
  HIPCHK(h, h->lp_rp.alloc((size_t)n + 1));
  HIPCHK(h, h->lp_ci.alloc((size_t)nnz));
  HIPCHK(h, h->lp_va.alloc((size_t)nnz));
  HIPCHK(h, hipMemcpyAsync(h->lp_rp.p, h->rp.p, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->lp_ci.p, h->ci.p, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, hipMemcpyAsync(h->lp_va.p, h->va.p, sizeof(double) * (size_t)nnz, hipMemcpyDeviceToDevice, s));
  HIPCHK(h, h->t_rp.alloc((size_t)n + 1));
  HIPCHK(h, h->t_ci.alloc((size_t)n));
  HIPCHK(h, h->t_va.alloc((size_t)n));
  HIPCHK(h, launch_iota(h->t_rp.p, n + 1, s));
  HIPCHK(h, launch_iota(h->t_ci.p, n, s));
  hipLaunchKernelGGL(k_fill_value, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, h->t_va.p, (int64_t)n, 1.0);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemsetAsync(h->target.p, 0xff, sizeof(int32_t) * (size_t)n, s));
  STCHK(build_plan(h, h->rew, n, nnz, h->lp_rp.p, h->lp_ci.p, h->lp_va.p, h->t_rp.p, h->t_ci.p, h->t_va.p, s,
                   h->orig.rev_io));
  r.nlev_after = h->rew.nlev;
  r.rows_rewritten = 0;
  r.max_distance = 0;
  r.target_steps = 0;
  r.nnz_Lp = nnz;
  r.nnz_T = n;
  r.total_cost_after = h->rew.total_cost;
  r.avg_level_cost_after = h->rew.avg_cost;
  r.rows_skipped = 0;
  return SPTRSV_OK;
}

}  // namespace

extern "C" {

sptrsv_status_t sptrsv_rewrite(sptrsv_handle_t h, const sptrsv_rewrite_opts_t *o, hipStream_t s,
                               sptrsv_rewrite_stats_t *st) {
  if (!h || !o) return SPTRSV_ERR_ARG;
  h->last_error.clear();
  Plan &P = h->orig;
  if (!P.ready) return set_err(h, SPTRSV_ERR_STATE, "rewrite: matrix not analysed");
  if (o->thin_metric != SPTRSV_THIN_ROWS && o->thin_metric != SPTRSV_THIN_COST)
    return set_err(h, SPTRSV_ERR_ARG, "rewrite: thin_metric %d", o->thin_metric);
  if (o->max_distance < 0) return set_err(h, SPTRSV_ERR_ARG, "rewrite: max_distance %d", o->max_distance);
  if (!(o->thin_threshold == o->thin_threshold) || !(o->fill_cap == o->fill_cap))
    return set_err(h, SPTRSV_ERR_ARG, "rewrite: NaN option");
  if (o->scan_workers < 0 || o->scan_workers > SPTRSV_MAX_SCAN_WORKERS)
    return set_err(h, SPTRSV_ERR_ARG, "rewrite: scan_workers %d outside [0, %d]", o->scan_workers,
                   SPTRSV_MAX_SCAN_WORKERS);
  if (!(o->self_check >= 0.0)) return set_err(h, SPTRSV_ERR_ARG, "rewrite: self_check %g", o->self_check);
  if (o->max_indegree < 0 || o->max_spread < 0 || (o->critical_only != 0 && o->critical_only != 1))
    return set_err(h, SPTRSV_ERR_ARG, "rewrite: row constraints max_indegree %d max_spread %lld critical_only %d",
                   o->max_indegree, (long long)o->max_spread, o->critical_only);
  h->has_rewrite = false;
  h->rew.ready = false;
  const int32_t n = P.n, nlev = P.nlev;
  const double W = (o->thin_metric == SPTRSV_THIN_COST && o->thin_threshold <= 0.0) ? P.avg_cost : o->thin_threshold;
  DArr<int32_t> cur, cntL, cntT, small_rows, big_rows;
  DArr<long long> cl, ct, ex;
  HIPCHK(h, cur.alloc(n));
  HIPCHK(h, h->target.alloc(n));
  HIPCHK(h, cntL.alloc(n));
  HIPCHK(h, cntT.alloc(n));
  HIPCHK(h, cl.alloc(n));
  HIPCHK(h, ct.alloc(n));
  HIPCHK(h, ex.alloc(n));
  HIPCHK(h, h->lp_rp.alloc((size_t)n + 1));
  HIPCHK(h, h->t_rp.alloc((size_t)n + 1));
  if (n > 0) {
    HIPCHK(h, hipMemcpyAsync(cur.p, P.row_level.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    HIPCHK(h, hipMemsetAsync(h->target.p, 0xff, sizeof(int32_t) * (size_t)n, s));
  }
  // [16..19] scan outputs, [20] error bits, [21..23] collect counters, [32] rows held by a row constraint
  int32_t *aux = h->d_aux.p;
  HIPCHK(h, hipMemsetAsync(aux + 16, 0, 8 * sizeof(int32_t), s));
  HIPCHK(h, hipMemsetAsync(aux + 32, 0, sizeof(int32_t), s));
  int32_t hout[8] = {0}, held = 0;
  DArr<uint8_t> oncrit;
  if (n > 0 && nlev > 1 && o->critical_only) {
    HIPCHK(h, oncrit.alloc(n));
    STCHK(crit_rows(h, P, oncrit.p, s));
  }
  if (n > 0 && nlev > 1) {
    const int32_t workers = std::max(1, o->scan_workers);
    const size_t big_bytes = rewrite_big_ws_bytes(kScanBigC, kScanBigH) * (size_t)workers;
    if (h->rw_big.n < big_bytes) HIPCHK(h, h->rw_big.alloc(big_bytes));
    DArr<int32_t> seg;
    DArr<unsigned long long> claim;
    HIPCHK(h, seg.alloc((size_t)nlev + 1));
    HIPCHK(h, claim.alloc(1));
    // the largest per-level row budget bounds how many candidates a step evaluates at once
    double Wmax = W;
    if (o->d_level_budget) {
      std::vector<int32_t> hb((size_t)nlev);
      HIPCHK(h, hipMemcpyAsync(hb.data(), o->d_level_budget, sizeof(int32_t) * (size_t)nlev, hipMemcpyDeviceToHost,
                               s));
      HIPCHK(h, hipStreamSynchronize(s));
      for (int32_t v : hb) Wmax = std::max(Wmax, (double)v);
    }
    HIPCHK(h, launch_rewrite_scan(n, nlev, h->rp.p, h->ci.p, h->va.p, P.level_ptr.p, P.perm.p, P.lv_rows.p,
                                  P.lv_cost.p, o->d_level_mask, o->thin_metric, W, o->fill_cap, o->d_level_budget,
                                  o->d_level_fill_cap, Wmax, o->max_distance,
                                  o->max_indegree, o->max_spread, o->critical_only ? oncrit.p : nullptr, aux + 32,
                                  cur.p, h->target.p, cntL.p, cntT.p, workers, seg.p, claim.p, h->rw_big.p, kScanBigC,
                                  kScanBigH, aux + 16, s));
    HIPCHK(h, hipMemcpyAsync(hout, aux + 16, sizeof(hout), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(&held, aux + 32, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (hout[3]) return set_err(h, status_from_bits(hout[3]), "rewrite scan failed (bits 0x%x)", hout[3]);
  }
  // row pointers of L' and T
  int64_t nnz_lp = 0, nnz_t = 0;
  if (n > 0) {
    const size_t scr = scan_scratch_elems(n) + 16;
    if (h->scan_tmp.n < scr) HIPCHK(h, h->scan_tmp.alloc(scr));
    HIPCHK(h, launch_row_counts(n, h->rp.p, h->target.p, cntL.p, cntT.p, cl.p, ct.p, s));
    HIPCHK(h, launch_scan_i64(cl.p, ex.p, n, h->scan_tmp.p, s));
    HIPCHK(h, launch_ptr_from_scan(ex.p, cl.p, n, h->lp_rp.p, aux + 20, s));
    HIPCHK(h, launch_scan_i64(ct.p, ex.p, n, h->scan_tmp.p, s));
    HIPCHK(h, launch_ptr_from_scan(ex.p, ct.p, n, h->t_rp.p, aux + 20, s));
    long long last[4];
    HIPCHK(h, hipMemcpyAsync(&last[0], ex.p + (n - 1), sizeof(long long), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(&last[1], ct.p + (n - 1), sizeof(long long), hipMemcpyDeviceToHost, s));
    int32_t lp_end = 0, bits = 0;
    HIPCHK(h, hipMemcpyAsync(&lp_end, h->lp_rp.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipMemcpyAsync(&bits, aux + 20, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (bits) return set_err(h, status_from_bits(bits), "rewritten matrix exceeds int32 indexing");
    nnz_lp = lp_end;
    nnz_t = last[0] + last[1];
  } else {
    HIPCHK(h, hipMemsetAsync(h->lp_rp.p, 0, sizeof(int32_t), s));
    HIPCHK(h, hipMemsetAsync(h->t_rp.p, 0, sizeof(int32_t), s));
  }
  HIPCHK(h, h->lp_ci.alloc((size_t)std::max<int64_t>(nnz_lp, 1)));
  HIPCHK(h, h->lp_va.alloc((size_t)std::max<int64_t>(nnz_lp, 1)));
  HIPCHK(h, h->t_ci.alloc((size_t)std::max<int64_t>(nnz_t, 1)));
  HIPCHK(h, h->t_va.alloc((size_t)std::max<int64_t>(nnz_t, 1)));
  if (n > 0) {
    HIPCHK(h, launch_copy_unmoved(n, h->rp.p, h->ci.p, h->va.p, h->target.p, h->lp_rp.p, h->lp_ci.p, h->lp_va.p,
                                  h->t_rp.p, h->t_ci.p, h->t_va.p, s));
    const int32_t moved = hout[0];
    if (moved > 0) {
      HIPCHK(h, small_rows.alloc(moved));
      HIPCHK(h, big_rows.alloc(moved));
      HIPCHK(h, launch_collect_moved(n, h->target.p, cntL.p, cntT.p, small_rows.p, aux + 21, big_rows.p, aux + 22,
                                     aux + 23, s));
      int32_t cnts[3];
      HIPCHK(h, hipMemcpyAsync(cnts, aux + 21, sizeof(cnts), hipMemcpyDeviceToHost, s));
      HIPCHK(h, hipStreamSynchronize(s));
      HIPCHK(h, launch_rewrite_rows(cnts[0], small_rows.p, h->rp.p, h->ci.p, h->va.p, cur.p, h->target.p,
                                    h->lp_rp.p, h->lp_ci.p, h->lp_va.p, h->t_rp.p, h->t_ci.p, h->t_va.p, nullptr, 0,
                                    0, 0, aux + 20, s));
      if (cnts[1] > 0) {
        const int32_t C = next_pow2((int64_t)cnts[2] + 1), H = 2 * C;
        const int32_t waves = rewrite_waves_per_block();
        const int32_t blocks = std::max(1, std::min(16, (cnts[1] + waves - 1) / waves));
        DArr<char> big;
        HIPCHK(h, big.alloc(rewrite_big_ws_bytes(C, H) * (size_t)blocks * (size_t)waves));
        HIPCHK(h, launch_rewrite_rows(cnts[1], big_rows.p, h->rp.p, h->ci.p, h->va.p, cur.p, h->target.p,
                                      h->lp_rp.p, h->lp_ci.p, h->lp_va.p, h->t_rp.p, h->t_ci.p, h->t_va.p, big.p, C,
                                      H, blocks, aux + 20, s));
        HIPCHK(h, hipStreamSynchronize(s));
      }
      int32_t bits = 0;
      HIPCHK(h, hipMemcpyAsync(&bits, aux + 20, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIPCHK(h, hipStreamSynchronize(s));
      if (bits) return set_err(h, status_from_bits(bits), "rewriting rows failed (bits 0x%x)", bits);
    }
  }
  // re-level L' (empty levels disappear) and build its solve plan with T
  STCHK(build_plan(h, h->rew, n, nnz_lp, h->lp_rp.p, h->lp_ci.p, h->lp_va.p, h->t_rp.p, h->t_ci.p, h->t_va.p, s,
                   h->orig.rev_io));
  sptrsv_rewrite_stats_t r{};
  r.nlev_before = nlev;
  r.nlev_after = h->rew.nlev;
  r.rows_rewritten = hout[0];
  r.max_distance = hout[1];
  r.target_steps = hout[2];
  r.nnz_L = h->nnz;
  r.nnz_Lp = nnz_lp;
  r.nnz_T = nnz_t;
  r.total_cost_before = P.total_cost;
  r.total_cost_after = h->rew.total_cost;
  r.avg_level_cost_before = P.avg_cost;
  r.avg_level_cost_after = h->rew.avg_cost;
  r.rows_skipped = held;
  if (o->self_check > 0.0 && n > 0) STCHK(self_check(h, o->self_check, r, s));
  h->rstats = r;
  h->has_rewrite = true;
  if (st) *st = r;
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_get_rewritten(sptrsv_handle_t h, int32_t *d_Lp_row_ptr, int32_t *d_Lp_col, double *d_Lp_val,
                                     int32_t *d_T_row_ptr, int32_t *d_T_col, double *d_T_val, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  if (!h->has_rewrite) return set_err(h, SPTRSV_ERR_STATE, "no rewrite yet");
  const size_t n1 = (size_t)h->n + 1, a = (size_t)h->rstats.nnz_Lp, b = (size_t)h->rstats.nnz_T;
  const hipMemcpyKind k = hipMemcpyDeviceToDevice;
  if (d_Lp_row_ptr) HIPCHK(h, hipMemcpyAsync(d_Lp_row_ptr, h->lp_rp.p, sizeof(int32_t) * n1, k, s));
  if (d_Lp_col && a) HIPCHK(h, hipMemcpyAsync(d_Lp_col, h->lp_ci.p, sizeof(int32_t) * a, k, s));
  if (d_Lp_val && a) HIPCHK(h, hipMemcpyAsync(d_Lp_val, h->lp_va.p, sizeof(double) * a, k, s));
  if (d_T_row_ptr) HIPCHK(h, hipMemcpyAsync(d_T_row_ptr, h->t_rp.p, sizeof(int32_t) * n1, k, s));
  if (d_T_col && b) HIPCHK(h, hipMemcpyAsync(d_T_col, h->t_ci.p, sizeof(int32_t) * b, k, s));
  if (d_T_val && b) HIPCHK(h, hipMemcpyAsync(d_T_val, h->t_va.p, sizeof(double) * b, k, s));
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_get_targets(sptrsv_handle_t h, int32_t *d_target, hipStream_t s) {
  if (!h || !d_target) return SPTRSV_ERR_ARG;
  if (!h->has_rewrite) return set_err(h, SPTRSV_ERR_STATE, "no rewrite yet");
  if (h->n)
    HIPCHK(h, hipMemcpyAsync(d_target, h->target.p, sizeof(int32_t) * (size_t)h->n, hipMemcpyDeviceToDevice, s));
  return SPTRSV_OK;
}

}  // extern "C"
