// Learned policy entry points: level features, network kernels, level times.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace {

// Backward scratch (per-wave partial gradients), grown on demand, per process.
DArr<float> g_part, g_part_loss;

}  // namespace

extern "C" {

sptrsv_status_t sptrsv_level_features(sptrsv_handle_t h, float *d_feat, hipStream_t s) {
  if (!h || !d_feat) return SPTRSV_ERR_ARG;
  Plan &P = h->orig;
  if (!P.ready) return set_err(h, SPTRSV_ERR_STATE, "features: matrix not analysed");
  const int32_t n = P.n, nlev = P.nlev;
  if (nlev == 0) return SPTRSV_OK;
  DArr<long long> sums;  // sum_lp, sum_t, sum_span
  DArr<int32_t> hist, redo;
  DArr<uint8_t> oncrit;
  HIPCHK(h, sums.alloc((size_t)nlev * 3));
  HIPCHK(h, hist.alloc((size_t)nlev * kFeatHist));
  HIPCHK(h, redo.alloc(n));
  HIPCHK(h, oncrit.alloc(n));
  HIPCHK(h, hipMemsetAsync(sums.p, 0, sizeof(long long) * (size_t)nlev * 3, s));
  HIPCHK(h, hipMemsetAsync(hist.p, 0, sizeof(int32_t) * (size_t)nlev * kFeatHist, s));
  STCHK(crit_rows(h, P, oncrit.p, s));
  const FeatAcc acc{sums.p, sums.p + nlev, sums.p + 2 * (size_t)nlev, hist.p, oncrit.p};
  int32_t *aux = h->d_aux.p;  // [24] redo count, [25] error bits
  HIPCHK(h, hipMemsetAsync(aux + 24, 0, 2 * sizeof(int32_t), s));
  HIPCHK(h, launch_feat_rows(n, nullptr, 0, h->rp.p, h->ci.p, h->va.p, P.row_level.p, acc, redo.p, aux + 24, nullptr,
                             0, 0, 0, aux + 25, s));
  int32_t hc[2];
  HIPCHK(h, hipMemcpyAsync(hc, aux + 24, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (hc[0] > 0) {  // rows whose distance-1 rewrite outgrows LDS
    // the largest such row has at most (nnz of the row and of everything it reads) entries
    const int32_t C = 1 << 16, H = 1 << 17;
    const int32_t blocks = std::max(1, std::min(8, (hc[0] + rewrite_waves_per_block() - 1) / rewrite_waves_per_block()));
    DArr<char> big;
    HIPCHK(h, big.alloc(rewrite_big_ws_bytes(C, H) * (size_t)blocks * (size_t)rewrite_waves_per_block()));
    HIPCHK(h, launch_feat_rows(n, redo.p, hc[0], h->rp.p, h->ci.p, h->va.p, P.row_level.p, acc, redo.p, aux + 24,
                               big.p, C, H, blocks, aux + 25, s));
    HIPCHK(h, hipMemcpyAsync(hc, aux + 24, sizeof(hc), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
  }
  if (hc[1]) return set_err(h, status_from_bits(hc[1]), "features: rewrite workspace overflow");
  HIPCHK(h, launch_feat_finalize(nlev, P.lv_rows.p, P.lv_nnz.p, P.lv_cost.p, P.avg_cost, acc, d_feat, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_mlp_forward(const float *d_params, const float *d_feat, const float *d_norm, int32_t batch,
                                   float *d_prob, hipStream_t s) {
  if (!d_params || (batch > 0 && (!d_feat || !d_prob)) || batch < 0) return SPTRSV_ERR_ARG;
  return launch_mlp_forward(d_params, d_feat, d_norm, batch, d_prob, s) == hipSuccess ? SPTRSV_OK : SPTRSV_ERR_HIP;
}

sptrsv_status_t sptrsv_mlp_backward(const float *d_params, const float *d_feat, const float *d_norm,
                                    const float *d_label, const float *d_weight, int32_t batch, float *d_grad,
                                    float *d_loss, hipStream_t s) {
  if (!d_params || !d_grad || !d_loss || batch < 1 || !d_feat || !d_label) return SPTRSV_ERR_ARG;
  const size_t parts = (size_t)mlp_backward_parts();
  if (g_part.n < parts * SPTRSV_MLP_NPARAM) {
    if (g_part.alloc(parts * SPTRSV_MLP_NPARAM) != hipSuccess) return SPTRSV_ERR_ALLOC;
    if (g_part_loss.alloc(parts) != hipSuccess) return SPTRSV_ERR_ALLOC;
  }
  return launch_mlp_backward(d_params, d_feat, d_norm, d_label, d_weight, batch, g_part.p, g_part_loss.p, d_grad,
                             d_loss, s) == hipSuccess
             ? SPTRSV_OK
             : SPTRSV_ERR_HIP;
}

sptrsv_status_t sptrsv_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int32_t step, float lr,
                                hipStream_t s) {
  if (!d_params || !d_grad || !d_m || !d_v || step < 1) return SPTRSV_ERR_ARG;
  const float c1 = 1.0f - std::pow(0.9f, (float)step), c2 = 1.0f - std::pow(0.999f, (float)step);
  return launch_mlp_adam(d_params, d_grad, d_m, d_v, lr, c1, c2, s) == hipSuccess ? SPTRSV_OK : SPTRSV_ERR_HIP;
}

sptrsv_status_t sptrsv_mlp_mask(const float *d_prob, int32_t nlev, float threshold, uint8_t *d_mask,
                                hipStream_t s) {
  if (nlev < 0 || (nlev > 0 && (!d_prob || !d_mask))) return SPTRSV_ERR_ARG;
  return launch_mlp_mask(d_prob, nlev, threshold, d_mask, s) == hipSuccess ? SPTRSV_OK : SPTRSV_ERR_HIP;
}

sptrsv_status_t sptrsv_mlp_actions(const float *d_prob, int32_t nlev, int32_t ntiers, const float *thresholds,
                                   const int32_t *budgets, const float *caps, uint8_t *d_mask, int32_t *d_budget,
                                   float *d_cap, hipStream_t s) {
  if (nlev < 0 || ntiers < 1 || ntiers > SPTRSV_MAX_TIERS || !thresholds || !budgets || !caps)
    return SPTRSV_ERR_ARG;
  if (nlev > 0 && (!d_prob || !d_mask || !d_budget || !d_cap)) return SPTRSV_ERR_ARG;
  MlpTiers t{};
  t.n = ntiers;
  for (int j = 0; j < ntiers; ++j) {
    if (!(thresholds[j] == thresholds[j]) || budgets[j] < 0 || !(caps[j] >= 0.0f)) return SPTRSV_ERR_ARG;
    if (j > 0 && !(thresholds[j] >= thresholds[j - 1])) return SPTRSV_ERR_ARG;
    t.thr[j] = thresholds[j];
    t.budget[j] = budgets[j];
    t.cap[j] = caps[j];
  }
  return launch_mlp_actions(d_prob, nlev, t, d_mask, d_budget, d_cap, s) == hipSuccess ? SPTRSV_OK : SPTRSV_ERR_HIP;
}

sptrsv_status_t sptrsv_level_finish_times(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b,
                                          float *d_times, hipStream_t s) {
  if (!h || !d_b || !d_times || nrhs < 1) return SPTRSV_ERR_ARG;
  Plan *P = which == SPTRSV_ORIGINAL ? &h->orig : which == SPTRSV_REWRITTEN ? &h->rew : nullptr;
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  if (!P->ready) return set_err(h, SPTRSV_ERR_STATE, "matrix not analysed/rewritten");
  if (P->n == 0) return SPTRSV_OK;
  int rate_khz = 100000;
  (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, h->dev);
  const float ns_per_tick = 1.0e6f / (float)(rate_khz > 0 ? rate_khz : 100000);
  STCHK(ensure_work(h, *P, nrhs));
  const auto tk = P->tuned.find(nrhs);
  const int32_t blocks = tk != P->tuned.end() && tk->second.mode == 3 ? tk->second.wide_grid : 0;
  DArr<unsigned long long> stamp, lmax;
  HIPCHK(h, stamp.alloc((size_t)P->n * (size_t)nrhs));
  HIPCHK(h, lmax.alloc((size_t)P->nlev + 1));
  HIPCHK(h, hipMemsetAsync(lmax.p + P->nlev, 0xff, sizeof(unsigned long long), s));
  STCHK(gather_b(h, *P, nrhs, d_b, P->n, P->bp.p, s));
  HIPCHK(h, launch_syncfree(P->n, nrhs, P->srp.p, P->sci.p, P->sva.p, P->sdg.p, P->bp.p, P->xp.p, P->sf_ticket.p,
                            h->d_err.p, blocks, wait_limit(h), s, stamp.p));
  HIPCHK(h, launch_stamp_levels(P->nlev, nrhs, P->level_ptr.p, stamp.p, lmax.p, lmax.p + P->nlev, ns_per_tick,
                                d_times, s));
  HIPCHK(h, hipStreamSynchronize(s));
  return sptrsv_check(h, s);
}

sptrsv_status_t sptrsv_level_times(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, float *d_times,
                                   hipStream_t s) {
  if (!h || !d_b || !d_times || nrhs < 1) return SPTRSV_ERR_ARG;
  Plan *P = which == SPTRSV_ORIGINAL ? &h->orig : which == SPTRSV_REWRITTEN ? &h->rew : nullptr;
  if (!P) return set_err(h, SPTRSV_ERR_ARG, "which=%d", which);
  if (!P->ready) return set_err(h, SPTRSV_ERR_STATE, "matrix not analysed/rewritten");
  if (P->n == 0) return SPTRSV_OK;
  int rate_khz = 100000;
  (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, h->dev);
  const float ns_per_tick = 1.0e6f / (float)(rate_khz > 0 ? rate_khz : 100000);
  STCHK(ensure_work(h, *P, nrhs));
  sptrsv_schedule_t sc{2, 0, 512, 256, 1};  // every level that fits runs in one workgroup
  STCHK(make_runs(h, *P, nrhs, sc, s));
  HIPCHK(h, hipMemsetAsync(d_times, 0, sizeof(float) * (size_t)P->nlev, s));
  STCHK(gather_b(h, *P, nrhs, d_b, P->n, P->bp.p, s));
  for (const Run &r : P->runs) {
    if (r.thin) {
      HIPCHK(h, launch_thin_run(512, P->win.p + r.wi, r.nw, nrhs, thin_args(*P), h->d_err.p, s, d_times, ns_per_tick));
    } else {
      HIPCHK(h, launch_wide_level(256, 1, P->h_level_ptr[r.l0], P->h_level_ptr[r.l1], nrhs, P->srp.p, P->sci.p,
                                  P->sva.p, P->sdg.p, P->ell_c.p, P->ell_v.p, P->bp.p, P->xp.p, h->d_err.p, s));
    }
  }
  HIPCHK(h, hipStreamSynchronize(s));
  P->runs_nrhs = -1;  // the next solve rebuilds its own schedule
  return sptrsv_check(h, s);
}

}  // extern "C"
