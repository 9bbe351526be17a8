// Batched solves: many independent matrices analysed as one block-diagonal
// system (levels per matrix), solved in one persistent launch.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "common.h"

namespace {

__global__ void k_fill_mat_of_row(const int64_t *__restrict__ row_off, int32_t nmat, int32_t *mat_of_row) {
  for (int32_t m = blockIdx.x; m < nmat; m += gridDim.x)
    for (int64_t r = row_off[m] + threadIdx.x; r < row_off[m + 1]; r += blockDim.x) mat_of_row[r] = m;
}

// Global row pointers of the block-diagonal union (local pointers of matrix m
// occupy n_m + 1 entries at row_off[m] + m of the concatenated array).
__global__ void k_global_rp(int64_t total, const int32_t *__restrict__ mat_of_row, const int64_t *__restrict__ row_off,
                            const int64_t *__restrict__ nnz_off, const int32_t *__restrict__ rp_cat, int32_t *grp,
                            int64_t total_nnz) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= total; r += (int64_t)gridDim.x * blockDim.x) {
    if (r == total) {
      grp[r] = (int32_t)total_nnz;
      continue;
    }
    const int32_t m = mat_of_row[r];
    grp[r] = (int32_t)(nnz_off[m] + rp_cat[row_off[m] + m + (r - row_off[m])]);
  }
}

// Entries of row r shifted to global column numbers.
__global__ void k_global_entries(int64_t total, const int32_t *__restrict__ mat_of_row,
                                 const int64_t *__restrict__ row_off, const int32_t *__restrict__ grp,
                                 const int32_t *__restrict__ ci_cat, const double *__restrict__ va_cat, int32_t *gci,
                                 double *gva) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < total; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t off = (int32_t)row_off[mat_of_row[r]];
    for (int32_t q = grp[r]; q < grp[r + 1]; ++q) {
      gci[q] = ci_cat[q] + off;
      gva[q] = va_cat[q];
    }
  }
}

__global__ void k_mat_max(int64_t total, const int32_t *__restrict__ mat_of_row, const int32_t *__restrict__ lev1,
                          int32_t *mx) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < total; r += (int64_t)gridDim.x * blockDim.x)
    atomicMax(mx + mat_of_row[r], lev1[r]);
}

__global__ void k_combined_keys(int64_t total, const int32_t *__restrict__ mat_of_row, const int32_t *__restrict__ lvl_off,
                                const int32_t *__restrict__ lev1, int32_t *keys) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < total; r += (int64_t)gridDim.x * blockDim.x)
    keys[r] = lvl_off[mat_of_row[r]] + lev1[r];
}

__global__ void k_offset_copy(const int32_t *__restrict__ src, int32_t n, int32_t off, int32_t *dst) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i] - off;
}

int bit_width64(int64_t v) {
  int b = 0;
  while (v > 0) ++b, v >>= 1;
  return b;
}

// Per-matrix LDS windows for nrhs (cached). A matrix whose levels all fit an
// LDS window goes in the persistent queue; a matrix with a level too wide for
// one is solved level by level instead (its narrow levels in thin runs, its
// wide ones one device-wide launch each, as a single plan's mode-0 schedule).
sptrsv_status_t batch_windows(sptrsv_ctx *h, int32_t nrhs, int32_t wg, hipStream_t s) {
  if (h->b_win_nrhs == nrhs && h->b_win_wg == wg) return SPTRSV_OK;
  Plan &P = h->bat;
  P.h_win.clear();
  h->b_h_mwin.assign((size_t)h->b_nmat + 1, 0);
  h->b_wide.clear();
  std::vector<char> fits((size_t)h->b_nmat, 1);
  for (int32_t m = 0; m < h->b_nmat; ++m) {
    const int32_t l0 = (int32_t)h->b_lvl_off[(size_t)m], l1 = (int32_t)h->b_lvl_off[(size_t)m + 1];
    for (int32_t l = l0; l < l1 && fits[(size_t)m]; ++l)
      if (!level_fits_window(P, l, nrhs)) fits[(size_t)m] = 0;
    h->b_h_mwin[(size_t)m] = (int32_t)P.h_win.size();
    if (fits[(size_t)m]) cut_windows(P, l0, l1, nrhs, wg, P.h_win);
  }
  h->b_h_mwin[(size_t)h->b_nmat] = (int32_t)P.h_win.size();
  for (int32_t m = 0; m < h->b_nmat; ++m) {
    if (fits[(size_t)m]) continue;
    BatchWide bw;
    bw.m = m;
    const int32_t l0 = (int32_t)h->b_lvl_off[(size_t)m], l1 = (int32_t)h->b_lvl_off[(size_t)m + 1];
    for (int32_t l = l0; l < l1; ++l) {
      const bool thin = level_fits_window(P, l, nrhs);
      if (!bw.runs.empty() && thin && bw.runs.back().thin && bw.runs.back().l1 == l)
        bw.runs.back().l1 = l + 1;
      else
        bw.runs.push_back(Run{l, l + 1, thin});
    }
    for (Run &r : bw.runs)
      if (r.thin) {
        r.wi = (int32_t)P.h_win.size();
        r.nw = cut_windows(P, r.l0, r.l1, nrhs, wg, P.h_win);
      }
    h->b_wide.push_back(std::move(bw));
  }
  // the persistent queue: the matrices that fit, in the analysis' order
  std::vector<int32_t> q;
  for (int32_t m : h->b_h_order)
    if (fits[(size_t)m]) q.push_back(m);
  h->b_nq = (int32_t)q.size();
  HIPCHK(h, h->b_order.reserve(std::max<size_t>(q.size(), 1)));
  if (!q.empty()) HIPCHK(h, hipMemcpy(h->b_order.p, q.data(), sizeof(int32_t) * q.size(), hipMemcpyHostToDevice));
  h->b_win_nrhs = -1;  // until the images are built
  STCHK(build_images(h, P, s));
  HIPCHK(h, h->b_mwin.alloc((size_t)h->b_nmat + 1));
  HIPCHK(h, hipMemcpy(h->b_mwin.p, h->b_h_mwin.data(), sizeof(int32_t) * ((size_t)h->b_nmat + 1),
                      hipMemcpyHostToDevice));
  h->b_win_nrhs = nrhs;
  h->b_win_wg = wg;
  return SPTRSV_OK;
}

// The matrices taken out of the persistent launch, level by level.
sptrsv_status_t batch_wide_solves(sptrsv_ctx *h, int32_t nrhs, int32_t wg, hipStream_t s) {
  Plan &P = h->bat;
  const sptrsv_schedule_t d = default_schedule();
  for (const BatchWide &bw : h->b_wide)
    for (const Run &r : bw.runs) {
      if (r.thin)
        HIPCHK(h, launch_thin_run(wg, P.win.p + r.wi, r.nw, nrhs, thin_args(P), h->d_err.p, s));
      else
        HIPCHK(h, launch_wide_level(d.wide_threads, 1, P.h_level_ptr[(size_t)r.l0], P.h_level_ptr[(size_t)r.l1], nrhs,
                                    P.srp.p, P.sci.p, P.sva.p, P.sdg.p, P.ell_c.p, P.ell_v.p, P.bp.p, P.xp.p,
                                    h->d_err.p, s));
    }
  return SPTRSV_OK;
}

}  // namespace

extern "C" {

sptrsv_status_t sptrsv_batch_analyze(sptrsv_handle_t h, int32_t nmat, const int32_t *h_n, const int64_t *h_row_off,
                                     const int64_t *h_nnz_off, const int32_t *d_row_ptr_cat, const int32_t *d_col_cat,
                                     const double *d_val_cat, hipStream_t s) {
  if (!h || nmat < 1 || !h_n || !h_row_off || !h_nnz_off || !d_row_ptr_cat || !d_col_cat || !d_val_cat)
    return SPTRSV_ERR_ARG;
  h->last_error.clear();
  h->b_ready = false;
  h->b_win_nrhs = -1;
  // host bookkeeping: offsets must describe back-to-back matrices
  std::vector<int64_t> row_off((size_t)nmat + 1), nnz_off((size_t)nmat + 1);
  int64_t acc = 0;
  for (int32_t m = 0; m < nmat; ++m) {
    if (h_n[m] < 1 || h_row_off[m] != acc) return set_err(h, SPTRSV_ERR_ARG, "batch: bad size/offset of matrix %d", m);
    row_off[(size_t)m] = acc;
    acc += h_n[m];
  }
  row_off[(size_t)nmat] = acc;
  const int64_t total = acc;
  if (total >= (int64_t)1 << 31) return set_err(h, SPTRSV_ERR_OVERFLOW, "batch: too many rows");
  for (int32_t m = 0; m < nmat; ++m) nnz_off[(size_t)m] = h_nnz_off[m];
  int32_t last_nnz = 0;
  HIPCHK(h, hipMemcpyAsync(&last_nnz, d_row_ptr_cat + (row_off[(size_t)nmat - 1] + nmat - 1 + h_n[nmat - 1]),
                           sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  const int64_t total_nnz = nnz_off[(size_t)nmat - 1] + last_nnz;
  nnz_off[(size_t)nmat] = total_nnz;
  for (int32_t m = 0; m < nmat; ++m)
    if (nnz_off[(size_t)m] < 0 || nnz_off[(size_t)m + 1] < nnz_off[(size_t)m])
      return set_err(h, SPTRSV_ERR_ARG, "batch: bad nonzero offset of matrix %d", m);
  if (total_nnz >= (int64_t)1 << 31) return set_err(h, SPTRSV_ERR_OVERFLOW, "batch: too many nonzeros");
  h->b_nmat = nmat;
  h->b_n.assign(h_n, h_n + nmat);
  h->b_row_off = row_off;
  DArr<int64_t> d_nnz_off;
  HIPCHK(h, h->b_row_off_d.alloc((size_t)nmat + 1));
  HIPCHK(h, d_nnz_off.alloc((size_t)nmat + 1));
  HIPCHK(h, hipMemcpy(h->b_row_off_d.p, row_off.data(), sizeof(int64_t) * ((size_t)nmat + 1), hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(d_nnz_off.p, nnz_off.data(), sizeof(int64_t) * ((size_t)nmat + 1), hipMemcpyHostToDevice));
  // block-diagonal union in global numbering
  HIPCHK(h, h->b_mat_of_row.alloc((size_t)total));
  HIPCHK(h, h->b_rp.alloc((size_t)total + 1));
  HIPCHK(h, h->b_ci.alloc((size_t)total_nnz));
  HIPCHK(h, h->b_va.alloc((size_t)total_nnz));
  hipLaunchKernelGGL(k_fill_mat_of_row, dim3(std::min(nmat, 4096)), dim3(256), 0, s, h->b_row_off_d.p, nmat,
                     h->b_mat_of_row.p);
  hipLaunchKernelGGL(k_global_rp, dim3(grid_for(total + 1, 256, 8192)), dim3(256), 0, s, total, h->b_mat_of_row.p,
                     h->b_row_off_d.p, d_nnz_off.p, d_row_ptr_cat, h->b_rp.p, total_nnz);
  HIPCHK(h, hipGetLastError());
  int32_t *aux = h->d_aux.p;
  HIPCHK(h, hipMemsetAsync(aux + 1, 0, sizeof(int32_t), s));
  // each matrix's local pointers must be well formed before entries are read
  HIPCHK(h, launch_validate((int32_t)total, (int32_t)total_nnz, h->b_rp.p, d_col_cat, d_val_cat, aux + 1, s));
  int32_t bits = 0;
  HIPCHK(h, hipMemcpyAsync(&bits, aux + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (bits & (EB_ARG | EB_NOT_LOWER))  // malformed pointers, or a negative local column
    return set_err(h, status_from_bits(bits & (EB_ARG | EB_NOT_LOWER)), "batch: malformed matrix (bits 0x%x)", bits);
  hipLaunchKernelGGL(k_global_entries, dim3(grid_for(total, 256, 8192)), dim3(256), 0, s, total, h->b_mat_of_row.p,
                     h->b_row_off_d.p, h->b_rp.p, d_col_cat, d_val_cat, h->b_ci.p, h->b_va.p);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipMemsetAsync(aux + 1, 0, sizeof(int32_t), s));
  HIPCHK(h, launch_validate((int32_t)total, (int32_t)total_nnz, h->b_rp.p, h->b_ci.p, h->b_va.p, aux + 1, s));
  HIPCHK(h, hipMemcpyAsync(&bits, aux + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (bits) return set_err(h, status_from_bits(bits), "batch: invalid matrix (bits 0x%x)", bits);
  // levels of every row (longest path; matrices are independent)
  const int32_t n = (int32_t)total;
  Plan &P = h->bat;
  P = Plan{};
  P.sched = default_schedule();
  P.n = n;
  P.nnz = total_nnz;
  DArr<int32_t> lev1, keys, ktmp, vtmp, hist, mx, lvl_off_d;
  DArr<long long> cnt, ex, hist64;
  HIPCHK(h, lev1.alloc(n));
  HIPCHK(h, keys.alloc(n));
  HIPCHK(h, ktmp.alloc(n));
  HIPCHK(h, vtmp.alloc(n));
  HIPCHK(h, cnt.alloc(n));
  HIPCHK(h, ex.alloc(n));
  HIPCHK(h, mx.alloc(nmat));
  HIPCHK(h, lvl_off_d.alloc(nmat));
  const size_t hn = radix_hist_elems(n);
  HIPCHK(h, hist.alloc(hn));
  HIPCHK(h, hist64.alloc(hn));
  const size_t scr = std::max(scan_scratch_elems((int64_t)hn), scan_scratch_elems(n)) + 16;
  if (h->scan_tmp.n < scr) HIPCHK(h, h->scan_tmp.alloc(scr));
  HIPCHK(h, hipMemsetAsync(aux, 0, 8 * sizeof(int32_t), s));
  HIPCHK(h, hipMemsetAsync(lev1.p, 0, sizeof(int32_t) * (size_t)n, s));
  HIPCHK(h, hipMemsetAsync(mx.p, 0, sizeof(int32_t) * (size_t)nmat, s));
  HIPCHK(h, launch_levels(n, h->b_rp.p, h->b_ci.p, lev1.p, reinterpret_cast<unsigned *>(aux), aux + 1, s));
  hipLaunchKernelGGL(k_mat_max, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, (int64_t)n, h->b_mat_of_row.p, lev1.p,
                     mx.p);
  HIPCHK(h, hipGetLastError());
  h->b_nlev.assign((size_t)nmat, 0);
  HIPCHK(h, hipMemcpyAsync(h->b_nlev.data(), mx.p, sizeof(int32_t) * (size_t)nmat, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(&bits, aux + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (bits) return set_err(h, status_from_bits(bits), "batch: level construction failed (bits 0x%x)", bits);
  h->b_lvl_off.assign((size_t)nmat + 1, 0);
  std::vector<int32_t> lvl_off32((size_t)nmat);
  for (int32_t m = 0; m < nmat; ++m) {
    lvl_off32[(size_t)m] = (int32_t)h->b_lvl_off[(size_t)m];
    h->b_lvl_off[(size_t)m + 1] = h->b_lvl_off[(size_t)m] + h->b_nlev[(size_t)m];
  }
  const int32_t nlev = (int32_t)h->b_lvl_off[(size_t)nmat];
  P.nlev = nlev;
  HIPCHK(h, hipMemcpy(lvl_off_d.p, lvl_off32.data(), sizeof(int32_t) * (size_t)nmat, hipMemcpyHostToDevice));
  // positions grouped by matrix, then level, rows ascending (stable sort)
  hipLaunchKernelGGL(k_combined_keys, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, (int64_t)n, h->b_mat_of_row.p,
                     lvl_off_d.p, lev1.p, keys.p);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, P.level_ptr.alloc((size_t)nlev + 1));
  HIPCHK(h, P.perm.alloc(n));
  HIPCHK(h, P.iperm.alloc(n));
  HIPCHK(h, P.row_level.alloc(n));
  HIPCHK(h, launch_iota(P.perm.p, n, s));
  HIPCHK(h, launch_radix_by_key(keys.p, P.perm.p, ktmp.p, vtmp.p, n, bit_width64(nlev), hist.p, hist64.p,
                                h->scan_tmp.p, s));
  HIPCHK(h, launch_level_ptr_from_sorted(keys.p, n, P.level_ptr.p, nlev, s));
  HIPCHK(h, launch_invert_perm(P.perm.p, n, P.iperm.p, s));
  HIPCHK(h, launch_sub1(lev1.p, n, P.row_level.p, s));
  // level-ordered copy, overflow prefix, statistics
  HIPCHK(h, P.srp.alloc((size_t)n + 1));
  HIPCHK(h, launch_count_off(P.perm.p, h->b_rp.p, n, cnt.p, s));
  HIPCHK(h, launch_scan_i64(cnt.p, ex.p, n, h->scan_tmp.p, s));
  HIPCHK(h, launch_ptr_from_scan(ex.p, cnt.p, n, P.srp.p, aux + 1, s));
  const int64_t noff = total_nnz - n;
  HIPCHK(h, P.sci.alloc((size_t)std::max<int64_t>(noff, 1)));
  HIPCHK(h, P.sva.alloc((size_t)std::max<int64_t>(noff, 1)));
  HIPCHK(h, P.sdg.alloc(n));
  HIPCHK(h, launch_fill_solve(n, P.perm.p, P.iperm.p, h->b_rp.p, h->b_ci.p, h->b_va.p, P.srp.p, P.sci.p, P.sva.p,
                              P.sdg.p, s));
  HIPCHK(h, P.ell_c.alloc(n));
  HIPCHK(h, P.ell_v.alloc((size_t)2 * n));
  HIPCHK(h, launch_fill_ell(n, P.srp.p, P.sci.p, P.sva.p, P.ell_c.p, P.ell_v.p, s));
  HIPCHK(h, P.lv_rows.alloc(nlev));
  HIPCHK(h, P.lv_nnz.alloc(nlev));
  HIPCHK(h, P.lv_cost.alloc(nlev));
  HIPCHK(h, launch_level_stats(nlev, P.level_ptr.p, P.srp.p, P.lv_rows.p, P.lv_nnz.p, P.lv_cost.p,
                               reinterpret_cast<long long *>(aux + 4), s));
  P.h_level_ptr.resize((size_t)nlev + 1);
  HIPCHK(h, hipMemcpyAsync(P.h_level_ptr.data(), P.level_ptr.p, sizeof(int32_t) * ((size_t)nlev + 1),
                           hipMemcpyDeviceToHost, s));
  P.h_lv_nnz.resize((size_t)nlev);
  HIPCHK(h, hipMemcpyAsync(P.h_lv_nnz.data(), P.lv_nnz.p, sizeof(int64_t) * (size_t)nlev, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipMemcpyAsync(&bits, aux + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (bits) return set_err(h, status_from_bits(bits), "batch: plan construction failed (bits 0x%x)", bits);
  STCHK(build_extra_hist(h, P, s));
  // longest-processing-time order: deepest matrices first, then largest
  std::vector<int32_t> order((size_t)nmat);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (h->b_nlev[(size_t)a] != h->b_nlev[(size_t)b]) return h->b_nlev[(size_t)a] > h->b_nlev[(size_t)b];
    return h->b_n[(size_t)a] > h->b_n[(size_t)b];
  });
  h->b_h_order = order;
  HIPCHK(h, h->b_q.alloc(2));
  HIPCHK(h, hipMemset(h->b_q.p, 0, 2 * sizeof(unsigned)));
  P.ready = true;
  h->b_ready = true;
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_batch_solve(sptrsv_handle_t h, int32_t nrhs, const double *d_b_cat, double *d_x_cat,
                                   hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  if (!h->b_ready) return set_err(h, SPTRSV_ERR_STATE, "batch: not analysed");
  if (nrhs < 1 || !d_b_cat || !d_x_cat) return set_err(h, SPTRSV_ERR_ARG, "batch solve args");
  Plan &P = h->bat;
  const size_t len = sizeof(double) * (size_t)P.n * (size_t)nrhs;
  const char *b0 = reinterpret_cast<const char *>(d_b_cat), *x0 = reinterpret_cast<const char *>(d_x_cat);
  if (b0 < x0 + len && x0 < b0 + len) return set_err(h, SPTRSV_ERR_ARG, "b and x overlap");
  STCHK(ensure_work(h, P, nrhs));
  const int32_t wg = effective_sched(P, nrhs).wg_threads;
  STCHK(batch_windows(h, nrhs, wg, s));
  HIPCHK(h, launch_batch_gather(P.n, nrhs, d_b_cat, h->b_mat_of_row.p, h->b_row_off_d.p, P.iperm.p, P.bp.p, s));
  if (h->b_nq > 0) {
    const int32_t grid = std::min(h->b_nq, batch_resident_blocks(wg));
    HIPCHK(h, launch_batch_run(wg, h->b_nq, grid, h->b_order.p, h->b_mwin.p, P.win.p, nrhs, thin_args(P), h->b_q.p,
                               h->d_err.p, s));
  }
  STCHK(batch_wide_solves(h, nrhs, wg, s));
  HIPCHK(h, launch_batch_scatter(P.n, nrhs, P.xp.p, h->b_mat_of_row.p, h->b_row_off_d.p, P.iperm.p, d_x_cat, s));
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_batch_solve_looped(sptrsv_handle_t h, int32_t nrhs, const double *d_b_cat, double *d_x_cat,
                                          hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  if (!h->b_ready) return set_err(h, SPTRSV_ERR_STATE, "batch: not analysed");
  if (nrhs < 1 || !d_b_cat || !d_x_cat) return set_err(h, SPTRSV_ERR_ARG, "batch solve args");
  Plan &P = h->bat;
  STCHK(ensure_work(h, P, nrhs));
  const int32_t wg = effective_sched(P, nrhs).wg_threads;
  STCHK(batch_windows(h, nrhs, wg, s));
  HIPCHK(h, launch_batch_gather(P.n, nrhs, d_b_cat, h->b_mat_of_row.p, h->b_row_off_d.p, P.iperm.p, P.bp.p, s));
  for (int32_t m = 0; m < h->b_nmat; ++m) {
    const int32_t wi = h->b_h_mwin[(size_t)m], nw = h->b_h_mwin[(size_t)m + 1] - wi - 1;
    if (nw >= 1) HIPCHK(h, launch_thin_run(wg, P.win.p + wi, nw, nrhs, thin_args(P), h->d_err.p, s));
  }
  STCHK(batch_wide_solves(h, nrhs, wg, s));
  HIPCHK(h, launch_batch_scatter(P.n, nrhs, P.xp.p, h->b_mat_of_row.p, h->b_row_off_d.p, P.iperm.p, d_x_cat, s));
  return SPTRSV_OK;
}

sptrsv_status_t sptrsv_batch_levels(sptrsv_handle_t h, int32_t i, int32_t *nlev, int32_t *d_level_ptr,
                                    int32_t *d_level_rows, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  if (!h->b_ready) return set_err(h, SPTRSV_ERR_STATE, "batch: not analysed");
  if (i < 0 || i >= h->b_nmat) return set_err(h, SPTRSV_ERR_ARG, "batch: matrix %d out of range", i);
  const int32_t nl = h->b_nlev[(size_t)i];
  if (nlev) *nlev = nl;
  const int32_t l0 = (int32_t)h->b_lvl_off[(size_t)i];
  const int32_t p0 = (int32_t)h->b_row_off[(size_t)i], n = h->b_n[(size_t)i];
  if (d_level_ptr)
    hipLaunchKernelGGL(k_offset_copy, dim3(grid_for(nl + 1, 256, 1024)), dim3(256), 0, s, h->bat.level_ptr.p + l0,
                       nl + 1, p0, d_level_ptr);
  if (d_level_rows)
    hipLaunchKernelGGL(k_offset_copy, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, h->bat.perm.p + p0, n, p0,
                       d_level_rows);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(s));
  return SPTRSV_OK;
}

}  // extern "C"
