// Static images of the thin-run LDS windows (the level-scheduled solve of
// Sec. II.A, Algorithm 1, applied to L or to the rewritten L' of Sec. II.B).
//
// Everything a window holds in LDS before its levels are solved, except the
// right-hand side and the values of x it reads from earlier windows, depends
// on the matrix and the window cut only. It is built here once per schedule:
// per window, back to back in device memory,
//   [R x double2]  the row's first two in-window dependencies, weights scaled
//                  by 1/diagonal (0 when absent);
//   [NO x Dep]     the third and later in-window dependencies of the rows, in
//                  row order, each row's contiguous and in its column order;
//   [R x uint2]    packed {slot0, slot1 | in-window count, first overflow
//                  record}, padded to 16 bytes; absent slots point to the
//                  window's zero row R.
// The dependencies of a row on positions before its window go to a CSR over
// positions (ext_ptr, ext) in the row's column order. Positions and window
// layouts come from exclusive scans, so the images do not depend on thread
// timing.
#include "common.h"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int32_t level_of(const int32_t *__restrict__ level_ptr, int32_t nlev, int32_t p) {
  int32_t lo = 0, hi = nlev - 1;
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (level_ptr[mid] <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_img_count(int32_t n, const int32_t *__restrict__ level_ptr, int32_t nlev,
                            const int32_t *__restrict__ lvl_win, const int4 *__restrict__ win,
                            const int32_t *__restrict__ srp, const int32_t *__restrict__ sci, long long *ovf_cnt,
                            long long *ext_cnt) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t wi = lvl_win[level_of(level_ptr, nlev, (int32_t)p)];
    long long in = 0, ex = 0;
    if (wi >= 0) {
      const int32_t P0 = level_ptr[win[wi].x];
      for (int32_t q = srp[p]; q < srp[p + 1]; ++q) {
        if (sci[q] >= P0) ++in; else ++ex;
      }
    }
    ovf_cnt[p] = in > 2 ? in - 2 : 0;
    ext_cnt[p] = ex;
  }
}

__global__ void k_win_prefix(int32_t nent, const int4 *__restrict__ win, const int32_t *__restrict__ level_ptr,
                             int32_t n, const long long *__restrict__ ovf_ex, const long long *__restrict__ ovf_cnt,
                             long long *out) {
  for (int32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < nent; e += gridDim.x * blockDim.x) {
    const int32_t p = level_ptr[win[e].x];
    out[e] = p < n ? ovf_ex[p] : (n > 0 ? ovf_ex[n - 1] + ovf_cnt[n - 1] : 0);
  }
}

__global__ void k_img_fill(int32_t n, const int32_t *__restrict__ level_ptr, int32_t nlev,
                           const int32_t *__restrict__ lvl_win, const int4 *__restrict__ win,
                           const int32_t *__restrict__ srp, const int32_t *__restrict__ sci,
                           const double *__restrict__ sva, const double *__restrict__ sdg,
                           const long long *__restrict__ ovf_ex, const int32_t *__restrict__ ext_ptr, uint4 *img,
                           ExtDep *ext, const int32_t *__restrict__ perm) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t wi = lvl_win[level_of(level_ptr, nlev, (int32_t)p)];
    if (wi < 0) continue;
    const int4 W = win[wi];
    const int32_t P0 = level_ptr[W.x], R = level_ptr[win[wi + 1].x] - P0, NO = W.z;
    const int32_t s = (int32_t)p - P0;
    const int32_t ob = (int32_t)(ovf_ex[p] - ovf_ex[P0]);
    double2 *rw = reinterpret_cast<double2 *>(img + W.w);
    Dep *ovf = reinterpret_cast<Dep *>(rw + R);
    uint2 *rix = reinterpret_cast<uint2 *>(ovf + NO);
    const double dinv = 1.0 / sdg[p];
    int32_t kin = 0, s0 = R, s1 = R, e = ext_ptr[p];
    double w0 = 0.0, w1 = 0.0;
    for (int32_t q = srp[p]; q < srp[p + 1]; ++q) {
      const int32_t k = sci[q];
      const double wv = sva[q];
      if (k < P0) {
        ExtDep d;
        d.w = wv;
        d.col = k;
        d.row = perm ? perm[k] : k;
        ext[e++] = d;
        continue;
      }
      if (kin == 0) {
        s0 = k - P0;
        w0 = wv * dinv;
      } else if (kin == 1) {
        s1 = k - P0;
        w1 = wv * dinv;
      } else {
        Dep d;
        d.w = wv * dinv;
        d.slot = k - P0;
        d.pad = 0;
        ovf[ob + kin - 2] = d;
      }
      ++kin;
    }
    rw[s] = make_double2(w0, w1);
    rix[s] = pack_rix(s0, s1, kin, kin > 2 ? ob : 0);
  }
}

}  // namespace

hipError_t launch_img_count(int32_t n, const int32_t *level_ptr, int32_t nlev, const int32_t *lvl_win,
                            const int4 *win, const int32_t *srp, const int32_t *sci, long long *ovf_cnt,
                            long long *ext_cnt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_img_count, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, level_ptr, nlev, lvl_win,
                     win, srp, sci, ovf_cnt, ext_cnt);
  return hipGetLastError();
}

hipError_t launch_win_prefix(int32_t nent, const int4 *win, const int32_t *level_ptr, int32_t n,
                             const long long *ovf_ex, const long long *ovf_cnt, long long *out, hipStream_t s) {
  if (nent == 0) return hipSuccess;
  hipLaunchKernelGGL(k_win_prefix, dim3(grid_for(nent, kBlock, 4096)), dim3(kBlock), 0, s, nent, win, level_ptr, n,
                     ovf_ex, ovf_cnt, out);
  return hipGetLastError();
}

hipError_t launch_img_fill(int32_t n, const int32_t *level_ptr, int32_t nlev, const int32_t *lvl_win, const int4 *win,
                           const int32_t *srp, const int32_t *sci, const double *sva, const double *sdg,
                           const long long *ovf_ex, const int32_t *ext_ptr, uint4 *img, ExtDep *ext,
                           const int32_t *perm, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_img_fill, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, level_ptr, nlev, lvl_win,
                     win, srp, sci, sva, sdg, ovf_ex, ext_ptr, img, ext, perm);
  return hipGetLastError();
}
