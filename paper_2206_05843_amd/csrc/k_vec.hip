// Vector kernels around the level chain: b (caller's column-major layout) to
// the level-ordered, RHS-interleaved work vector and back, the b-transform of
// the rewritten system (Sec. II.B), the residual check, and the batched
// variants of the gather and scatter.
#include <algorithm>

#include "common.h"

namespace {

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

// The gather and scatter over a list of tiles (workgroups stride the list;
// the grid is capped so that a group running beside the level chain leaves
// most of the device to it).
__global__ void k_gather_tiles(int32_t n, int32_t nrhs, const double *__restrict__ b, int64_t ldb,
                               const int32_t *__restrict__ iperm, const int32_t *__restrict__ tiles, int32_t ntiles,
                               double *bp) {
  __shared__ double tile[64][33];
  for (int32_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const int32_t r0 = tiles[ti] * 64;
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
}

__global__ void k_scatter_tiles(int32_t n, int32_t nrhs, const double *__restrict__ xp,
                                const int32_t *__restrict__ iperm, const int32_t *__restrict__ tiles, int32_t ntiles,
                                double *x, int64_t ldx) {
  __shared__ double tile[64][33];
  for (int32_t ti = blockIdx.x; ti < ntiles; ti += gridDim.x) {
    const int32_t r0 = tiles[ti] * 64;
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
}

// Smallest and largest position of the rows of each 64-row tile (a wave per tile).
__global__ void k_tile_span(int32_t n, const int32_t *__restrict__ iperm, int32_t *first, int32_t *last) {
  const int32_t ntiles = (n + 63) / 64;
  const int lane = threadIdx.x & 63;
  for (int32_t t = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); t < ntiles;
       t += (int32_t)((gridDim.x * blockDim.x) >> 6)) {
    const int32_t r = t * 64 + lane;
    int32_t lo = r < n ? iperm[r] : INT32_MAX, hi = r < n ? iperm[r] : -1;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      lo = min(lo, __shfl_xor(lo, off, 64));
      hi = max(hi, __shfl_xor(hi, off, 64));
    }
    if (lane == 0) {
      first[t] = lo;
      last[t] = hi;
    }
  }
}

__global__ void k_gather1(int32_t n, const double *__restrict__ b, const int32_t *__restrict__ iperm, double *bp) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    bp[iperm[r]] = b[r];
}

// The b-transform of the rewritten system (Sec. II.B) on the rows where T has
// off-diagonals (positions tpos): b'(pos, c) = b(row, c) + sum over T's row
// of T(pos, k) b(k, c), with row = perm[pos], T's columns k in the caller's
// row numbering and b the caller's column-major right-hand sides (T's unit
// diagonal is implicit). Only b is read, so the items are independent.
//
// One thread per (row, column of b): for short rows of T.
__global__ void k_apply_t(int32_t nt, int32_t nrhs, const int32_t *__restrict__ tpos, const int32_t *__restrict__ perm,
                          const int32_t *__restrict__ trp, const int32_t *__restrict__ tcol,
                          const double *__restrict__ tva, const double *__restrict__ b, int64_t rs, int64_t cs,
                          double *bp) {
  const int64_t total = (int64_t)nt * nrhs;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = (int32_t)(i / nrhs);
    const int32_t c = (int32_t)(i - (int64_t)j * nrhs);
    const int32_t pos = tpos[j];
    const double *bc = b + (int64_t)c * cs;
    double acc = bc[(int64_t)perm[pos] * rs];
    const int32_t qb = trp[pos], qe = trp[pos + 1];
    for (int32_t q = qb; q < qe; ++q) acc += tva[q] * bc[(int64_t)tcol[q] * rs];
    bp[(int64_t)pos * nrhs + c] = acc;
  }
}

// G lanes per row of T (G divides 64): the lanes stride the row together, so
// its columns and values are read in coalesced runs, and the partial sums are
// combined by a butterfly inside the group. For long rows of T.
template <int G>
__global__ void k_apply_t_group(int32_t nt, int32_t nrhs, const int32_t *__restrict__ tpos,
                                const int32_t *__restrict__ perm, const int32_t *__restrict__ trp,
                                const int32_t *__restrict__ tcol, const double *__restrict__ tva,
                                const double *__restrict__ b, int64_t rs, int64_t cs, double *bp) {
  const int lane = threadIdx.x % G;
  const int64_t ng = (int64_t)gridDim.x * (blockDim.x / G);
  // every lane of a group takes the same trip count, so the butterfly sees
  // the whole group
  for (int64_t j = (int64_t)blockIdx.x * (blockDim.x / G) + threadIdx.x / G; j < nt; j += ng) {
    const int32_t pos = tpos[j];
    const int32_t qb = trp[pos], qe = trp[pos + 1];
    const int32_t row = perm[pos];
    for (int32_t c = 0; c < nrhs; ++c) {
      const double *bc = b + (int64_t)c * cs;
      double acc = 0.0;
      for (int32_t q = qb + lane; q < qe; q += G) acc += tva[q] * bc[(int64_t)tcol[q] * rs];
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, G);
      if (lane == 0) bp[(int64_t)pos * nrhs + c] = bc[(int64_t)row * rs] + acc;
    }
  }
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

// Right-hand sides stored by rows: one row's nrhs values move together.
__global__ void k_gather_rows(int64_t total, int32_t nrhs, const double *__restrict__ b,
                              const int32_t *__restrict__ perm, double *bp) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pos = i / nrhs;
    bp[i] = b[(int64_t)perm[pos] * nrhs + (i - pos * nrhs)];
  }
}

__global__ void k_scatter_rows(int64_t total, int32_t nrhs, const double *__restrict__ xp,
                               const int32_t *__restrict__ perm, double *x) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pos = i / nrhs;
    x[(int64_t)perm[pos] * nrhs + (i - pos * nrhs)] = xp[i];
  }
}

__global__ void k_map_ell(int32_t n, const int4 *__restrict__ ell_c, const int32_t *__restrict__ perm, int4 *ell_r) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int4 e = ell_c[i];
    ell_r[i] = make_int4(e.x >= 0 ? perm[e.x] : -1, e.y >= 0 ? perm[e.y] : -1, e.z >= 0 ? perm[e.z] : -1,
                         e.w >= 0 ? perm[e.w] : -1);
  }
}

__global__ void k_map_cols(int64_t nnz, const int32_t *__restrict__ col, const int32_t *__restrict__ perm, int32_t *out) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x)
    out[q] = perm[col[q]];
}

__global__ void k_tflag_zero(int32_t n, uint8_t *tflag) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) tflag[i] = 0;
}

__global__ void k_tflag_set(int32_t nt, const int32_t *__restrict__ tpos, uint8_t *tflag) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nt; i += gridDim.x * blockDim.x) tflag[tpos[i]] = 1;
}

__global__ void k_scatter1(int32_t n, const double *__restrict__ xp, const int32_t *__restrict__ iperm, double *x) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    x[r] = xp[iperm[r]];
}

// max_i |(L x - b)[i, c]| per column, original numbering; results as the bit
// patterns of non-negative doubles (monotone as unsigned integers).
__global__ void k_residual(int32_t n, int32_t nrhs, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ va, const double *__restrict__ b, int64_t ldb,
                           const double *__restrict__ x, int64_t ldx, int rev, unsigned long long *out) {
  for (int32_t c = 0; c < nrhs; ++c) {
    double m = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
      double s = 0.0;
      for (int32_t q = rp[r]; q < rp[r + 1]; ++q) s += va[q] * x[(int64_t)c * ldx + (rev ? n - 1 - ci[q] : ci[q])];
      const double d = fabs(s - b[(int64_t)c * ldb + (rev ? n - 1 - r : r)]);
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
// offset nrhs * row_off[m], ld = n_m. A tile of 64 global rows x up to 32
// columns is staged in LDS: the caller's side is read/written down columns
// (contiguous within each matrix), the work vector's side one row's
// right-hand sides at a time (contiguous at the row's position).
__global__ void k_batch_gather(int64_t total, int32_t nrhs, const double *__restrict__ b,
                               const int32_t *__restrict__ mat_of_row, const int64_t *__restrict__ row_off,
                               const int32_t *__restrict__ iperm, double *bp) {
  __shared__ double tile[64][33];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  for (int32_t c0 = 0; c0 < nrhs; c0 += 32) {
    const int32_t nc = min(32, nrhs - c0);
    for (int idx = threadIdx.x; idx < 64 * nc; idx += blockDim.x) {
      const int c = idx / 64, rr = idx % 64;
      const int64_t r = r0 + rr;
      if (r < total) {
        const int32_t m = mat_of_row[r];
        const int64_t ro = row_off[m], nm = row_off[m + 1] - ro;
        tile[rr][c] = b[nrhs * ro + (int64_t)(c0 + c) * nm + (r - ro)];
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * nc; idx += blockDim.x) {
      const int rr = idx / nc, c = idx % nc;
      const int64_t r = r0 + rr;
      if (r < total) bp[(int64_t)iperm[r] * nrhs + c0 + c] = tile[rr][c];
    }
    __syncthreads();
  }
}

__global__ void k_batch_scatter(int64_t total, int32_t nrhs, const double *__restrict__ xp,
                                const int32_t *__restrict__ mat_of_row, const int64_t *__restrict__ row_off,
                                const int32_t *__restrict__ iperm, double *x) {
  __shared__ double tile[64][33];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  for (int32_t c0 = 0; c0 < nrhs; c0 += 32) {
    const int32_t nc = min(32, nrhs - c0);
    for (int idx = threadIdx.x; idx < 64 * nc; idx += blockDim.x) {
      const int rr = idx / nc, c = idx % nc;
      const int64_t r = r0 + rr;
      if (r < total) tile[rr][c] = xp[(int64_t)iperm[r] * nrhs + c0 + c];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * nc; idx += blockDim.x) {
      const int c = idx / 64, rr = idx % 64;
      const int64_t r = r0 + rr;
      if (r < total) {
        const int32_t m = mat_of_row[r];
        const int64_t ro = row_off[m], nm = row_off[m + 1] - ro;
        x[nrhs * ro + (int64_t)(c0 + c) * nm + (r - ro)] = tile[rr][c];
      }
    }
    __syncthreads();
  }
}

// b = A 1: row sums of a CSR matrix (the right-hand side of the rewrite's
// self-check, whose exact solution is all ones).
__global__ void k_row_sums(int32_t n, const int32_t *__restrict__ rp, const double *__restrict__ va, double *b) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int32_t q = rp[r]; q < rp[r + 1]; ++q) s += va[q];
    b[r] = s;
  }
}

// out[0] = max |x1 - x0| (a NaN counts as infinite), out[1] = max |x0|, as
// the bit patterns of non-negative doubles (monotone as unsigned integers).
__global__ void k_max_abs_diff(int32_t n, const double *__restrict__ x0, const double *__restrict__ x1,
                               unsigned long long *out) {
  double d = 0.0, m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double e = fabs(x1[i] - x0[i]);
    if (e != e) e = INFINITY;
    d = e > d ? e : d;
    double a = fabs(x0[i]);
    if (a != a) a = INFINITY;
    m = a > m ? a : m;
  }
  for (int off = 32; off > 0; off >>= 1) {
    d = fmax(d, __shfl_xor(d, off, 64));
    m = fmax(m, __shfl_xor(m, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(d));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(m));
  }
}

#ifndef SPTRSV_TILE_GRID
#define SPTRSV_TILE_GRID 1024
#endif
constexpr int32_t kTileGrid = SPTRSV_TILE_GRID;  // workgroups of one tile-group transpose

}  // namespace

hipError_t launch_gather(int32_t n, int32_t nrhs, const double *b, int64_t ldb, const int32_t *iperm, double *bp,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nrhs == 1)
    hipLaunchKernelGGL(k_gather1, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, b, iperm, bp);
  else
    hipLaunchKernelGGL(k_gather, dim3((n + 63) / 64), dim3(256), 0, s, n, nrhs, b, ldb, iperm, bp);
  return hipGetLastError();
}

hipError_t launch_gather_tiles(int32_t n, int32_t nrhs, const double *b, int64_t ldb, const int32_t *iperm,
                               const int32_t *tiles, int32_t ntiles, double *bp, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_tiles, dim3(std::min(ntiles, kTileGrid)), dim3(256), 0, s, n, nrhs, b, ldb, iperm, tiles,
                     ntiles, bp);
  return hipGetLastError();
}

hipError_t launch_scatter_tiles(int32_t n, int32_t nrhs, const double *xp, const int32_t *iperm,
                                const int32_t *tiles, int32_t ntiles, double *x, int64_t ldx, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_tiles, dim3(std::min(ntiles, kTileGrid)), dim3(256), 0, s, n, nrhs, xp, iperm, tiles,
                     ntiles, x, ldx);
  return hipGetLastError();
}

hipError_t launch_row_sums(int32_t n, const int32_t *rp, const double *va, double *b, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_sums, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, rp, va, b);
  return hipGetLastError();
}

hipError_t launch_max_abs_diff(int32_t n, const double *x0, const double *x1, unsigned long long *out,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_max_abs_diff, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n, x0, x1, out);
  return hipGetLastError();
}

hipError_t launch_tile_span(int32_t n, const int32_t *iperm, int32_t *first, int32_t *last, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t ntiles = (n + 63) / 64;
  hipLaunchKernelGGL(k_tile_span, dim3(grid_for(ntiles * 64, 256, 16384)), dim3(256), 0, s, n, iperm, first, last);
  return hipGetLastError();
}

hipError_t launch_apply_t(int32_t nt, int32_t nrhs, int32_t lanes, const int32_t *tpos, const int32_t *perm,
                          const int32_t *trp, const int32_t *tcol, const double *tva, const double *b, int64_t rs,
                          int64_t cs, double *bp, hipStream_t s) {
  if (nt == 0) return hipSuccess;
  const int64_t groups = nt;
  switch (lanes) {
    case 1:
      hipLaunchKernelGGL(k_apply_t, dim3(grid_for((int64_t)nt * nrhs, 256, 16384)), dim3(256), 0, s, nt, nrhs, tpos,
                         perm, trp, tcol, tva, b, rs, cs, bp);
      break;
    case 4:
      hipLaunchKernelGGL(k_apply_t_group<4>, dim3(grid_for(groups * 4, 256, 16384)), dim3(256), 0, s, nt, nrhs, tpos,
                         perm, trp, tcol, tva, b, rs, cs, bp);
      break;
    case 16:
      hipLaunchKernelGGL(k_apply_t_group<16>, dim3(grid_for(groups * 16, 256, 16384)), dim3(256), 0, s, nt, nrhs,
                         tpos, perm, trp, tcol, tva, b, rs, cs, bp);
      break;
    case 64:
      hipLaunchKernelGGL(k_apply_t_group<64>, dim3(grid_for(groups * 64, 256, 16384)), dim3(256), 0, s, nt, nrhs,
                         tpos, perm, trp, tcol, tva, b, rs, cs, bp);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather_rows(int32_t n, int32_t nrhs, const double *b, const int32_t *perm, double *bp,
                              hipStream_t s) {
  const int64_t total = (int64_t)n * nrhs;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(total, 256, 16384)), dim3(256), 0, s, total, nrhs, b, perm, bp);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(int32_t n, int32_t nrhs, const double *xp, const int32_t *perm, double *x,
                               hipStream_t s) {
  const int64_t total = (int64_t)n * nrhs;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_rows, dim3(grid_for(total, 256, 16384)), dim3(256), 0, s, total, nrhs, xp, perm, x);
  return hipGetLastError();
}

hipError_t launch_map_ell(int32_t n, const int4 *ell_c, const int32_t *perm, int4 *ell_r, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_map_ell, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, ell_c, perm, ell_r);
  return hipGetLastError();
}

hipError_t launch_map_cols(int64_t nnz, const int32_t *col, const int32_t *perm, int32_t *out, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_map_cols, dim3(grid_for(nnz, 256, 16384)), dim3(256), 0, s, nnz, col, perm, out);
  return hipGetLastError();
}

hipError_t launch_tflag(int32_t n, int32_t nt, const int32_t *tpos, uint8_t *tflag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tflag_zero, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n, tflag);
  if (nt > 0) hipLaunchKernelGGL(k_tflag_set, dim3(grid_for(nt, 256, 4096)), dim3(256), 0, s, nt, tpos, tflag);
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

hipError_t launch_residual(int32_t n, int32_t nrhs, const int32_t *rp, const int32_t *ci, const double *va,
                           const double *b, int64_t ldb, const double *x, int64_t ldx, unsigned long long *out,
                           bool rev, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n, nrhs, rp, ci, va, b, ldb, x,
                     ldx, rev ? 1 : 0, out);
  return hipGetLastError();
}

hipError_t launch_batch_gather(int64_t total, int32_t nrhs, const double *b, const int32_t *mat_of_row,
                               const int64_t *row_off, const int32_t *iperm, double *bp, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_gather, dim3((unsigned)((total + 63) / 64)), dim3(256), 0, s, total, nrhs, b, mat_of_row,
                     row_off, iperm, bp);
  return hipGetLastError();
}

hipError_t launch_batch_scatter(int64_t total, int32_t nrhs, const double *xp, const int32_t *mat_of_row,
                                const int64_t *row_off, const int32_t *iperm, double *x, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_scatter, dim3((unsigned)((total + 63) / 64)), dim3(256), 0, s, total, nrhs, xp,
                     mat_of_row, row_off, iperm, x);
  return hipGetLastError();
}
