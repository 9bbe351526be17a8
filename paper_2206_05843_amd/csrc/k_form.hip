// Triangular forms other than L x = b, brought to the lower-triangular form
// the level-set solve (Sec. II.A, Algorithm 1) and the rewriting (Sec. II.B,
// Sec. III) work on:
//   U x = b     ->  (J U J)(J x) = J b          J = row and column reversal
//   L^T x = b   ->  (J L^T J)(J x) = J b
//   U^T x = b   ->  U^T x = b, U^T = J (J U J)^T J
// J A J of a CSR is the CSR read backwards: entry q goes to nnz - 1 - q with
// column n - 1 - c, and row i starts at nnz - rp[n - i]. A transpose is a
// stable sort of the entries by column (rows stay ascending within a column).
#include "common.h"

namespace {

constexpr int kBlock = 256;

__global__ void k_rev_entries(int32_t n, int32_t nnz, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              const double *__restrict__ va, int32_t *orp, int32_t *oci, double *ova) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnz; q += stride) {
    oci[nnz - 1 - q] = n - 1 - ci[q];
    ova[nnz - 1 - q] = va[q];
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) orp[i] = nnz - rp[n - i];
}

__global__ void k_row_of_entry(int32_t n, const int32_t *__restrict__ rp, int32_t *row_of) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    for (int32_t q = rp[r]; q < rp[r + 1]; ++q) row_of[q] = (int32_t)r;
}

// ptr[c] = first entry whose (sorted, 0-based) key is >= c; ptr[n] = nnz.
__global__ void k_ptr_from_sorted(const int32_t *__restrict__ keys, int32_t nnz, int32_t n, int32_t *ptr) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t k = keys[e], kp = e == 0 ? -1 : keys[e - 1];
    for (int32_t c = kp + 1; c <= k; ++c) ptr[c] = (int32_t)e;
    if (e == nnz - 1)
      for (int32_t c = k + 1; c <= n; ++c) ptr[c] = nnz;
  }
}

__global__ void k_take_entries(int32_t nnz, const int32_t *__restrict__ order, const int32_t *__restrict__ row_of,
                               const double *__restrict__ va, int32_t *oci, double *ova) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t q = order[e];
    oci[e] = row_of[q];
    ova[e] = va[q];
  }
}

// Caller-facing index maps of a reversed system: caller row r is row n-1-r of
// the lower form, so position p holds caller row n-1-perm[p] and caller row r
// sits at position iperm[n-1-r].
__global__ void k_rev_io(int32_t n, const int32_t *__restrict__ perm, const int32_t *__restrict__ iperm,
                         int32_t *perm_io, int32_t *iperm_io) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    perm_io[i] = n - 1 - perm[i];
    iperm_io[i] = iperm[n - 1 - i];
  }
}

}  // namespace

hipError_t launch_rev_entries(int32_t n, int32_t nnz, const int32_t *rp, const int32_t *ci, const double *va,
                              int32_t *orp, int32_t *oci, double *ova, hipStream_t s) {
  hipLaunchKernelGGL(k_rev_entries, dim3(grid_for(nnz > n ? (int64_t)nnz : (int64_t)n + 1, kBlock, 8192)),
                     dim3(kBlock), 0, s, n, nnz, rp, ci, va, orp, oci, ova);
  return hipGetLastError();
}

hipError_t launch_row_of_entry(int32_t n, const int32_t *rp, int32_t *row_of, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_of_entry, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, rp, row_of);
  return hipGetLastError();
}

hipError_t launch_ptr_from_sorted(const int32_t *keys, int32_t nnz, int32_t n, int32_t *ptr, hipStream_t s) {
  if (nnz == 0) return hipMemsetAsync(ptr, 0, sizeof(int32_t) * ((size_t)n + 1), s);
  hipLaunchKernelGGL(k_ptr_from_sorted, dim3(grid_for(nnz, kBlock, 8192)), dim3(kBlock), 0, s, keys, nnz, n, ptr);
  return hipGetLastError();
}

hipError_t launch_take_entries(int32_t nnz, const int32_t *order, const int32_t *row_of, const double *va,
                               int32_t *oci, double *ova, hipStream_t s) {
  if (nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(k_take_entries, dim3(grid_for(nnz, kBlock, 8192)), dim3(kBlock), 0, s, nnz, order, row_of, va,
                     oci, ova);
  return hipGetLastError();
}

hipError_t launch_rev_io(int32_t n, const int32_t *perm, const int32_t *iperm, int32_t *perm_io, int32_t *iperm_io,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rev_io, dim3(grid_for(n, kBlock, 8192)), dim3(kBlock), 0, s, n, perm, iperm, perm_io,
                     iperm_io);
  return hipGetLastError();
}
