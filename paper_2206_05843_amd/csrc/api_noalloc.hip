// sptrsv_solve_noalloc: the solve of sptrsv_solve with its two work vectors
// (b, or b' = T b, in level order and the solution in level order) taken from
// a static device array instead of handle-owned allocations, for callers that
// cannot allocate device memory.
//
// The array is a file-scope __device__ symbol: one copy per GPU, created when
// the code object is loaded and held until the process ends. Host code never
// uses its name as an address (that would be a host-side stand-in); every
// device's address comes from hipGetSymbolAddress, taken once per device with
// that device current, when the first handle is created on it.
#include <mutex>

#include "common.h"

namespace {

// 64 MiB: both work vectors of a solve with n * nrhs <= 4M.
constexpr size_t kScratchDoubles = (size_t)8 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

}  // namespace

// Address of this device's copy of the work area (null if it could not be
// found). Called by sptrsv_create with the handle's device current.
hipError_t noalloc_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[dev]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[dev] = static_cast<double *>(p);
  return hipSuccess;
}

extern "C" {

sptrsv_status_t sptrsv_solve_noalloc(sptrsv_handle_t h, int which, int32_t nrhs, const double *d_b, int64_t ldb,
                                     double *d_x, int64_t ldx, hipStream_t s) {
  if (!h) return SPTRSV_ERR_ARG;
  sptrsv_status_t st;
  Plan *P = solve_plan(h, which, nrhs, d_b, ldb, d_x, ldx, &st);
  if (!P) return st;
  const size_t need = (size_t)P->n * (size_t)nrhs;
  if (2 * need > kScratchDoubles)
    return set_err(h, SPTRSV_ERR_ARG,
                   "solve_noalloc: n * nrhs = %zu exceeds the static work area (%zu per work vector)", need,
                   kScratchDoubles / 2);
  if (P->n == 0) return SPTRSV_OK;
  if (!runs_ready(*P, nrhs))
    return set_err(h, SPTRSV_ERR_STATE,
                   "solve_noalloc: the schedule for nrhs=%d is not built; call sptrsv_prepare first", nrhs);
  double *base = (h->dev >= 0 && h->dev < kMaxDevices) ? g_scratch[h->dev] : nullptr;
  if (!base) return set_err(h, SPTRSV_ERR_STATE, "solve_noalloc: no work area address for device %d", h->dev);
  return solve_runs(h, *P, nrhs, d_b, ldb, d_x, ldx, base, base + need, s);
}

}  // extern "C"
