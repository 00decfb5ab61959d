// trals_fit_error_noalloc: the relative fit error ||TR(G) - X||_F / ||X||_F (the error
// trals_fit_error reports, Section 4.1) of given cores against a given dense tensor, for
// callers that cannot allocate device memory.  It runs the same kernels as the handle's fit
// (core import to slice-major FP64, per-block squared residuals, ||X||^2 partial sums,
// fixed-order sums), with their scratch in one fixed device array of this file instead of a
// workspace, and never synchronises: the result is written to a device double on the caller's
// stream.
//
// Scratch layout (doubles): slice-major copies of the N cores (sum_n I_n R_{n-1} R_n), the fit
// kernel's per-block partial sums (ceil(prod_{k<N-1} I_k / kFitRows)), the ||X||^2 partial sums
// (kScanBlocks), then r2 and x2.  Every word the kernels read is written earlier in the same
// call, so nothing needs clearing.  The array is per GPU and shared by every call on it: calls
// that overlap on one GPU (different streams, or host threads) race on it and must be
// serialised by the caller.
#include <string.h>

#include <mutex>

#include "../../include/trals.h"
#include "kernels.h"

namespace trals {
namespace {

constexpr size_t kScratchDoubles = TRALS_NOALLOC_SCRATCH_BYTES / sizeof(double);
static_assert(TRALS_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch is whole 256-byte lines");

// The device array.  In host code this name is only a handle for hipGetSymbolAddress; the
// address every kernel receives is the per-device pointer that call returns.
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// scratch's address on the current device (looked up once per device, with it current)
hipError_t scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = (double*)p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace trals

using namespace trals;

extern "C" int trals_fit_error_noalloc(int32_t order, const int64_t* dims, const int32_t* ranks,
                                       const void* cores_dev, int32_t cores_dtype, const void* X_dev,
                                       int32_t x_dtype, double* rel_err_dev, void* stream) {
  if (!dims || !ranks || !cores_dev || !X_dev || !rel_err_dev) return TRALS_EINVAL;
  if (order < 2 || order > kMaxOrder) return TRALS_EINVAL;
  if ((cores_dtype != TRALS_F64 && cores_dtype != TRALS_F32) || (x_dtype != TRALS_F64 && x_dtype != TRALS_F32))
    return TRALS_EINVAL;
  int64_t E = 1;
  size_t need = 0;
  for (int n = 0; n < order; ++n) {
    if (dims[n] < 1 || dims[n] > ((int64_t)1 << 21)) return TRALS_EINVAL;
    if (ranks[n] < 1 || ranks[n] > kMaxRank) return TRALS_EINVAL;
    if (E > ((int64_t)1 << 40) / dims[n]) return TRALS_EINVAL;
    E *= dims[n];
    need += (size_t)dims[n] * ranks[(n + order - 1) % order] * ranks[n];
  }
  const int64_t rows = E / dims[order - 1];
  const int64_t fit_blocks = (rows + kFitRows - 1) / kFitRows;
  need += (size_t)fit_blocks + kScanBlocks + 2;
  if (need > kScratchDoubles) return TRALS_ERANGE;
  double* base = nullptr;
  if (scratch_on_current_device(&base) != hipSuccess) return TRALS_EHIP;
  hipStream_t s = (hipStream_t)stream;
  Ring ring;
  memset(&ring, 0, sizeof(ring));
  ring.N = order;
  FitArgs fa;
  memset(&fa, 0, sizeof(fa));
  double* cur = base;
  size_t src_off = 0;
  const size_t esz = cores_dtype == TRALS_F64 ? 8 : 4;
  for (int n = 0; n < order; ++n) {
    const int Rp = ranks[(n + order - 1) % order], Rn = ranks[n];
    const int I = (int)dims[n];
    ring.dims[n] = I;
    ring.ranks[n] = Rn;
    if (launch_core_import((const char*)cores_dev + src_off, cores_dtype == TRALS_F64 ? 0 : 1, cur, 0, Rp, I, Rn, s) !=
        hipSuccess)
      return TRALS_EHIP;
    fa.cores.p[n] = cur;
    cur += (size_t)Rp * I * Rn;
    src_off += (size_t)Rp * I * Rn * esz;
  }
  double* fit_part = cur;
  double* scan_part = fit_part + fit_blocks;
  double* r2 = scan_part + kScanBlocks;
  double* x2 = r2 + 1;
  fa.ring = ring;
  fa.X = X_dev;
  fa.rows = rows;
  fa.partial = fit_part;
  int nb = 0;
  const int xdt = x_dtype == TRALS_F64 ? 0 : 1;
  if (launch_fit(fa, 0, xdt, &nb, s) != hipSuccess) return TRALS_EHIP;
  if (launch_sum_partials(fit_part, nb, r2, s) != hipSuccess) return TRALS_EHIP;
  if (launch_scan_x(X_dev, xdt, E, scan_part, kScanBlocks, nullptr, s) != hipSuccess) return TRALS_EHIP;
  if (launch_sum_partials(scan_part, kScanBlocks, x2, s) != hipSuccess) return TRALS_EHIP;
  if (launch_dense_fit_dev(r2, x2, rel_err_dev, s) != hipSuccess) return TRALS_EHIP;
  return TRALS_OK;
}
