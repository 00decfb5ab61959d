// Normalisation of the updated core (an optional step between updates; the paper notes that
// normalisation steps can be added to its algorithms, Section 2.1).
//
// Core n viewed as the (I_n R_{n-1}) x R_n matrix G (rows (i, a), column b: slice-major storage
// is exactly this row-major matrix) is replaced by Q = G R^{-1} from G = Q R, R upper
// triangular with a positive diagonal, and R is multiplied into the next core:
// G_{n+1}(:, i, :) <- R G_{n+1}(:, i, :).  TR(G) is unchanged, and so is every leverage
// distribution (R acts on one bond index, an invertible change of the unfolding's columns).
// R comes from the Cholesky factor of the small Gram S = G^T G = L L^T, R = L^T (the Gram is
// formed by k_syrk); Q = G L^{-T}, i.e. row q = L^{-1} g.
#include "kernels.h"

namespace trals {

namespace {

constexpr int kGMax = 32;  // bond ranks up to kMaxRank
constexpr int kGLd = kGMax + 1;

// One wave: S (lower triangle, row-major R x R) -> L and L^{-1} (row-major, zero above).
__global__ __launch_bounds__(64) void k_gauge_factor(const double* __restrict__ S, int R, double* __restrict__ out,
                                                     int* status) {
  __shared__ double a[kGMax * kGLd];
  __shared__ double li[kGMax * kGLd];
  if (*status != kDevOk) return;
  const int lane = threadIdx.x;
  for (int e = lane; e < R * R; e += 64) {
    const int i = e / R, j = e - i * R;
    a[i * kGLd + j] = j <= i ? S[i * R + j] : 0.0;
  }
  __syncthreads();
  double mx = 0.0;
  for (int i = 0; i < R; ++i) mx = fmax(mx, a[i * kGLd + i]);
  const double tol = (double)R * 2.220446049250313e-16 * mx;
  int bad = !(mx > 0.0) || !(mx < __builtin_huge_val());
  // right-looking Cholesky in LDS: lane i owns row i (one wave: LDS keeps its accesses in order)
  for (int k = 0; k < R && !bad; ++k) {
    const double p = a[k * kGLd + k];
    if (!(p > tol) || !(p < __builtin_huge_val())) {
      bad = 1;
      break;
    }
    const double d = sqrt(p);
    const int i = lane;
    if (i > k && i < R) a[i * kGLd + k] /= d;
    __builtin_amdgcn_wave_barrier();
    if (i == k) a[k * kGLd + k] = d;
    if (i > k && i < R) {
      const double lik = a[i * kGLd + k];
      for (int j = k + 1; j <= i; ++j) a[i * kGLd + j] -= lik * a[j * kGLd + k];
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (bad) {
    if (lane == 0) *status = kDevSingular;
    return;
  }
  // L^{-1}: lane c computes column c by forward substitution
  if (lane < R) {
    const int c = lane;
    for (int i = 0; i < R; ++i) {
      double s = i == c ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= a[i * kGLd + k] * li[k * kGLd + c];
      li[i * kGLd + c] = i < c ? 0.0 : s / a[i * kGLd + i];
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int e = lane; e < R * R; e += 64) {
    const int i = e / R, j = e - i * R;
    out[e] = j <= i ? a[i * kGLd + j] : 0.0;                // L
    out[kGMax * kGMax + e] = j <= i ? li[i * kGLd + j] : 0.0;  // L^{-1}
  }
}

// Blocks [0, rb): rows of core n, q = L^{-1} g (one row per thread).  Blocks [rb, ...): columns
// of the next core's slices, s(:, c) <- L^T s(:, c) (one (slice, column) per thread).
__global__ __launch_bounds__(256) void k_gauge_apply(double* __restrict__ core, int64_t rows, int R,
                                                     double* __restrict__ next, int64_t cols, int Rnext,
                                                     const double* __restrict__ f, int64_t rb, const int* status) {
  __shared__ double m[kGMax * kGMax];
  if (*status != kDevOk) return;
  const bool first = (int64_t)blockIdx.x < rb;
  const double* src = f + (first ? kGMax * kGMax : 0);  // L^{-1} for the rows, L for the slices
  for (int e = threadIdx.x; e < R * R; e += 256) m[e] = src[e];
  __syncthreads();
  double v[kGMax], o[kGMax];
  if (first) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= rows) return;
    double* g = core + r * R;
#pragma unroll
    for (int b = 0; b < kGMax; ++b) v[b] = b < R ? g[b] : 0.0;
#pragma unroll
    for (int b = 0; b < kGMax; ++b) {
      double t = 0.0;
#pragma unroll
      for (int c = 0; c <= b; ++c) t = b < R ? fma(m[b * R + c], v[c], t) : t;
      o[b] = t;
    }
#pragma unroll
    for (int b = 0; b < kGMax; ++b)
      if (b < R) g[b] = o[b];
  } else {
    const int64_t e = ((int64_t)blockIdx.x - rb) * 256 + threadIdx.x;
    if (e >= cols) return;
    const int64_t i = e / Rnext;
    const int c = (int)(e - i * Rnext);
    double* s = next + i * (int64_t)R * Rnext + c;  // slice i is R x Rnext, row-major
#pragma unroll
    for (int b = 0; b < kGMax; ++b) v[b] = b < R ? s[(int64_t)b * Rnext] : 0.0;
#pragma unroll
    for (int b = 0; b < kGMax; ++b) {
      double t = 0.0;
#pragma unroll
      for (int b2 = b; b2 < kGMax; ++b2) t = b2 < R ? fma(m[b2 * R + b], v[b2], t) : t;  // L^T(b, b2) = L(b2, b)
      o[b] = t;
    }
#pragma unroll
    for (int b = 0; b < kGMax; ++b)
      if (b < R) s[(int64_t)b * Rnext] = o[b];
  }
}

}  // namespace

size_t gauge_work_doubles() { return 2 * kGMax * kGMax; }

hipError_t launch_gauge(double* core, int64_t In, int Rp, int R, double* next, int64_t In_next, int Rnext,
                        double* S, double* work, int* status, hipStream_t s) {
  if (R > kGMax || R < 1) return hipErrorInvalidValue;
  const int64_t rows = In * Rp;
  hipError_t e = launch_syrk(core, rows, R, S, status, s);
  if (e != hipSuccess) return e;
  k_gauge_factor<<<1, 64, 0, s>>>(S, R, work, status);
  const int64_t rb = (rows + 255) / 256;
  const int64_t cols = In_next * Rnext;
  const int64_t cb = (cols + 255) / 256;
  k_gauge_apply<<<(unsigned)(rb + cb), 256, 0, s>>>(core, rows, R, next, cols, Rnext, work, rb, status);
  return hipGetLastError();
}

}  // namespace trals
