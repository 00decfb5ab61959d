// Sampled least-squares solve of one core update (Algorithm 2, LS step) by the normal
// equations in FP64: H = A^T A (P x P), B = A^T X~ (P x I_n), H = L L^T (Cholesky),
// Z = H^{-1} B, and lateral slice i of the new core is column i of Z.  The paper solves the
// same problem with a QR factorisation; the two agree up to cond(A)^2 * eps.
//
// k_chol also serves the leverage scores of a core (eq. (3)): with K = G_(2)^T G_(2) = L L^T,
// row i of G_(2) has leverage ||L^{-1} g_i||^2.
#include "kernels.h"

namespace trals {

namespace {

constexpr int kCholThreads = 1024;

// Single workgroup.  M (P x P, row-major, FP64) is factorised in place (lower triangle).
__global__ __launch_bounds__(kCholThreads) void k_chol(const double* __restrict__ parts, int nparts, int P,
                                                       double* M, double* W, int want, int* status) {
  __shared__ int s_fail;
  __shared__ double s_tol;
  if (*status != kDevOk) return;
  const int tid = threadIdx.x;
  const int64_t PP = (int64_t)P * P;
  if (nparts > 0) {
    for (int64_t e = tid; e < PP; e += kCholThreads) {
      double acc = 0.0;
      for (int s = 0; s < nparts; ++s) acc += parts[s * PP + e];
      M[e] = acc;
    }
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < P; ++i) mx = fmax(mx, M[(int64_t)i * P + i]);
    s_tol = (double)P * 2.220446049250313e-16 * mx;
    s_fail = !(mx > 0.0) || !isfinite(mx);
  }
  __syncthreads();
  if (s_fail) {
    if (tid == 0) *status = kDevSingular;
    return;
  }
  // right-looking Cholesky
  for (int k = 0; k < P; ++k) {
    if (tid == 0) {
      const double d = M[(int64_t)k * P + k];
      if (!(d > s_tol) || !isfinite(d)) s_fail = 1;
      else M[(int64_t)k * P + k] = sqrt(d);
    }
    __syncthreads();
    if (s_fail) {
      if (tid == 0) *status = kDevSingular;
      return;
    }
    const double lkk = M[(int64_t)k * P + k];
    for (int i = k + 1 + tid; i < P; i += kCholThreads) M[(int64_t)i * P + k] /= lkk;
    __syncthreads();
    const int rem = P - k - 1;
    const int64_t pairs = (int64_t)rem * (rem + 1) / 2;
    for (int64_t e = tid; e < pairs; e += kCholThreads) {
      // e -> (ii, jj) with 0 <= jj <= ii < rem
      int ii = (int)((sqrt(8.0 * (double)e + 1.0) - 1.0) * 0.5);
      while ((int64_t)ii * (ii + 1) / 2 > e) --ii;
      while ((int64_t)(ii + 1) * (ii + 2) / 2 <= e) ++ii;
      const int jj = (int)(e - (int64_t)ii * (ii + 1) / 2);
      const int i = k + 1 + ii, j = k + 1 + jj;
      M[(int64_t)i * P + j] -= M[(int64_t)i * P + k] * M[(int64_t)j * P + k];
    }
    __syncthreads();
  }
  // W = L^{-1}: column c by forward substitution, one thread per column
  for (int c = tid; c < P; c += kCholThreads) {
    for (int i = 0; i < c; ++i) W[(int64_t)i * P + c] = 0.0;
    W[(int64_t)c * P + c] = 1.0 / M[(int64_t)c * P + c];
    for (int i = c + 1; i < P; ++i) {
      double acc = 0.0;
      for (int k = c; k < i; ++k) acc += M[(int64_t)i * P + k] * W[(int64_t)k * P + c];
      W[(int64_t)i * P + c] = -acc / M[(int64_t)i * P + i];
    }
  }
  __syncthreads();
  if (want == 0) {
    // M <- W^T W = (L L^T)^{-1}
    for (int64_t e = tid; e < PP; e += kCholThreads) {
      const int i = (int)(e / P), j = (int)(e % P);
      const int k0 = i > j ? i : j;
      double acc = 0.0;
      for (int k = k0; k < P; ++k) acc += W[(int64_t)k * P + i] * W[(int64_t)k * P + j];
      M[e] = acc;
    }
  }
}

// Inverse of an SPD matrix (P <= 16 MB) by Gauss-Jordan elimination without pivoting, the
// matrix held in registers: thread (ty, tx) of a 16 x 16 grid owns entries (ty + 16a, tx + 16b).
// Each pivot step publishes row k and column k through LDS (double-buffered, one barrier).
// The pivots are the Schur-complement diagonals of the Cholesky factorisation; a pivot below
// P * eps * max(diag) marks the matrix singular.  Input: the sum of nparts partial matrices in
// a fixed order, or Min when nparts == 0.  Out may alias Min.
template <int MB>
__global__ __launch_bounds__(256) void k_spd_inv(const double* __restrict__ parts, int nparts, int P,
                                                 const double* Min, double* Out, int* status) {
  constexpr int W = 16 * MB;
  __shared__ double rowk[2][W];
  __shared__ double colk[2][W];
  __shared__ double dmax[256];
  if (*status != kDevOk) return;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t PP = (int64_t)P * P;
  double M[MB][MB];
  double dm = 0.0;
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int i = ty + 16 * a, j = tx + 16 * b;
      double v = 0.0;
      if (i < P && j < P) {
        const int64_t e = (int64_t)i * P + j;
        if (nparts > 0)
          for (int s = 0; s < nparts; ++s) v += parts[s * PP + e];
        else
          v = Min[e];
      }
      M[a][b] = v;
      if (i == j) dm = fmax(dm, v);
    }
  dmax[threadIdx.x] = dm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) dmax[threadIdx.x] = fmax(dmax[threadIdx.x], dmax[threadIdx.x + o]);
    __syncthreads();
  }
  const double tol = (double)P * 2.220446049250313e-16 * dmax[0];
  if (!(dmax[0] > 0.0) || !isfinite(dmax[0])) {
    if (threadIdx.x == 0) *status = kDevSingular;
    return;
  }
  for (int k = 0; k < P; ++k) {
    const int buf = k & 1, kb = k >> 4, kr = k & 15;
    if (ty == kr) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
        if (a == kb)
#pragma unroll
          for (int b = 0; b < MB; ++b) rowk[buf][tx + 16 * b] = M[a][b];
    }
    if (tx == kr) {
#pragma unroll
      for (int b = 0; b < MB; ++b)
        if (b == kb)
#pragma unroll
          for (int a = 0; a < MB; ++a) colk[buf][ty + 16 * a] = M[a][b];
    }
    __syncthreads();
    const double piv = rowk[buf][k];
    if (!(piv > tol) || !isfinite(piv)) {
      if (threadIdx.x == 0) *status = kDevSingular;
      return;
    }
    const double ip = 1.0 / piv;
    double rk[MB], ci[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) rk[b] = rowk[buf][tx + 16 * b] * ip;
#pragma unroll
    for (int a = 0; a < MB; ++a) ci[a] = colk[buf][ty + 16 * a];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < MB; ++b) M[a][b] -= ci[a] * rk[b];
    if (ty == kr) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
        if (a == kb)
#pragma unroll
          for (int b = 0; b < MB; ++b) M[a][b] = rk[b];
    }
    if (tx == kr) {
#pragma unroll
      for (int b = 0; b < MB; ++b)
        if (b == kb)
#pragma unroll
          for (int a = 0; a < MB; ++a) M[a][b] = -ci[a] * ip;
    }
    if (ty == kr && tx == kr) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
        if (a == kb) M[a][a] = ip;
    }
  }
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int i = ty + 16 * a, j = tx + 16 * b;
      if (i < P && j < P) Out[(int64_t)i * P + j] = M[a][b];
    }
}

// Z = Hinv * (sum_s Bpart[s]); one block per group of kCols columns.
template <typename Real, typename Acc>
__global__ __launch_bounds__(256) void k_solve(const double* __restrict__ Hinv, const Acc* __restrict__ Bpart,
                                               int nparts, int P, int In, Real* __restrict__ core,
                                               const int* status) {
  constexpr int kCols = 8;
  extern __shared__ double sB[];  // P x kCols
  if (*status != kDevOk) return;
  const int i0 = blockIdx.x * kCols;
  const int64_t PI = (int64_t)P * In;
  for (int e = threadIdx.x; e < P * kCols; e += blockDim.x) {
    const int p = e / kCols, c = e % kCols;
    const int i = i0 + c;
    double acc = 0.0;
    if (i < In)
      for (int s = 0; s < nparts; ++s) acc += (double)Bpart[s * PI + (int64_t)p * In + i];
    sB[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < P * kCols; e += blockDim.x) {
    const int c = e / P, p = e % P;  // consecutive threads: consecutive p (coalesced core write)
    const int i = i0 + c;
    if (i >= In) continue;
    const double* h = Hinv + (int64_t)p * P;
    double acc = 0.0;
    for (int k = 0; k < P; ++k) acc += h[k] * sB[k * kCols + c];
    core[(int64_t)i * P + p] = (Real)acc;
  }
}

}  // namespace

hipError_t launch_chol(const double* parts, int nparts, int P, double* M, double* W, int want, int* status,
                       hipStream_t s) {
  k_chol<<<1, kCholThreads, 0, s>>>(parts, nparts, P, M, W, want, status);
  return hipGetLastError();
}

hipError_t launch_spd_inverse(const double* parts, int nparts, int P, double* work, double* scratch, int* status,
                              hipStream_t s) {
  const int mb = (P + 15) / 16;
  switch (mb) {
#define TRALS_INV_CASE(MB) \
  case MB: k_spd_inv<MB><<<1, 256, 0, s>>>(parts, nparts, P, work, work, status); break;
    TRALS_INV_CASE(1)
    TRALS_INV_CASE(2)
    TRALS_INV_CASE(3)
    TRALS_INV_CASE(4)
    TRALS_INV_CASE(5)
    TRALS_INV_CASE(6)
    TRALS_INV_CASE(7)
    TRALS_INV_CASE(8)
    TRALS_INV_CASE(9)
#undef TRALS_INV_CASE
    default:
      // larger systems: Cholesky, triangular inverse and product in one workgroup
      k_chol<<<1, kCholThreads, 0, s>>>(parts, nparts, P, work, scratch, 0, status);
  }
  return hipGetLastError();
}

hipError_t launch_solve(const double* Hinv, const void* Bpart, int nparts, int P, int In, void* core,
                        int real_dtype, const int* status, hipStream_t s) {
  const unsigned blocks = (unsigned)((In + 7) / 8);
  const size_t lds = (size_t)P * 8 * sizeof(double);
  if (real_dtype == 0)
    k_solve<double, double><<<blocks, 256, lds, s>>>(Hinv, (const double*)Bpart, nparts, P, In, (double*)core, status);
  else if (real_dtype == 1)
    k_solve<float, double><<<blocks, 256, lds, s>>>(Hinv, (const double*)Bpart, nparts, P, In, (float*)core, status);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace trals
