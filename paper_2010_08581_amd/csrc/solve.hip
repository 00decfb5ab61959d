// Sampled least-squares solve of one core update (Algorithm 2, LS step) by the normal
// equations in FP64: with H = A^T A (P x P) and B = A^T X~ (P x I_n), Z = H^{-1} B, and lateral
// slice i of the new core is column i of Z.  The paper solves the same problem with a QR
// factorisation; the two agree up to cond(A)^2 * eps.
//
// The SPD inverse also serves the leverage scores of a core (eq. (3)): with K = G_(2)^T G_(2),
// row i of G_(2) has leverage g_i^T K^{-1} g_i.
#include "kernels.h"

namespace trals {

namespace {

constexpr int kCholThreads = 1024;

// Larger systems (P > 160): one workgroup, matrix in global memory (L2-resident).
// Right-looking Cholesky H = L L^T in place, W = L^{-1} by column forward substitution, then
// the inverse W^T W into M.
__global__ __launch_bounds__(kCholThreads) void k_chol_inv(int P, double* M, double* W, int* status) {
  __shared__ int s_fail;
  __shared__ double s_tol;
  if (*status != kDevOk) return;
  const int tid = threadIdx.x;
  const int64_t PP = (int64_t)P * P;
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
  for (int64_t e = tid; e < PP; e += kCholThreads) {
    const int i = (int)(e / P), j = (int)(e % P);
    const int k0 = i > j ? i : j;
    double acc = 0.0;
    for (int k = k0; k < P; ++k) acc += W[(int64_t)k * P + i] * W[(int64_t)k * P + j];
    M[e] = acc;
  }
}

// Inverse of an SPD matrix (P <= TG * MB) by Gauss-Jordan elimination without pivoting, the
// matrix held in registers: thread (ty, tx) of a TG x TG grid owns entries (ty + TG a, tx + TG b).
// Each pivot step publishes row k and column k through LDS (double-buffered, one barrier).
// The pivots are the Schur-complement diagonals of the Cholesky factorisation; a pivot below
// P * eps * max(diag) marks the matrix singular.  M is read and overwritten in place.
template <int TG, int MB>
__global__ __launch_bounds__(TG * TG) void k_spd_inv(int P, double* M, int* status) {
  constexpr int W = TG * MB;
  constexpr int NT = TG * TG;
  __shared__ double rowk[2][W];
  __shared__ double colk[2][W];
  __shared__ double dmax[NT];
  if (*status != kDevOk) return;
  const int tx = threadIdx.x % TG, ty = threadIdx.x / TG;
  double R[MB][MB];
  double dm = 0.0;
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int i = ty + TG * a, j = tx + TG * b;
      const double v = (i < P && j < P) ? M[(int64_t)i * P + j] : 0.0;
      R[a][b] = v;
      if (i == j) dm = fmax(dm, v);
    }
  dmax[threadIdx.x] = dm;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) dmax[threadIdx.x] = fmax(dmax[threadIdx.x], dmax[threadIdx.x + o]);
    __syncthreads();
  }
  const double tol = (double)P * 2.220446049250313e-16 * dmax[0];
  if (!(dmax[0] > 0.0) || !isfinite(dmax[0])) {
    if (threadIdx.x == 0) *status = kDevSingular;
    return;
  }
  for (int k = 0; k < P; ++k) {
    const int buf = k & 1, kb = k / TG, kr = k % TG;
    if (ty == kr) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
        if (a == kb)
#pragma unroll
          for (int b = 0; b < MB; ++b) rowk[buf][tx + TG * b] = R[a][b];
    }
    if (tx == kr) {
#pragma unroll
      for (int b = 0; b < MB; ++b)
        if (b == kb)
#pragma unroll
          for (int a = 0; a < MB; ++a) colk[buf][ty + TG * a] = R[a][b];
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
    for (int b = 0; b < MB; ++b) rk[b] = rowk[buf][tx + TG * b] * ip;
#pragma unroll
    for (int a = 0; a < MB; ++a) ci[a] = colk[buf][ty + TG * a];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < MB; ++b) R[a][b] -= ci[a] * rk[b];
    if (ty == kr) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
        if (a == kb)
#pragma unroll
          for (int b = 0; b < MB; ++b) R[a][b] = rk[b];
    }
    if (tx == kr) {
#pragma unroll
      for (int b = 0; b < MB; ++b)
        if (b == kb)
#pragma unroll
          for (int a = 0; a < MB; ++a) R[a][b] = -ci[a] * ip;
    }
    if (ty == kr && tx == kr) {
#pragma unroll
      for (int a = 0; a < MB; ++a)
        if (a == kb) R[a][a] = ip;
    }
  }
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int i = ty + TG * a, j = tx + TG * b;
      if (i < P && j < P) M[(int64_t)i * P + j] = R[a][b];
    }
}

// Z = Hinv * B; core n slice i <- Z[:, i].  One block per group of kCols columns.
template <typename Real>
__global__ __launch_bounds__(256) void k_solve(const double* __restrict__ Hinv, const double* __restrict__ B, int P,
                                               int In, Real* __restrict__ core, const int* status) {
  constexpr int kCols = 8;
  extern __shared__ double sB[];  // P x kCols
  if (*status != kDevOk) return;
  const int i0 = blockIdx.x * kCols;
  for (int e = threadIdx.x; e < P * kCols; e += blockDim.x) {
    const int p = e / kCols, c = e % kCols;
    const int i = i0 + c;
    sB[e] = i < In ? B[(int64_t)p * In + i] : 0.0;
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

hipError_t launch_spd_inverse(int P, double* M, double* scratch, int* status, hipStream_t s) {
  if (P <= 16) {
    k_spd_inv<16, 1><<<1, 256, 0, s>>>(P, M, status);
  } else if (P <= 160) {
    switch ((P + 31) / 32) {
      case 1: k_spd_inv<32, 1><<<1, 1024, 0, s>>>(P, M, status); break;
      case 2: k_spd_inv<32, 2><<<1, 1024, 0, s>>>(P, M, status); break;
      case 3: k_spd_inv<32, 3><<<1, 1024, 0, s>>>(P, M, status); break;
      case 4: k_spd_inv<32, 4><<<1, 1024, 0, s>>>(P, M, status); break;
      default: k_spd_inv<32, 5><<<1, 1024, 0, s>>>(P, M, status); break;
    }
  } else {
    k_chol_inv<<<1, kCholThreads, 0, s>>>(P, M, scratch, status);
  }
  return hipGetLastError();
}

hipError_t launch_solve(const double* Hinv, const double* B, int P, int In, void* core, int real_dtype,
                        const int* status, hipStream_t s) {
  const unsigned blocks = (unsigned)((In + 7) / 8);
  const size_t lds = (size_t)P * 8 * sizeof(double);
  if (real_dtype == 0) k_solve<double><<<blocks, 256, lds, s>>>(Hinv, B, P, In, (double*)core, status);
  else if (real_dtype == 1) k_solve<float><<<blocks, 256, lds, s>>>(Hinv, B, P, In, (float*)core, status);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace trals
