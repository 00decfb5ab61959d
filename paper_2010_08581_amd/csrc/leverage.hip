// Leverage-score sampling table of one core (eq. (3), Definition 4).
//
// G_(2) is I_n x P (P = R_{n-1} R_n); in slice-major storage its row i is lateral slice i.
//  * I_n > P: K = G_(2)^T G_(2) in FP64 and l_i = g_i^T K^{-1} g_i, which equals the squared
//    norm of row i of the orthonormal factor G_(2) L^{-T} (K = L L^T), p_i = l_i / P.  A
//    non-positive pivot of K means rank(G_(2)) < P and is reported as singular.
//  * I_n <= P: the unfolding is taken to have full row rank, so every row of its left singular
//    factor is a unit vector and p_i = 1 / I_n exactly.
// Integer weights Q_i = floor(p_i * 2^52) (exact power-of-two scaling of an FP64 value), then
// the inclusive prefix sum C in place; T = C[I_n - 1].
#include "kernels.h"

namespace trals {

namespace {

constexpr int kT = 32;

template <typename Real>
__global__ __launch_bounds__(256) void k_lev_gram(const Real* __restrict__ G, int In, int P, double* K,
                                                  const int* status) {
  if (*status != kDevOk) return;
  __shared__ double As[kT][kT + 1];
  __shared__ double Bs[kT][kT + 1];
  const int p0 = blockIdx.x * kT, q0 = blockIdx.y * kT;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[2][2] = {{0, 0}, {0, 0}};
  for (int rb = 0; rb < In; rb += kT) {
    for (int e = threadIdx.x; e < kT * kT; e += 256) {
      const int r = e / kT, c = e % kT;
      const int row = rb + r;
      As[r][c] = (row < In && p0 + c < P) ? (double)G[(int64_t)row * P + p0 + c] : 0.0;
      Bs[r][c] = (row < In && q0 + c < P) ? (double)G[(int64_t)row * P + q0 + c] : 0.0;
    }
    __syncthreads();
    for (int r = 0; r < kT; ++r) {
      const double a0 = As[r][ty * 2], a1 = As[r][ty * 2 + 1];
      const double b0 = Bs[r][tx * 2], b1 = Bs[r][tx * 2 + 1];
      acc[0][0] += a0 * b0;
      acc[0][1] += a0 * b1;
      acc[1][0] += a1 * b0;
      acc[1][1] += a1 * b1;
    }
    __syncthreads();
  }
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const int p = p0 + ty * 2 + u, q = q0 + tx * 2 + v;
      if (p < P && q < P) K[(int64_t)p * P + q] = acc[u][v];
    }
}

// One block per row i: l_i = g_i^T K^{-1} g_i (= ||L^{-1} g_i||^2 for K = L L^T).
template <typename Real>
__global__ __launch_bounds__(256) void k_lev_rows(const Real* __restrict__ G, int In, int P,
                                                  const double* __restrict__ Kinv, uint64_t* Q,
                                                  const int* status) {
  extern __shared__ double sg[];
  __shared__ double red[256];
  if (*status != kDevOk) return;
  const int i = blockIdx.x;
  for (int k = threadIdx.x; k < P; k += blockDim.x) sg[k] = (double)G[(int64_t)i * P + k];
  __syncthreads();
  double part = 0.0;
  for (int c = threadIdx.x; c < P; c += blockDim.x) {
    const double* l = Kinv + (int64_t)c * P;
    double y = 0.0;
    for (int k = 0; k < P; ++k) y += l[k] * sg[k];
    part += sg[c] * y;
  }
  red[threadIdx.x] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ell = 0.0;
    for (int t = 0; t < (int)blockDim.x; ++t) ell += red[t];
    const double p = ell / (double)P;
    Q[i] = (uint64_t)floor(p * 4503599627370496.0);  // 2^52
  }
}

__global__ void k_lev_uniform(int In, uint64_t* Q, const int* status) {
  if (*status != kDevOk) return;
  const double p = 1.0 / (double)In;
  const uint64_t q = (uint64_t)floor(p * 4503599627370496.0);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < In; i += gridDim.x * blockDim.x) Q[i] = q;
}

// In-place inclusive prefix sum of In uint64 values by one block.
__global__ __launch_bounds__(1024) void k_scan_u64(uint64_t* Q, int In, const int* status) {
  __shared__ uint64_t part[1024];
  if (*status != kDevOk) return;
  const int tid = threadIdx.x;
  const int per = (In + 1023) / 1024;
  const int b = tid * per;
  const int e = b + per < In ? b + per : In;
  uint64_t s = 0;
  for (int i = b; i < e; ++i) s += Q[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint64_t v = tid >= off ? part[tid - off] : 0ull;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint64_t run = tid > 0 ? part[tid - 1] : 0ull;
  for (int i = b; i < e; ++i) {
    run += Q[i];
    Q[i] = run;
  }
}

}  // namespace

hipError_t launch_lev_gram(const void* core, int real_dtype, int In, int P, double* K, const int* status,
                           hipStream_t s) {
  const int tp = (P + kT - 1) / kT;
  dim3 grid(tp, tp);
  if (real_dtype == 0) k_lev_gram<double><<<grid, 256, 0, s>>>((const double*)core, In, P, K, status);
  else if (real_dtype == 1) k_lev_gram<float><<<grid, 256, 0, s>>>((const float*)core, In, P, K, status);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_lev_rows(const void* core, int real_dtype, int In, int P, const double* Linv, uint64_t* Q,
                           const int* status, hipStream_t s) {
  const size_t lds = (size_t)P * sizeof(double);
  if (real_dtype == 0) k_lev_rows<double><<<In, 256, lds, s>>>((const double*)core, In, P, Linv, Q, status);
  else if (real_dtype == 1) k_lev_rows<float><<<In, 256, lds, s>>>((const float*)core, In, P, Linv, Q, status);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_lev_uniform(int In, uint64_t* Q, const int* status, hipStream_t s) {
  k_lev_uniform<<<(In + 255) / 256, 256, 0, s>>>(In, Q, status);
  return hipGetLastError();
}

hipError_t launch_scan_u64(uint64_t* Q, int In, const int* status, hipStream_t s) {
  k_scan_u64<<<1, 1024, 0, s>>>(Q, In, status);
  return hipGetLastError();
}

}  // namespace trals
