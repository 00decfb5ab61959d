// Leverage-score sampling table of one core (eq. (3), Definition 4).
//
// G_(2) is I_n x P (P = R_{n-1} R_n); in slice-major storage its row i is lateral slice i.
//  * I_n > P: the Gram K = G_(2)^T G_(2) (normal-equation kernel, Gram-only form) is
//    Cholesky-factored in FP64, K = L L^T, and l_i = ||L^{-1} g_i||^2, the squared norm of row
//    i of the orthonormal factor G_(2) L^{-T}; p_i = l_i / P (chol.hip writes the weights).  A
//    non-positive pivot of K means rank(G_(2)) < P and is reported as singular.
//  * I_n <= P: the unfolding is taken to have full row rank, so every row of its left singular
//    factor is a unit vector and p_i = 1 / I_n exactly.
// Integer weights Q_i = floor(p_i * 2^52) (exact power-of-two scaling of an FP64 value), then
// the inclusive prefix sum C in place; T = C[I_n - 1].
#include "kernels.h"

namespace trals {

namespace {

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

// After a table formed beside the next update: if its factorisation broke down (*fail set),
// the table Qalt replaces Q, and *redo = kDevOk lets the launches guarded by it repeat the next
// update's draws and contraction; otherwise *redo = kDevIdle and they skip.
__global__ __launch_bounds__(1024) void k_table_settle(const int* fail, const int* status, const uint64_t* Qalt,
                                                       uint64_t* Q, int In, int* redo) {
  const bool take = *status == kDevOk && *fail != 0;
  if (take)
    for (int i = threadIdx.x; i < In; i += 1024) Q[i] = Qalt[i];
  if (threadIdx.x == 0) *redo = take ? kDevOk : kDevIdle;
}

}  // namespace

hipError_t launch_table_settle(const int* fail, const int* status, const uint64_t* Qalt, uint64_t* Q, int In, int* redo,
                               hipStream_t s) {
  k_table_settle<<<1, 1024, 0, s>>>(fail, status, Qalt, Q, In, redo);
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
