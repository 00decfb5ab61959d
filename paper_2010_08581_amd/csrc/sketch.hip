// Sketched design matrix of one core update (Algorithm 4, eq. (5)).
//
// Row j of the sketch is the product of the sampled lateral slices
// G^(m_0)(:, i_{m_0}, :) ... G^(m_{N-2})(:, i_{m_{N-2}}, :) (an R_n x R_{n-1} matrix M_j) times
// w_j, stored with column a*R_n + b holding w_j M_j(b, a).  (This column order is a
// permutation of the paper's a + R_{n-1} b; it makes the solution columns the lateral slices
// of the new core in slice-major storage.)
#include "kernels.h"

namespace trals {

namespace {

// One thread per (sample j, row b of M_j); the running row stays in registers.
template <typename Real, int RM>
__global__ __launch_bounds__(256) void k_sketch(SketchArgs a) {
  if (*a.status != kDevOk) return;
  const int N = a.ring.N;
  const int K = N - 1;
  const int n = a.n;
  const int Rn = a.ring.ranks[n];
  const int Rp = rank_before(a.ring, n);
  const int P = Rn * Rp;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t j = t / Rn;
  const int b = (int)(t % Rn);
  if (j >= a.J) return;
  const int32_t* ij = a.idx + j * K;
  Real row[RM];
  int m = (n + 1) % N;
  int cols = a.ring.ranks[m];
  {
    const Real* S = (const Real*)a.cores.p[m] + ((int64_t)ij[0] * Rn + b) * cols;
#pragma unroll
    for (int c = 0; c < RM; ++c) row[c] = c < cols ? S[c] : Real(0);
  }
  for (int k = 1; k < K; ++k) {
    m = m + 1 == N ? 0 : m + 1;
    const int rin = cols;
    const int rout = a.ring.ranks[m];
    const Real* S = (const Real*)a.cores.p[m] + (int64_t)ij[k] * rin * rout;
    Real nr[RM];
#pragma unroll
    for (int co = 0; co < RM; ++co) nr[co] = Real(0);
#pragma unroll
    for (int ci = 0; ci < RM; ++ci) {
      if (ci < rin) {
        const Real v = row[ci];
#pragma unroll
        for (int co = 0; co < RM; ++co)
          if (co < rout) nr[co] += v * S[ci * rout + co];
      }
    }
#pragma unroll
    for (int c = 0; c < RM; ++c) row[c] = nr[c];
    cols = rout;
  }
  const Real wj = (Real)a.w[j];
  Real* Aj = (Real*)a.A + j * P;
#pragma unroll
  for (int c = 0; c < RM; ++c)
    if (c < Rp) Aj[c * Rn + b] = wj * row[c];
}

template <typename Real>
hipError_t sketch_dispatch(const SketchArgs& a, hipStream_t s) {
  int rmax = 0;
  for (int m = 0; m < a.ring.N; ++m) rmax = a.ring.ranks[m] > rmax ? a.ring.ranks[m] : rmax;
  const int Rn = a.ring.ranks[a.n];
  const int64_t threads = a.J * Rn;
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  if (rmax <= 4) k_sketch<Real, 4><<<blocks, 256, 0, s>>>(a);
  else if (rmax <= 8) k_sketch<Real, 8><<<blocks, 256, 0, s>>>(a);
  else if (rmax <= 16) k_sketch<Real, 16><<<blocks, 256, 0, s>>>(a);
  else if (rmax <= 32) k_sketch<Real, 32><<<blocks, 256, 0, s>>>(a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sketch(const SketchArgs& a, int real_dtype, hipStream_t s) {
  if (real_dtype == 0) return sketch_dispatch<double>(a, s);
  if (real_dtype == 1) return sketch_dispatch<float>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace trals
