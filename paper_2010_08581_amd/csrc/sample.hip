// Sampler of one core update (Algorithm 3; Definition 5 rescaling).
//
// Sample j, mode draw k (mode m = (n+1+k) mod N) takes 64-bit word (k mod 4) of the
// Philox4x64-10 block with key (seed, stream_id) and counter (j, k/4, u, 0), u the update
// number.  With the mode's inclusive integer table C (total T = C[I-1]) the draw is
// t = floor(r T / 2^64) (high word of the 128-bit product) and i = min{i : t < C_i}, found by
// binary search; zero-weight entries are never drawn.  The rescaling is w = 1/sqrt(J q) with
// q = prod_k Q_{i_k} / T_k the exact probability of the tuple, multiplied in FP64 in k order.
//
// The tables of the N-1 sampled modes are staged in LDS when they fit (kLdsTableBytes), so
// the dependent loads of the binary searches stay on chip.
#include "kernels.h"

namespace trals {

namespace {

constexpr int kThreads = 256;
constexpr size_t kLdsTableBytes = 48 * 1024;

template <bool kLds>
__global__ __launch_bounds__(kThreads) void k_sample(SampleArgs a) {
  extern __shared__ uint64_t tab[];
  if (*a.status != kDevOk) return;
  const int N = a.ring.N;
  const int K = N - 1;
  int off[kMaxOrder];
  if (kLds) {
    int o = 0;
    for (int k = 0; k < K; ++k) {
      int m = a.n + 1 + k;
      if (m >= N) m -= N;
      off[k] = o;
      const int I = a.ring.dims[m];
      for (int i = threadIdx.x; i < I; i += kThreads) tab[o + i] = a.cdf.p[m][i];
      o += I;
    }
    __syncthreads();
  }
  const int64_t j = blockIdx.x * (int64_t)kThreads + threadIdx.x;
  if (j >= a.J) return;
  uint64_t x[4] = {0, 0, 0, 0};
  double q = 1.0;
  for (int k = 0; k < K; ++k) {
    const int word = k & 3;
    if (word == 0) {
      x[0] = (uint64_t)j;
      x[1] = (uint64_t)(k >> 2);
      x[2] = a.u;
      x[3] = 0;
      philox4x64_10(x, a.seed, a.stream_id);
    }
    const uint64_t r = word == 0 ? x[0] : word == 1 ? x[1] : word == 2 ? x[2] : x[3];
    int m = a.n + 1 + k;
    if (m >= N) m -= N;
    const uint64_t* C = kLds ? tab + off[k] : a.cdf.p[m];
    const int I = a.ring.dims[m];
    const uint64_t T = C[I - 1];
    const uint64_t t = __umul64hi(r, T);
    int lo = 0, hi = I - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (C[mid] > t) hi = mid;
      else lo = mid + 1;
    }
    const uint64_t Qi = C[lo] - (lo > 0 ? C[lo - 1] : 0ull);
    q = q * ((double)Qi / (double)T);
    a.idx[j * K + k] = lo;
  }
  a.w[j] = 1.0 / sqrt((double)a.J * q);
}

}  // namespace

hipError_t launch_sample(const SampleArgs& a, hipStream_t s) {
  const int64_t blocks = (a.J + kThreads - 1) / kThreads;
  size_t bytes = 0;
  for (int k = 0; k < a.ring.N - 1; ++k) bytes += (size_t)a.ring.dims[(a.n + 1 + k) % a.ring.N] * 8;
  if (bytes <= kLdsTableBytes) k_sample<true><<<(unsigned)blocks, kThreads, bytes, s>>>(a);
  else k_sample<false><<<(unsigned)blocks, kThreads, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace trals
