// Internal definitions shared by the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trals {

constexpr int kMaxOrder = 16;   // N
constexpr int kMaxRank = 32;    // R_n

// Status word kept in device memory; kernels raise it, the host reads it at sync points.
// kDevIdle: the word of a guarded launch with nothing to do (its kernels skip like after an error)
enum DevStatus : int { kDevOk = 0, kDevSingular = 1, kDevIdle = 2 };

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): multipliers and Weyl key increments.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t x[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = kPhiloxM0 * x[0];
    const uint64_t hi0 = __umul64hi(kPhiloxM0, x[0]);
    const uint64_t lo1 = kPhiloxM1 * x[2];
    const uint64_t hi1 = __umul64hi(kPhiloxM1, x[2]);
    const uint64_t y0 = hi1 ^ x[1] ^ k0;
    const uint64_t y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
}

// Copies n elements src -> dst (typically global -> LDS) with each thread keeping kBatch loads
// in flight before it stores, so that a latency-bound staging pass costs one memory round trip
// per kBatch elements per thread instead of one per element.  Requires n >= 1.
template <int kBatch, typename T>
__device__ __forceinline__ void copy_batched(T* dst, const T* src, int64_t n, int tid, int nthreads) {
  for (int64_t base = 0; base < n; base += (int64_t)kBatch * nthreads) {
    T v[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int64_t e = base + tid + (int64_t)q * nthreads;
      v[q] = src[e < n ? e : n - 1];
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int64_t e = base + tid + (int64_t)q * nthreads;
      if (e < n) dst[e] = v[q];
    }
  }
}

// MI355X dispatches the workgroups of a launch to its 8 XCDs (each with its own L2) round
// robin by workgroup index.  xcd_linear_block renumbers them so that the workgroups one XCD
// runs form one contiguous range of logical indices (bijective for any grid size): work that
// shares inputs and has neighbouring logical indices then shares one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_linear_block(int b, int grid) {
  const int x = b % kXcds, k = b / kXcds;
  const int per = grid / kXcds, rem = grid % kXcds;
  return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Per-mode view of the ring passed by value to kernels.
struct Ring {
  int N;
  int dims[kMaxOrder];
  int ranks[kMaxOrder];  // bond after core n; core n is ranks[n-1] x dims[n] x ranks[n]
};

__host__ __device__ __forceinline__ int rank_before(const Ring& g, int n) {
  return g.ranks[(n + g.N - 1) % g.N];
}

// Pointers to per-mode device arrays.
template <typename T>
struct PerMode {
  T* p[kMaxOrder];
};

}  // namespace trals
