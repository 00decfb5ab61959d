// One-time passes at handle creation: data panels, norm / NaN scan, core import/export and
// the N(0,1) initial cores (Section 3 draws each initial core entry from a standard normal).
#include <hip/hip_bf16.h>

#include "kernels.h"

namespace trals {

namespace {

template <typename T>
__device__ __forceinline__ double to_f64(T v) {
  return static_cast<double>(v);
}
template <typename T>
__device__ __forceinline__ T from_f64(double v) {
  return static_cast<T>(v);
}
template <>
__device__ __forceinline__ __hip_bfloat16 from_f64<__hip_bfloat16>(double v) {
  return __float2bfloat16(static_cast<float>(v));
}

constexpr int kTile = 32;

// Batched 2-D transpose through LDS: for every a, (I_n x B) -> (B x I_n).
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_panel(const Tin* __restrict__ X, Tout* __restrict__ P, int64_t A,
                                               int64_t In, int64_t B, int64_t tiles_i, int64_t tiles_b) {
  __shared__ double tile[kTile][kTile + 1];
  const int tx = threadIdx.x % kTile;  // 32 x 8 threads
  const int ty = threadIdx.x / kTile;
  const int64_t total = A * tiles_i * tiles_b;
  for (int64_t t0 = blockIdx.x; t0 < total; t0 += gridDim.x) {
    int64_t t = t0;
    const int64_t tb = t % tiles_b;
    t /= tiles_b;
    const int64_t ti = t % tiles_i;
    const int64_t a = t / tiles_i;
    const Tin* src = X + a * In * B;
    Tout* dst = P + a * B * In;
    // read rows i (tile y), columns b (tile x): coalesced along b
    for (int r = ty; r < kTile; r += 8) {
      const int64_t i = ti * kTile + r;
      const int64_t b = tb * kTile + tx;
      if (i < In && b < B) tile[r][tx] = to_f64(src[i * B + b]);
    }
    __syncthreads();
    // write rows b, columns i: coalesced along i
    for (int r = ty; r < kTile; r += 8) {
      const int64_t b = tb * kTile + r;
      const int64_t i = ti * kTile + tx;
      if (i < In && b < B) dst[b * In + i] = from_f64<Tout>(tile[tx][r]);
    }
    __syncthreads();
  }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_copy(const Tin* __restrict__ X, Tout* __restrict__ P, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    P[e] = from_f64<Tout>(to_f64(X[e]));
}

template <typename Tin>
__global__ __launch_bounds__(256) void k_scan_x(const Tin* __restrict__ X, int64_t n, double* partial,
                                                unsigned long long* nonfinite) {
  __shared__ double red[256];
  double acc = 0.0;
  unsigned long long bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const double v = to_f64(X[e]);
    if (!isfinite(v)) ++bad;
    else acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
  if (bad && nonfinite) atomicAdd(nonfinite, bad);
}

__global__ void k_sum_partials(const double* partial, int n, double* out) {
  // fixed-order reduction by one wave: deterministic
  __shared__ double red[64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) acc += partial[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < 64; ++i) s += red[i];
    *out = s;
  }
}

// C-order core (Rp, I, Rn) <-> slice-major (I, Rp, Rn).
template <typename Tin, typename Tout>
__global__ void k_core_import(const Tin* __restrict__ src, Tout* __restrict__ dst, int Rp, int I, int Rn) {
  const int64_t n = (int64_t)Rp * I * Rn;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = e % Rn;
    const int64_t t = e / Rn;
    const int i = t % I;
    const int a = t / I;
    dst[((int64_t)i * Rp + a) * Rn + b] = from_f64<Tout>(to_f64(src[e]));
  }
}
template <typename Tin, typename Tout>
__global__ void k_core_export(const Tin* __restrict__ src, Tout* __restrict__ dst, int Rp, int I, int Rn) {
  const int64_t n = (int64_t)Rp * I * Rn;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = e % Rn;
    const int64_t t = e / Rn;
    const int i = t % I;
    const int a = t / I;
    dst[e] = from_f64<Tout>(to_f64(src[((int64_t)i * Rp + a) * Rn + b]));
  }
}

// N(0,1) by the Box-Muller transform of two Philox words; counter (e, core, ~0, 0).
template <typename Tout>
__global__ void k_core_normal(Tout* dst, int64_t count, uint64_t seed, uint64_t sid, int core) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t x[4] = {(uint64_t)e, (uint64_t)core, ~0ull, 0ull};
    philox4x64_10(x, seed, sid);
    const double u1 = ((double)(x[0] >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
    const double u2 = (double)(x[1] >> 11) * 0x1.0p-53;          // [0, 1)
    dst[e] = from_f64<Tout>(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  }
}

int grid_for(int64_t n, int per = 256, int cap = 65536) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

}  // namespace

#define TRALS_DISPATCH2(DT_IN, DT_OUT, LAUNCH)                                              \
  do {                                                                                      \
    if (DT_IN == 0 && DT_OUT == 0) { using Tin = double; using Tout = double; LAUNCH; }     \
    else if (DT_IN == 0 && DT_OUT == 1) { using Tin = double; using Tout = float; LAUNCH; } \
    else if (DT_IN == 1 && DT_OUT == 0) { using Tin = float; using Tout = double; LAUNCH; } \
    else if (DT_IN == 1 && DT_OUT == 1) { using Tin = float; using Tout = float; LAUNCH; }  \
    else if (DT_IN == 0 && DT_OUT == 2) { using Tin = double; using Tout = __hip_bfloat16; LAUNCH; } \
    else if (DT_IN == 1 && DT_OUT == 2) { using Tin = float; using Tout = __hip_bfloat16; LAUNCH; }  \
    else return hipErrorInvalidValue;                                                       \
  } while (0)

hipError_t launch_panel(const void* X, int x_dtype, void* panel, int p_dtype, int64_t A, int64_t In, int64_t B,
                        hipStream_t s) {
  if (B == 1) {
    const int64_t n = A * In;
    TRALS_DISPATCH2(x_dtype, p_dtype,
                    (k_copy<Tin, Tout><<<grid_for(n), 256, 0, s>>>((const Tin*)X, (Tout*)panel, n)));
    return hipGetLastError();
  }
  const int64_t ti = (In + kTile - 1) / kTile, tb = (B + kTile - 1) / kTile;
  const int64_t tiles = A * ti * tb;
  const unsigned grid = (unsigned)(tiles < (1 << 20) ? tiles : (1 << 20));
  TRALS_DISPATCH2(x_dtype, p_dtype,
                  (k_panel<Tin, Tout><<<grid, 256, 0, s>>>((const Tin*)X, (Tout*)panel, A, In, B, ti, tb)));
  return hipGetLastError();
}

hipError_t launch_scan_x(const void* X, int x_dtype, int64_t n, double* partial, int nblocks,
                         unsigned long long* nonfinite, hipStream_t s) {
  if (x_dtype == 0) k_scan_x<double><<<nblocks, 256, 0, s>>>((const double*)X, n, partial, nonfinite);
  else if (x_dtype == 1) k_scan_x<float><<<nblocks, 256, 0, s>>>((const float*)X, n, partial, nonfinite);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* partial, int n, double* out, hipStream_t s) {
  k_sum_partials<<<1, 64, 0, s>>>(partial, n, out);
  return hipGetLastError();
}

hipError_t launch_core_import(const void* src, int src_dtype, void* dst, int dst_dtype, int Rp, int I, int Rn,
                              hipStream_t s) {
  const int64_t n = (int64_t)Rp * I * Rn;
  TRALS_DISPATCH2(src_dtype, dst_dtype,
                  (k_core_import<Tin, Tout><<<grid_for(n), 256, 0, s>>>((const Tin*)src, (Tout*)dst, Rp, I, Rn)));
  return hipGetLastError();
}

hipError_t launch_core_export(const void* src, int src_dtype, void* dst, int dst_dtype, int Rp, int I, int Rn,
                              hipStream_t s) {
  const int64_t n = (int64_t)Rp * I * Rn;
  TRALS_DISPATCH2(src_dtype, dst_dtype,
                  (k_core_export<Tin, Tout><<<grid_for(n), 256, 0, s>>>((const Tin*)src, (Tout*)dst, Rp, I, Rn)));
  return hipGetLastError();
}

hipError_t launch_core_normal(void* dst, int dst_dtype, int64_t count, uint64_t seed, uint64_t stream_id, int core,
                              hipStream_t s) {
  if (dst_dtype == 0) k_core_normal<double><<<grid_for(count), 256, 0, s>>>((double*)dst, count, seed, stream_id, core);
  else if (dst_dtype == 1) k_core_normal<float><<<grid_for(count), 256, 0, s>>>((float*)dst, count, seed, stream_id, core);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace trals
