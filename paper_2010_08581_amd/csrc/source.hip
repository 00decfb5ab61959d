// Generated data source and transfer-matrix inner products.
//
// Generated source.  The data tensor is X = TR(G*) + sigma Z: a tensor ring of given "true"
// cores G* (eq. (1)) plus iid standard normal noise Z, never materialised.  The sampled fibers
// of an update (Algorithm 2, "sample X") are computed where they are needed: with T_j the
// product of the true cores' lateral slices for sample j's indices in the other modes (the
// same chain Algorithm 4 forms from the current cores), entry i of fiber j is
// trace(G*_n(:, i, :) T_j) = sum_p G*_n[i][p] T_j[p] in the column order shared by cores and
// sketch rows.  Z at C-order linear index e is the Box-Muller transform of two Philox4x64-10
// words, key (noise_seed, noise_stream), counter (e, ~0, ~0, 0).
//
// Transfer matrices.  For two rings A, B with cores of the same mode sizes,
// <TR(A), TR(B)> = trace(E_0 E_1 ... E_{N-1}) with E_n = sum_i A_n(:, i, :) (x) B_n(:, i, :), a
// (Ra_{n-1} Rb_{n-1}) x (Ra_n Rb_n) matrix (the Frobenius inner product of eq. (1) rings,
// evaluated without forming either tensor).
#include "kernels.h"

namespace trals {

namespace {

__device__ __forceinline__ double philox_normal(uint64_t e, uint64_t k0, uint64_t k1) {
  uint64_t x[4] = {e, ~0ull, ~0ull, 0ull};
  philox4x64_10(x, k0, k1);
  const double u1 = ((double)(x[0] >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
  const double u2 = (double)(x[1] >> 11) * 0x1.0p-53;          // [0, 1)
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

template <typename Tout>
__device__ __forceinline__ Tout cvt_out(double v);
template <>
__device__ __forceinline__ double cvt_out<double>(double v) { return v; }
template <>
__device__ __forceinline__ float cvt_out<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ __bf16 cvt_out<__bf16>(double v) { return (__bf16)(float)v; }

typedef double d4 __attribute__((ext_vector_type(4)));

// The fibers of 16 samples are the product F = T G^T (16 x P times P x I_n, T the samples'
// true-core chains, G the true core n's slices): one wave per 16 x 16 tile of F on
// v_mfma_f64_16x16x4 (A(s, k) in lane s + 16 k, B(k, i) in lane i + 16 k, D(s, i) in lane
// i + 16 (s % 4), register s / 4), four waves per workgroup along i (they share the T rows
// through the cache).  The operands of twelve k-steps are loaded at once, without branches (past
// P the A operand is 0), so a round costs one memory latency.  The noise term is added per entry.
constexpr int kFiberSamples = 16;
template <typename Tout>
__global__ __launch_bounds__(256) void k_fibers(FiberArgs a) {
  __shared__ int64_t s_base[kFiberSamples];
  if (*a.status != kDevOk) return;
  const int P = a.P, In = a.In, K = a.K;
  const int64_t j0 = (int64_t)blockIdx.x * kFiberSamples;
  const int ns = a.J - j0 < kFiberSamples ? (int)(a.J - j0) : kFiberSamples;
  if ((int)threadIdx.x < ns) {
    const int32_t* ij = a.idx + (j0 + threadIdx.x) * K;
    int64_t b = 0;
    for (int k = 0; k < K; ++k) b += (int64_t)ij[k] * a.lin_stride[k];
    s_base[threadIdx.x] = b;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int i0 = ((int)blockIdx.y * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * 16;
  if (i0 >= In) return;
  const int r16 = lane & 15, k4 = lane >> 4;
  // operand rows (clamped: rows past the samples or I_n are computed, not stored)
  const double* Trow = a.T + (j0 + (r16 < ns ? r16 : ns - 1)) * (int64_t)P;
  const double* Grow = a.true_core + (int64_t)(i0 + r16 < In ? i0 + r16 : In - 1) * P;
  constexpr int kSteps = 12;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int p0 = 0; p0 < P; p0 += 4 * kSteps) {
    double tv[kSteps], gv[kSteps];
#pragma unroll
    for (int q = 0; q < kSteps; ++q) {
      const int p = p0 + 4 * q + k4;
      const int pc = p < P ? p : P - 1;
      tv[q] = (p < P ? 1.0 : 0.0) * Trow[pc];
      gv[q] = Grow[pc];
    }
#pragma unroll
    for (int q = 0; q < kSteps; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[q], gv[q], acc, 0, 0, 0);
  }
  const double sigma = *a.sigma;
  Tout* out = (Tout*)a.out;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int sm = 4 * r + k4, i = i0 + r16;
    if (sm < ns && i < In) {
      const int64_t lin = s_base[sm] + (int64_t)i * a.lin_stride_n;
      const double v = acc[r] + sigma * philox_normal((uint64_t)lin, a.noise_seed, a.noise_stream);
      out[(j0 + sm) * In + i] = cvt_out<Tout>(v);
    }
  }
}

// E[(a a') x (b b')] = sum_i A(a, i, b) B(a', i, b'); A, B slice-major (I, Ra0, Ra1), (I, Rb0, Rb1).
// As a product: E is M = Ahat^T Bhat with its index pairs regrouped, where row i of Ahat is
// slice i of A flattened ((a b), Ra0 Ra1 entries) and row i of Bhat slice i of B.  One wave per
// 16 x 16 tile of M on v_mfma_f64_16x16x4 (A(r, k) in lane r + 16 k, B(k, c) in lane c + 16 k,
// D(r, c) in lane c + 16 (r % 4), register r / 4): four slices per instruction, alternate steps
// into two accumulators; the result is written to E in the regrouped order.
__global__ __launch_bounds__(256) void k_transfer(const double* __restrict__ A, const double* __restrict__ B, int I,
                                                  int Ra0, int Ra1, int Rb0, int Rb1, double* __restrict__ E,
                                                  int tiles_n, int ntiles) {
  const int lane = threadIdx.x & 63;
  const int tile = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (tile >= ntiles) return;
  const int tm = tile / tiles_n, tn = tile - tm * tiles_n;
  const int pa = Ra0 * Ra1, pb = Rb0 * Rb1;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int m = 16 * tm + r16, n = 16 * tn + r16;
  const int mc = m < pa ? m : pa - 1, nc = n < pb ? n : pb - 1;  // clamped: loads stay in bounds
  const double fm = m < pa ? 1.0 : 0.0;
  d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < I; i0 += 8) {
    const int i1 = i0 + k4, i2 = i0 + 4 + k4;
    const int i1c = i1 < I ? i1 : I - 1, i2c = i2 < I ? i2 : I - 1;
    const double a1 = (i1 < I ? fm : 0.0) * A[(int64_t)i1c * pa + mc];
    const double b1 = B[(int64_t)i1c * pb + nc];
    const double a2 = (i2 < I ? fm : 0.0) * A[(int64_t)i2c * pa + mc];
    const double b2 = B[(int64_t)i2c * pb + nc];
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2, b2, acc1, 0, 0, 0);
  }
  const int cols = Ra1 * Rb1;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int mm = 16 * tm + 4 * r + k4, nn = 16 * tn + r16;
    if (mm < pa && nn < pb) {
      const int a = mm / Ra1, b = mm - a * Ra1, a2 = nn / Rb1, b2 = nn - a2 * Rb1;
      E[(int64_t)(a * Rb0 + a2) * cols + b * Rb1 + b2] = acc0[r] + acc1[r];
    }
  }
}

// C = A (m x k) B (k x n), row-major FP64, 16 x 16 tiles through LDS
__global__ __launch_bounds__(256) void k_gemm(const double* __restrict__ A, const double* __restrict__ B, int m, int k,
                                              int n, double* __restrict__ C) {
  __shared__ double sa[16][17], sb[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < k; k0 += 16) {
    sa[ty][tx] = (row < m && k0 + tx < k) ? A[(int64_t)row * k + k0 + tx] : 0.0;
    sb[ty][tx] = (k0 + ty < k && col < n) ? B[(int64_t)(k0 + ty) * n + col] : 0.0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) acc = fma(sa[ty][q], sb[q][tx], acc);
    __syncthreads();
  }
  if (row < m && col < n) C[(int64_t)row * n + col] = acc;
}

// out[0] = trace of the m x m matrix M (fixed-order reduction)
__global__ __launch_bounds__(256) void k_trace(const double* __restrict__ M, int m, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) s += M[(int64_t)i * m + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// sigma = noise_rel sqrt(<G*, G*> / prod I); a zero or non-finite norm marks the source unusable
__global__ void k_source_scale(const double* t2, double noise_rel, double entries, double* sigma, int* status) {
  if (*status != kDevOk) return;
  const double x = *t2;
  if (!(x > 0.0) || !isfinite(x)) {
    *status = kDevSingular;
    return;
  }
  *sigma = noise_rel * sqrt(x / entries);
}

// fit = sqrt(max(0, <G,G> - 2 <G,G*> + <G*,G*>) / <G*,G*>), r = {<G,G>, <G,G*>, <G*,G*>}
__global__ void k_clean_fit(const double* r, double* fit) {
  const double d2 = r[0] - 2.0 * r[1] + r[2];
  *fit = sqrt((d2 > 0.0 ? d2 : 0.0) / r[2]);
}

// fit = sqrt(r2 / x2) for the residual sum r2 of a full pass
__global__ void k_dense_fit(const double* r2, double x2, double* fit) { *fit = sqrt(*r2 / x2); }
__global__ void k_dense_fit_dev(const double* r2, const double* x2, double* fit) { *fit = sqrt(*r2 / *x2); }

}  // namespace

hipError_t launch_source_scale(const double* t2, double noise_rel, double entries, double* sigma, int* status,
                               hipStream_t s) {
  k_source_scale<<<1, 1, 0, s>>>(t2, noise_rel, entries, sigma, status);
  return hipGetLastError();
}

hipError_t launch_clean_fit(const double* r, double* fit, hipStream_t s) {
  k_clean_fit<<<1, 1, 0, s>>>(r, fit);
  return hipGetLastError();
}

hipError_t launch_dense_fit(const double* r2, double x2, double* fit, hipStream_t s) {
  k_dense_fit<<<1, 1, 0, s>>>(r2, x2, fit);
  return hipGetLastError();
}

hipError_t launch_dense_fit_dev(const double* r2, const double* x2, double* fit, hipStream_t s) {
  k_dense_fit_dev<<<1, 1, 0, s>>>(r2, x2, fit);
  return hipGetLastError();
}

hipError_t launch_fibers(const FiberArgs& a, int out_dtype, hipStream_t s) {
  if (a.J < 1 || a.P < 1 || a.In < 1) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((a.J + kFiberSamples - 1) / kFiberSamples), (unsigned)((a.In + 63) / 64));
  if (out_dtype == 0) k_fibers<double><<<grid, 256, 0, s>>>(a);
  else if (out_dtype == 1) k_fibers<float><<<grid, 256, 0, s>>>(a);
  else if (out_dtype == 2) k_fibers<__bf16><<<grid, 256, 0, s>>>(a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

size_t ring_inner_doubles(const Ring& ra, const Ring& rb) {
  // two chain buffers + one transfer matrix, each at most max_n (Ra Rb)^2
  size_t m = 0;
  for (int n = 0; n < ra.N; ++n) {
    const size_t d = (size_t)ra.ranks[n] * rb.ranks[n];
    m = d * d > m ? d * d : m;
  }
  return 3 * m + 8;
}

hipError_t launch_ring_inner(const Ring& ra, PerMode<const double> A, const Ring& rb, PerMode<const double> B,
                             double* work, double* out, hipStream_t s) {
  const int N = ra.N;
  size_t m = 0;
  for (int n = 0; n < N; ++n) {
    const size_t d = (size_t)ra.ranks[n] * rb.ranks[n];
    m = d * d > m ? d * d : m;
  }
  double* E = work;
  double* C0 = work + m;
  double* C1 = work + 2 * m;
  double* cur = nullptr;
  int cur_rows = 0, cur_cols = 0;
  for (int n = 0; n < N; ++n) {
    const int Ra0 = rank_before(ra, n), Ra1 = ra.ranks[n], Rb0 = rank_before(rb, n), Rb1 = rb.ranks[n];
    const int rows = Ra0 * Rb0, cols = Ra1 * Rb1;
    double* dst = n == 0 ? C0 : E;
    const int tiles_n = (Rb0 * Rb1 + 15) / 16, ntiles = (Ra0 * Ra1 + 15) / 16 * tiles_n;
    k_transfer<<<(unsigned)((ntiles + 3) / 4), 256, 0, s>>>(A.p[n], B.p[n], ra.dims[n], Ra0, Ra1, Rb0, Rb1, dst,
                                                             tiles_n, ntiles);
    if (n == 0) {
      cur = C0;
      cur_rows = rows;
      cur_cols = cols;
    } else {
      double* nxt = cur == C0 ? C1 : C0;
      dim3 grid((unsigned)((cols + 15) / 16), (unsigned)((cur_rows + 15) / 16));
      k_gemm<<<grid, 256, 0, s>>>(cur, E, cur_rows, cur_cols, cols, nxt);
      cur = nxt;
      cur_cols = cols;
    }
  }
  k_trace<<<1, 256, 0, s>>>(cur, cur_rows, out);
  return hipGetLastError();
}

}  // namespace trals
