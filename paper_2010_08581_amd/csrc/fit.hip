// Relative fit error ||TR(G) - X||_F / ||X||_F (Section 4.1) over every entry of X.
//
// X in C order is a (prod_{k<N-1} I_k) x I_{N-1} matrix.  For row r = (i_0..i_{N-2}) the left
// chain L = G^(0)(:, i_0, :) ... G^(N-2)(:, i_{N-2}, :) is R_{N-1} x R_{N-2}, and by eq. (1)
// X^(r, i) = trace(L G^(N-1)(:, i, :)) = sum_{a,b} L(a, b) G^(N-1)(b, i, a).  Squared residuals
// are accumulated in FP64 per block and summed in a fixed order.
#include "kernels.h"

namespace trals {

namespace {

constexpr int kRows = kFitRows;

template <typename Real, typename Tx, int RM>
__global__ __launch_bounds__(256) void k_fit(FitArgs a) {
  extern __shared__ unsigned char smem[];
  Real* Lt = (Real*)smem;  // kRows x P_last, column b * R_{N-1} + a
  __shared__ double red[256];
  const int N = a.ring.N;
  const int Rl = a.ring.ranks[N - 1];  // R_{N-1}: rows of L
  const int Rm = a.ring.ranks[N - 2 >= 0 ? N - 2 : 0];
  const int Pl = Rl * Rm;
  const int Il = a.ring.dims[N - 1];
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  // left chains: thread (rr, row a of L)
  for (int t = threadIdx.x; t < kRows * Rl; t += blockDim.x) {
    const int rr = t / Rl, arow = t % Rl;
    const int64_t r = r0 + rr;
    if (r >= a.rows) continue;
    int ii[kMaxOrder];
    int64_t rem = r;
    for (int k = N - 2; k >= 0; --k) {
      ii[k] = (int)(rem % a.ring.dims[k]);
      rem /= a.ring.dims[k];
    }
    Real row[RM];
    int cols = a.ring.ranks[0];
    {
      const Real* S = (const Real*)a.cores.p[0] + ((int64_t)ii[0] * Rl + arow) * cols;
#pragma unroll
      for (int c = 0; c < RM; ++c) row[c] = c < cols ? S[c] : Real(0);
    }
    for (int k = 1; k <= N - 2; ++k) {
      const int rin = cols, rout = a.ring.ranks[k];
      const Real* S = (const Real*)a.cores.p[k] + (int64_t)ii[k] * rin * rout;
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
#pragma unroll
    for (int b = 0; b < RM; ++b)
      if (b < Rm) Lt[rr * Pl + b * Rl + arow] = row[b];
  }
  __syncthreads();
  const Real* SL = (const Real*)a.cores.p[N - 1];
  const Tx* X = (const Tx*)a.X;
  double acc = 0.0;
  for (int e = threadIdx.x; e < kRows * Il; e += blockDim.x) {
    const int rr = e / Il, i = e % Il;
    const int64_t r = r0 + rr;
    if (r >= a.rows) continue;
    const Real* s = SL + (int64_t)i * Pl;
    const Real* l = Lt + rr * Pl;
    double xh = 0.0;
    for (int k = 0; k < Pl; ++k) xh += (double)l[k] * (double)s[k];
    const double d = xh - (double)X[r * Il + i];
    acc += d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[blockIdx.x] = red[0];
}

// Sampled squared residual (Section 3.1, estimate of the error from sampled entries): sample s
// takes word 0 of the Philox4x64-10 block with key (seed, stream_id) and counter (s, tag, 0, 1);
// its C-order linear index is t = floor(r E / 2^64).  Rl = R_{N-1} threads per sample: thread
// a carries row a of the slice chain G^(0)(:, i_0, :) ... G^(N-2)(:, i_{N-2}, :) and forms
// sum_b L(a, b) G^(N-1)(b, i_{N-1}, a); the entry TR(G)(i) is the sum over a (in order).  Each
// block sums (entry - X(t))^2 over its samples (fixed assignment and order) into partial[block].
template <typename Tx, int RM>
__global__ __launch_bounds__(256) void k_fit_sample(FitSampleArgs a) {
  __shared__ double s_v[256];
  __shared__ double red[256];
  const int N = a.ring.N;
  const int Rl = a.ring.ranks[N - 1];
  const int Rm = a.ring.ranks[N - 2 >= 0 ? N - 2 : 0];
  const int per = 256 / Rl;  // samples per round of the block
  const int tid = threadIdx.x, sl = tid / Rl, arow = tid - sl * Rl;
  const double* SL = (const double*)a.cores.p[N - 1];
  const Tx* X = (const Tx*)a.X;
  double acc = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * per; base < a.S; base += (int64_t)gridDim.x * per) {
    const int64_t s = base + sl;
    const bool live = sl < per && s < a.S;
    double v = 0.0;
    int64_t lin = 0;
    if (live) {
      uint64_t x[4] = {(uint64_t)s, a.tag, 0ull, 1ull};
      philox4x64_10(x, a.seed, a.stream_id);
      lin = (int64_t)__umul64hi(x[0], (uint64_t)a.E);
      int ii[kMaxOrder];
      int64_t rem = lin;
      for (int k = N - 1; k >= 0; --k) {
        ii[k] = (int)(rem % a.ring.dims[k]);
        rem /= a.ring.dims[k];
      }
      double row[RM];
      int cols = a.ring.ranks[0];
      {
        const double* S0 = (const double*)a.cores.p[0] + ((int64_t)ii[0] * Rl + arow) * cols;
#pragma unroll
        for (int c = 0; c < RM; ++c) row[c] = c < cols ? S0[c] : 0.0;
      }
      for (int k = 1; k <= N - 2; ++k) {
        const int rin = cols, rout = a.ring.ranks[k];
        const double* Sk = (const double*)a.cores.p[k] + (int64_t)ii[k] * rin * rout;
        double nr[RM];
#pragma unroll
        for (int co = 0; co < RM; ++co) nr[co] = 0.0;
#pragma unroll
        for (int ci = 0; ci < RM; ++ci)
          if (ci < rin) {
#pragma unroll
            for (int co = 0; co < RM; ++co)
              if (co < rout) nr[co] += row[ci] * Sk[ci * rout + co];
          }
#pragma unroll
        for (int c = 0; c < RM; ++c) row[c] = nr[c];
        cols = rout;
      }
      const double* sN = SL + (int64_t)ii[N - 1] * Rm * Rl;
#pragma unroll
      for (int b = 0; b < RM; ++b)
        if (b < Rm) v += row[b] * sN[b * Rl + arow];
    }
    s_v[tid] = v;
    __syncthreads();
    if (live && arow == 0) {
      double e = 0.0;
      for (int r = 0; r < Rl; ++r) e += s_v[sl * Rl + r];
      const double d = e - (double)X[lin];
      acc += d * d;
    }
    __syncthreads();
  }
  red[tid] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) a.partial[blockIdx.x] = red[0];
}

template <typename Real, typename Tx>
hipError_t fit_dispatch(const FitArgs& a, int* nb, hipStream_t s) {
  int rmax = 0;
  for (int m = 0; m < a.ring.N; ++m) rmax = a.ring.ranks[m] > rmax ? a.ring.ranks[m] : rmax;
  const int N = a.ring.N;
  const int Pl = a.ring.ranks[N - 1] * a.ring.ranks[N - 2];
  const unsigned blocks = (unsigned)((a.rows + kRows - 1) / kRows);
  const size_t lds = (size_t)kRows * Pl * sizeof(Real);
  *nb = (int)blocks;
  if (rmax <= 4) k_fit<Real, Tx, 4><<<blocks, 256, lds, s>>>(a);
  else if (rmax <= 8) k_fit<Real, Tx, 8><<<blocks, 256, lds, s>>>(a);
  else if (rmax <= 16) k_fit<Real, Tx, 16><<<blocks, 256, lds, s>>>(a);
  else if (rmax <= 32) k_fit<Real, Tx, 32><<<blocks, 256, lds, s>>>(a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fit_sample(const FitSampleArgs& a, int x_dtype, int* nblocks_out, hipStream_t s) {
  int rmax = 0;
  for (int m = 0; m < a.ring.N; ++m) rmax = a.ring.ranks[m] > rmax ? a.ring.ranks[m] : rmax;
  if (a.S < 1 || a.ring.N < 2) return hipErrorInvalidValue;
  const int per = 256 / a.ring.ranks[a.ring.N - 1];
  const int64_t need = (a.S + per - 1) / per;
  const unsigned blocks = (unsigned)(need < kFitSampleBlocks ? need : kFitSampleBlocks);
  *nblocks_out = (int)blocks;
#define TRALS_FS(TX)                                                                            \
  if (rmax <= 4) k_fit_sample<TX, 4><<<blocks, 256, 0, s>>>(a);                                 \
  else if (rmax <= 8) k_fit_sample<TX, 8><<<blocks, 256, 0, s>>>(a);                            \
  else if (rmax <= 16) k_fit_sample<TX, 16><<<blocks, 256, 0, s>>>(a);                          \
  else if (rmax <= 32) k_fit_sample<TX, 32><<<blocks, 256, 0, s>>>(a);                          \
  else return hipErrorInvalidValue;
  if (x_dtype == 0) {
    TRALS_FS(double)
  } else if (x_dtype == 1) {
    TRALS_FS(float)
  } else {
    return hipErrorInvalidValue;
  }
#undef TRALS_FS
  return hipGetLastError();
}

hipError_t launch_fit(const FitArgs& a, int real_dtype, int x_dtype, int* nblocks_out, hipStream_t s) {
  if (real_dtype == 0 && x_dtype == 0) return fit_dispatch<double, double>(a, nblocks_out, s);
  if (real_dtype == 1 && x_dtype == 1) return fit_dispatch<float, float>(a, nblocks_out, s);
  if (real_dtype == 1 && x_dtype == 0) return fit_dispatch<float, double>(a, nblocks_out, s);
  if (real_dtype == 0 && x_dtype == 1) return fit_dispatch<double, float>(a, nblocks_out, s);
  return hipErrorInvalidValue;
}

}  // namespace trals
