// Blocked FP64 Cholesky factorisation and triangular solves on matrix cores, for the sampled
// least-squares solve (Algorithm 2, LS step: H Z = B with H = A^T A, B = A^T X~) and for the
// leverage scores of a core (eq. (3): with K = G_(2)^T G_(2) = L L^T, row i of G_(2) has
// leverage ||L^{-1} g_i||^2).  The paper solves the LS problem by QR; the normal equations
// agree with it up to cond(A)^2 * eps.
//
// Matrices are split into 16 x 16 blocks (P padded to 16 nblk with an identity block tail).
// The lower-triangular factor is stored block-packed: block (i, j), i >= j, at slot
// i (i + 1) / 2 + j, each block 16 rows of kLd doubles.  Diagonal blocks of L^{-1} are kept
// beside it so that every triangular solve is a chain of 16 x 16 x 16 products.
//
// v_mfma_f64_16x16x4 layouts (one wave): A(i, k) in lane i + 16 k, B(k, j) in lane j + 16 k,
// D(i, j) in lane j + 16 (i % 4), register i / 4.  Register r of an accumulator therefore holds
// exactly the B operand of k-step r of a following product.
#include "kernels.h"

namespace trals {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kLd = 17;             // padded row stride of a 16 x 16 block (doubles)
constexpr int kBlk = 16 * kLd;      // doubles per stored block
constexpr int kLdsBlocks = 9;       // nblk up to which the factor lives in LDS (45 blocks)

__device__ __forceinline__ int slot(int i, int j) { return i * (i + 1) / 2 + j; }

// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps y <- y (3 - x y^2) / 2
// (each step squares the relative error), instead of the longer correctly-rounded sqrt and
// division sequences on the pivot chain of the factorisation.
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}


// acc += A * B^T for 16 x 16 blocks A, B (row-major, stride kLd); sign folds a subtraction.
template <typename PA, typename PB>
__device__ __forceinline__ d4 mma_abt(PA A, PB B, d4 acc, int lane, double sign) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int r = lane & 15, k = 4 * ks + (lane >> 4);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(sign * A[r * kLd + k], B[r * kLd + k], acc, 0, 0, 0);
  }
  return acc;
}

template <typename Ptr>
__device__ __forceinline__ d4 load_acc(Ptr C, int lane) {
  d4 v;
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = C[(4 * r + (lane >> 4)) * kLd + (lane & 15)];
  return v;
}

template <typename Ptr>
__device__ __forceinline__ void store_acc(Ptr C, d4 v, int lane) {
#pragma unroll
  for (int r = 0; r < 4; ++r) C[(4 * r + (lane >> 4)) * kLd + (lane & 15)] = v[r];
}

// One workgroup of 256 threads.  Input: H (P x P, row-major, full symmetric) in global memory.
// Output: Lp (packed blocks of L) and Dinv (nblk blocks of L_KK^{-1}) in global memory.
template <bool kInLds>
__global__ __launch_bounds__(256) void k_chol_blocked(int P, const double* __restrict__ H, double* Lp,
                                                      double* Dinv, int* status) {
  extern __shared__ double lds[];
  __shared__ int s_fail;
  __shared__ double s_tol;
  __shared__ double s_dinv[kBlk];
  __shared__ double s_col[2][16];
  __shared__ double s_lkk[kBlk];
  if (*status != kDevOk) return;
  const int nblk = (P + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* Ls = kInLds ? lds : Lp;
  // load the lower blocks (identity on the padded diagonal)
  const int nslots = nblk * (nblk + 1) / 2;
  {
    // thread (r, c) of a 16 x 16 grid loads element (r, c) of every lower block
    const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    for (int bi = 0; bi < nblk; ++bi) {
      const int i = 16 * bi + r;
#pragma unroll 4
      for (int bj = 0; bj <= bi; ++bj) {
        const int j = 16 * bj + c;
        double v = 0.0;
        if (i < P && j < P) v = H[(int64_t)i * P + j];
        else if (i == j) v = 1.0;
        Ls[slot(bi, bj) * kBlk + r * kLd + c] = v;
      }
    }
  }
  __syncthreads();
  // largest diagonal entry (from the staged blocks; wave 0, one diagonal element per lane)
  if (wave == 0) {
    double mx = 0.0;
    for (int i = lane; i < P; i += 64) mx = fmax(mx, Ls[slot(i >> 4, i >> 4) * kBlk + (i & 15) * kLd + (i & 15)]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (lane == 0) {
      s_tol = (double)P * 2.220446049250313e-16 * mx;
      s_fail = !(mx > 0.0) || !isfinite(mx);
    }
  }
  __syncthreads();
  if (s_fail) {
    if (threadIdx.x == 0) *status = kDevSingular;
    return;
  }
  for (int K = 0; K < nblk; ++K) {
    double* DK = Ls + slot(K, K) * kBlk;
    // (a) wave 0: factor the diagonal block (lane l < 16 holds row l) and invert it
    if (wave == 0) {
      // Lane l < 16 keeps row l of the block in registers.  Pivot step k publishes column k
      // (16 doubles) through LDS; every lane reads it back as broadcasts and computes the
      // pivot's reciprocal square root itself.  LDS operations of one wave complete in issue
      // order, so only the compiler needs to be kept from reordering them (empty asm barrier).
      double a[16], il[16];
      const int l = lane & 15;
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] = DK[l * kLd + c];
      bool bad = false;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (lane < 16) s_col[k & 1][l] = a[k];
        asm volatile("" ::: "memory");
        double colk[16];
#pragma unroll
        for (int j = k; j < 16; ++j) colk[j] = s_col[k & 1][j];
        const double pk = colk[k];
        if (!(pk > s_tol) || !isfinite(pk)) bad = true;
        il[k] = rsqrt_f64(fmax(pk, 1e-300));
        if (l > k) a[k] *= il[k];
        else if (l == k) a[k] = pk * il[k];
#pragma unroll
        for (int j = k + 1; j < 16; ++j)
          if (l >= j) a[j] -= a[k] * (colk[j] * il[k]);
      }
      if (lane < 16) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
          const double v = c <= l ? a[c] : 0.0;
          DK[l * kLd + c] = v;
          s_lkk[l * kLd + c] = v;
        }
      }
      if (lane == 0 && bad) s_fail = 1;
      asm volatile("" ::: "memory");
      // column l of L_KK^{-1} by forward substitution (lane l < 16), L read back from LDS as
      // broadcasts
      double x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        double acc = (i == l) ? 1.0 : 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) acc -= s_lkk[i * kLd + k] * x[k];
        x[i] = (i >= l) ? acc * il[i] : 0.0;
      }
      if (lane < 16) {
#pragma unroll
        for (int i = 0; i < 16; ++i) s_dinv[i * kLd + l] = x[i];
      }
    }
    __syncthreads();
    if (s_fail) {
      if (threadIdx.x == 0) *status = kDevSingular;
      return;
    }
    for (int e = threadIdx.x; e < 256; e += 256) Dinv[K * 256 + e] = s_dinv[(e >> 4) * kLd + (e & 15)];
    // (b) panel: L_iK = A_iK L_KK^{-T} = A_iK (L_KK^{-1})^T, block rows i > K over waves
    for (int i = K + 1 + wave; i < nblk; i += 4) {
      double* Ai = Ls + slot(i, K) * kBlk;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      acc = mma_abt(Ai, (const double*)s_dinv, acc, lane, 1.0);
      store_acc(Ai, acc, lane);
    }
    __syncthreads();
    // (c) trailing update: A_ij -= L_iK L_jK^T for K < j <= i
    const int rem = nblk - 1 - K;
    const int pairs = rem * (rem + 1) / 2;
    for (int q = wave; q < pairs; q += 4) {
      int ii = 0;
      while ((ii + 1) * (ii + 2) / 2 <= q) ++ii;
      const int jj = q - ii * (ii + 1) / 2;
      const int i = K + 1 + ii, j = K + 1 + jj;
      double* Aij = Ls + slot(i, j) * kBlk;
      d4 acc = load_acc(Aij, lane);
      acc = mma_abt(Ls + slot(i, K) * kBlk, Ls + slot(j, K) * kBlk, acc, lane, -1.0);
      store_acc(Aij, acc, lane);
    }
    __syncthreads();
  }
  if (kInLds)
#pragma unroll 8
    for (int e = threadIdx.x; e < nslots * kBlk; e += 256) Lp[e] = Ls[e];
}

// Solve L L^T Z = B for 16 columns per wave (64 per workgroup); the factor is staged in LDS
// when it fits.  NB > 0: exactly NB blocks, loops unrolled so the right-hand sides stay in
// registers; NB == 0: any nblk <= 64 (right-hand sides in scratch).
// mode 0: write Z into the slice-major core (core[i * P + p] = Z[p][i]).
// mode 1: leverage rows: l_i = ||L^{-1} g_i||^2 with g_i = row i of the core (B^T = G_(2));
//         writes the integer weights Q_i = floor(l_i / P * 2^52).
template <typename Real, bool kInLds, int NB>
__global__ __launch_bounds__(256) void k_chol_solve(int P, int In, const double* __restrict__ Lp,
                                                    const double* __restrict__ Dinv, const double* __restrict__ B,
                                                    void* core, uint64_t* Q, int mode, const int* status) {
  extern __shared__ double lds[];
  if (*status != kDevOk) return;
  constexpr int kCap = NB > 0 ? NB : 64;
  constexpr int kUnroll = NB > 0 ? NB : 1;
  const int nblk = NB > 0 ? NB : (P + 15) / 16;
  const int nslots = nblk * (nblk + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* Ls = Lp;
  const double* Ds = Dinv;
  if (kInLds) {
    double* l2 = lds;
    double* d2 = lds + nslots * kBlk;
#pragma unroll 8
    for (int e = threadIdx.x; e < nslots * kBlk; e += 256) l2[e] = Lp[e];
#pragma unroll 8
    for (int e = threadIdx.x; e < nblk * 256; e += 256) d2[(e >> 8) * kBlk + ((e >> 4) & 15) * kLd + (e & 15)] = Dinv[e];
    __syncthreads();
    Ls = l2;
    Ds = d2;
  }
  const int dstride = kInLds ? kBlk : 256;
  const int dld = kInLds ? kLd : 16;
  const int col = blockIdx.x * 64 + wave * 16 + (lane & 15);
  const bool live = col < In;
  const int ar = lane & 15, ak = lane >> 4;
  d4 Y[kCap];
#pragma unroll kUnroll
  for (int K = 0; K < kCap; ++K) {
    if (K < nblk) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = 16 * K + 4 * r + ak;
        double v = 0.0;
        if (live && p < P) {
          if (mode == 0) v = B[(int64_t)p * In + col];
          else v = (double)((const Real*)core)[(int64_t)col * P + p];
        }
        Y[K][r] = v;
      }
    }
  }
  // forward: Y_K = L_KK^{-1} (B_K - sum_{J<K} L_KJ Y_J)
#pragma unroll kUnroll
  for (int K = 0; K < kCap; ++K) {
    if (K < nblk) {
      // two independent accumulation chains (even / odd J), combined in a fixed order
      d4 acc = Y[K], acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll kUnroll
      for (int J = 0; J < kCap; ++J) {
        if (J < K) {
          const double* LKJ = Ls + slot(K, J) * kBlk;
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            if (J & 1)
              acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(-LKJ[ar * kLd + 4 * ks + ak], Y[J][ks], acc1, 0, 0, 0);
            else
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-LKJ[ar * kLd + 4 * ks + ak], Y[J][ks], acc, 0, 0, 0);
          }
        }
      }
      acc += acc1;
      d4 y = {0.0, 0.0, 0.0, 0.0};
      const double* D = Ds + K * dstride;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        y = __builtin_amdgcn_mfma_f64_16x16x4f64(D[ar * dld + 4 * ks + ak], acc[ks], y, 0, 0, 0);
      Y[K] = y;
    }
  }
  if (mode == 1) {
    double s = 0.0;
#pragma unroll kUnroll
    for (int K = 0; K < kCap; ++K)
      if (K < nblk)
#pragma unroll
        for (int r = 0; r < 4; ++r) s += Y[K][r] * Y[K][r];
    // lanes c, c + 16, c + 32, c + 48 hold the four row groups of column c
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (live && lane < 16) {
      const double p = s / (double)P;
      Q[col] = (uint64_t)floor(p * 4503599627370496.0);  // 2^52
    }
    return;
  }
  // backward: Z_K = L_KK^{-T} (Y_K - sum_{J>K} L_JK^T Z_J)
#pragma unroll kUnroll
  for (int K = kCap - 1; K >= 0; --K) {
    if (K < nblk) {
      d4 acc = Y[K], acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll kUnroll
      for (int J = 0; J < kCap; ++J) {
        if (J > K && J < nblk) {
          const double* LJK = Ls + slot(J, K) * kBlk;
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            if (J & 1)
              acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(-LJK[(4 * ks + ak) * kLd + ar], Y[J][ks], acc1, 0, 0, 0);
            else
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-LJK[(4 * ks + ak) * kLd + ar], Y[J][ks], acc, 0, 0, 0);
          }
        }
      }
      acc += acc1;
      d4 z = {0.0, 0.0, 0.0, 0.0};
      const double* D = Ds + K * dstride;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        z = __builtin_amdgcn_mfma_f64_16x16x4f64(D[(4 * ks + ak) * dld + ar], acc[ks], z, 0, 0, 0);
      Y[K] = z;
    }
  }
  if (!live) return;
  Real* out = (Real*)core;
#pragma unroll kUnroll
  for (int K = 0; K < kCap; ++K)
    if (K < nblk)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = 16 * K + 4 * r + ak;
        if (p < P) out[(int64_t)col * P + p] = (Real)Y[K][r];
      }
}

template <typename Real, bool kInLds>
void solve_dispatch(int nblk, unsigned blocks, size_t lds, int P, int In, const double* Lp, const double* Dinv,
                    const double* B, void* core, uint64_t* Q, int mode, const int* status, hipStream_t s) {
  const size_t sh = kInLds ? lds : 0;
  switch (nblk) {
#define TRALS_SOLVE_CASE(NB) \
  case NB: k_chol_solve<Real, kInLds, NB><<<blocks, 256, sh, s>>>(P, In, Lp, Dinv, B, core, Q, mode, status); break;
    TRALS_SOLVE_CASE(1)
    TRALS_SOLVE_CASE(2)
    TRALS_SOLVE_CASE(3)
    TRALS_SOLVE_CASE(4)
    TRALS_SOLVE_CASE(5)
    TRALS_SOLVE_CASE(6)
    TRALS_SOLVE_CASE(7)
    TRALS_SOLVE_CASE(8)
    TRALS_SOLVE_CASE(9)
#undef TRALS_SOLVE_CASE
    default: k_chol_solve<Real, kInLds, 0><<<blocks, 256, sh, s>>>(P, In, Lp, Dinv, B, core, Q, mode, status);
  }
}

}  // namespace

size_t chol_factor_doubles(int P) {
  const int nblk = (P + 15) / 16;
  return (size_t)nblk * (nblk + 1) / 2 * kBlk + (size_t)nblk * 256;
}

hipError_t launch_chol_factor(int P, const double* H, double* F, int* status, hipStream_t s) {
  const int nblk = (P + 15) / 16;
  double* Lp = F;
  double* Dinv = F + (size_t)nblk * (nblk + 1) / 2 * kBlk;
  if (nblk <= kLdsBlocks) {
    const size_t lds = (size_t)nblk * (nblk + 1) / 2 * kBlk * sizeof(double);
    k_chol_blocked<true><<<1, 256, lds, s>>>(P, H, Lp, Dinv, status);
  } else {
    k_chol_blocked<false><<<1, 256, 0, s>>>(P, H, Lp, Dinv, status);
  }
  return hipGetLastError();
}

hipError_t launch_chol_solve(int P, int In, const double* F, const double* B, void* core, int real_dtype,
                             uint64_t* Q, int mode, const int* status, hipStream_t s) {
  const int nblk = (P + 15) / 16;
  if (nblk > 64) return hipErrorInvalidValue;
  const double* Lp = F;
  const double* Dinv = F + (size_t)nblk * (nblk + 1) / 2 * kBlk;
  const unsigned blocks = (unsigned)((In + 63) / 64);
  const size_t lds = ((size_t)nblk * (nblk + 1) / 2 + nblk) * kBlk * sizeof(double);
  const bool in_lds = nblk <= kLdsBlocks;
  if (real_dtype == 0) {
    if (in_lds) solve_dispatch<double, true>(nblk, blocks, lds, P, In, Lp, Dinv, B, core, Q, mode, status, s);
    else solve_dispatch<double, false>(nblk, blocks, lds, P, In, Lp, Dinv, B, core, Q, mode, status, s);
  } else if (real_dtype == 1) {
    if (in_lds) solve_dispatch<float, true>(nblk, blocks, lds, P, In, Lp, Dinv, B, core, Q, mode, status, s);
    else solve_dispatch<float, false>(nblk, blocks, lds, P, In, Lp, Dinv, B, core, Q, mode, status, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace trals
