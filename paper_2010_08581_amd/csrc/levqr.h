// Rank-revealing leverage table of one core (eq. (3), Definition 4), by Householder QR with
// column pivoting of its unfolding G_(2) itself (no Gram matrix, so the condition number is
// not squared).  This is the path for cores whose Gram factorisation is not certain: a wide
// core (I <= P) whose row Gram G G^T did not factor, or a tall core (I > P) whose column Gram
// G^T G did not.
//
//   G Pi = Q R,  |R_00| >= |R_11| >= ... (pivot = largest remaining column norm)
//   rank r = number of k with |R_kk| > max(I, P) eps |R_00|
//   l_i = ||Q(i, 0:r)||^2  (Q(:, 0:r) spans the column space of G), or exactly 1 when r = I
//   Q_i = floor(l_i / r * 2^52)
//
// The tolerance is the usual numerical-rank tolerance max(rows, cols) eps, taken relative to
// the largest column norm |R_00| (between sigma_max / sqrt(P) and sigma_max).  A zero core
// (r = 0) has no distribution and raises *status = kDevSingular.
//
// One workgroup runs it (nthr threads, a multiple of 64) on a column-major copy A of G in
// global memory.  Pivoting keeps a map from logical to physical columns instead of moving
// columns.  Every reduction is a fixed-order butterfly within a wave and a fixed-order sum over
// waves, so the table is reproducible bit for bit.  Shared scratch: lev_qr_smem_bytes(P).
#pragma once

#include "kernels.h"

namespace trals {

__host__ __device__ constexpr size_t lev_qr_smem_bytes(int P) {
  // u0, tau' (P doubles each), wave maxima (16 doubles + 16 ints), map (P ints)
  return (size_t)2 * P * 8 + 16 * 8 + 16 * 4 + (size_t)P * 4;
}

__device__ __forceinline__ double lq_wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// G: slice-major I x P (row i = lateral slice i), A: I * P doubles of work memory, Q: I table
// weights.  Every thread of the workgroup must call it; it holds barriers.
__device__ inline void lev_qr_table(const double* __restrict__ G, int I, int P, double* __restrict__ A,
                             uint64_t* __restrict__ Qout, int* status, unsigned char* smem, int tid,
                             int nthr) {
  const int m = I, n = P, kmax = m < n ? m : n;
  const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  // per-wave maxima of the remaining column norms sum_{i >= k} A(i, j)^2 (logical j): the
  // pivot candidates of step k
  double* wmax = (double*)smem;
  int* widx = (int*)(wmax + 16);
  double* u0 = (double*)(widx + 16);  // first entry of reflector k (alpha - beta)
  double* tq = u0 + n;                // tau' of reflector k: H = I - tau' u u^T
  int* map = (int*)(tq + n);          // logical column -> physical column
  // column-major copy: A[j m + i] = G[i n + j]
  for (int64_t e = tid; e < (int64_t)m * n; e += nthr) {
    const int j = (int)(e / m), i = (int)(e - (int64_t)j * m);
    A[e] = G[(int64_t)i * n + j];
  }
  for (int j = tid; j < n; j += nthr) map[j] = j;
  __syncthreads();
  // initial column norms and the first pivot candidates
  {
    double bv = -1.0;
    int bi = n;
    for (int j = wave; j < n; j += nw) {
      const double* c = A + (int64_t)j * m;
      double s1 = 0.0;
      for (int i = lane; i < m; i += 64) s1 += c[i] * c[i];
      s1 = lq_wave_sum(s1);
      if (s1 > bv) {
        bv = s1;
        bi = j;
      }
    }
    if (lane == 0) {
      wmax[wave] = bv;
      widx[wave] = bi;
    }
  }
  __syncthreads();
  int r = kmax;
  double r00 = 0.0;
  const double tolf = (double)(m > n ? m : n) * 2.220446049250313e-16;
  for (int k = 0; k < kmax; ++k) {
    // pivot: the largest remaining column norm (first index on ties), the same in every thread
    double vmax = wmax[0];
    int p = widx[0];
    for (int w = 1; w < nw; ++w)
      if (wmax[w] > vmax || (wmax[w] == vmax && widx[w] < p)) {
        vmax = wmax[w];
        p = widx[w];
      }
    const double rkk = sqrt(vmax > 0.0 ? vmax : 0.0);
    if (k == 0) r00 = rkk;
    if (!(rkk > tolf * r00)) {
      r = k;
      break;
    }
    const int pc = map[p];  // physical pivot column
    const double* cp = A + (int64_t)pc * m;
    // the reflector's tail norm, summed by every wave alike (the same operations in the same
    // order, so every thread derives the same reflector)
    double t2 = 0.0;
    for (int i = k + 1 + lane; i < m; i += 64) t2 += cp[i] * cp[i];
    t2 = lq_wave_sum(t2);
    const double alpha = cp[k];
    const double nrm = sqrt(alpha * alpha + t2);
    const double beta = alpha >= 0.0 ? -nrm : nrm;
    const double uk = alpha - beta;                           // |uk| >= nrm > 0
    const double taup = (beta - alpha) / (beta * uk * uk);    // H = I - taup u u^T, u = (uk, A(k+1:, pc))
    __syncthreads();  // every thread has read the maxima and map[p] of this step
    if (tid == 0) {
      map[p] = map[k];
      map[k] = pc;
      u0[k] = uk;
      tq[k] = taup;
    }
    __syncthreads();
    // apply H_k to logical columns k+1 .. n-1 and take their norms over rows k+1 ..
    double bv = -1.0;
    int bi = n;
    for (int j = k + 1 + wave; j < n; j += nw) {
      double* c = A + (int64_t)map[j] * m;
      double d = 0.0;
      for (int i = k + 1 + lane; i < m; i += 64) d += cp[i] * c[i];
      d = lq_wave_sum(d) + uk * c[k];
      const double f = taup * d;
      double s1 = 0.0;
      for (int i = k + 1 + lane; i < m; i += 64) {
        const double v = c[i] - f * cp[i];
        c[i] = v;
        s1 += v * v;
      }
      s1 = lq_wave_sum(s1);
      if (lane == 0) c[k] -= f * uk;
      if (s1 > bv) {
        bv = s1;
        bi = j;
      }
    }
    if (lane == 0) {
      wmax[wave] = bv;
      widx[wave] = bi;
    }
    __syncthreads();
  }
  if (r == 0) {
    if (tid == 0) *status = kDevSingular;
    return;
  }
  if (r == m) {
    // full row rank: every row of the left singular factor is a unit vector
    const double pr = 1.0 / (double)r;
    const uint64_t q = (uint64_t)floor(pr * 4503599627370496.0);
    for (int i = tid; i < m; i += nthr) Qout[i] = q;
    return;
  }
  // Q(:, 0:r) = H_0 ... H_{r-1} [I_r; 0], backward over the reflectors, in place over the
  // pivot columns: column k of Q is H_k e_k (rows < k zero); H_k also acts on the columns
  // k+1 .. r-1 already formed.
  for (int k = r - 1; k >= 0; --k) {
    const double* cp = A + (int64_t)map[k] * m;
    const double uk = u0[k], taup = tq[k];
    for (int j = k + 1 + wave; j < r; j += nw) {
      double* c = A + (int64_t)map[j] * m;
      double d = 0.0;
      for (int i = k + 1 + lane; i < m; i += 64) d += cp[i] * c[i];
      d = lq_wave_sum(d) + uk * c[k];
      const double f = taup * d;
      for (int i = k + 1 + lane; i < m; i += 64) c[i] -= f * cp[i];
      if (lane == 0) c[k] -= f * uk;
    }
    __syncthreads();  // column k's reflector is read above; it is overwritten next
    double* ck = A + (int64_t)map[k] * m;
    const double g = -taup * uk;
    for (int i = tid; i < m; i += nthr) {
      if (i < k) ck[i] = 0.0;
      else if (i == k) ck[i] = 1.0 - taup * uk * uk;
      else ck[i] = g * ck[i];
    }
    __syncthreads();
  }
  const double rr = (double)r;
  for (int i = tid; i < m; i += nthr) {
    double l = 0.0;
    for (int j = 0; j < r; ++j) {
      const double v = A[(int64_t)map[j] * m + i];
      l += v * v;
    }
    Qout[i] = (uint64_t)floor(l / rr * 4503599627370496.0);
  }
}

}  // namespace trals
