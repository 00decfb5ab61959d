// Small dense FP64 linear algebra of one core update, on matrix cores:
//
//  * The Gram matrix K = G_(2)^T G_(2) of a core's I x P unfolding, for its leverage scores
//    (eq. (3)).
//  * Cholesky factorisation H = L L^T of a P x P SPD matrix (H of the LS step of Algorithm 2,
//    or K) and the explicit inverse factor W = L^{-1}.  The paper solves the LS problem by QR;
//    the normal equations agree with it up to cond(A)^2 * eps.
//  * With W: the solve Z = W^T (W B) (lateral slices of the new core) and the leverage rows
//    l_i = ||W g_i||^2 (Definition 4 via K^{-1} = W^T W), as block products without
//    dependency chains.
//
// Matrices are split into 16 x 16 blocks (P padded to 16 nblk with an identity tail).  Lower
// triangular block matrices are stored block-packed: block (i, j), i >= j, at slot
// i (i + 1) / 2 + j, each block 16 rows of kLd doubles.
//
// v_mfma_f64_16x16x4 layouts (one wave): A(i, k) in lane i + 16 k, B(k, j) in lane j + 16 k,
// D(i, j) in lane j + 16 (i % 4), register i / 4.  Register r of an accumulator therefore holds
// exactly the B operand of k-step r of a following product.
#include <string.h>

#include "kernels.h"
#include "levqr.h"
#include "reduce.h"

namespace trals {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kLd = kPackLd;    // padded row stride of a 16 x 16 block (doubles)
constexpr int kBlk = kPackBlk;  // doubles per stored block
constexpr int kLdsBlocks = 9;   // nblk up to which a factor is staged in LDS (45 blocks, 98 KB)
constexpr int kCholWaves = 8;  // waves per workgroup of the large-P steps
static_assert(kCholWaves % 4 == 0, "band workgroups split 4, 2 or 1 rows over the waves");
// dynamic LDS of a large-P step: a four-block region (10 blocks), its staging blocks (4), the
// previous step's panel rows (16), that panel's operands (10 + 16); the band workgroups of the
// same launch use the first 16 blocks.  With the static arrays of the factorisation (about
// 12 KB) it stays within the 160 KB of a workgroup.
constexpr size_t kRegionLdsBytes = (size_t)(10 + 4 + 16 + 10 + 16) * kBlk * sizeof(double);
constexpr size_t kWrowLdsBytes = (size_t)16 * kBlk * sizeof(double);
static_assert(kRegionLdsBytes + 16384 <= 160 * 1024, "large-P step LDS");
constexpr int kMaxBlk = 64;     // P <= 1024
constexpr int kMaxSolveParts = 8;  // workgroups per 16-row group and half of a split solve

// 1/sqrt(x) for x > 0: hardware estimate refined by two Newton steps y <- y (3 - x y^2) / 2
// (each step squares the relative error), instead of the longer correctly-rounded sqrt and
// division sequences on the pivot chain of the factorisation.
__device__ __forceinline__ double rsqrt_f64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  y = y * (1.5 - 0.5 * x * y * y);
  return y;
}

// value of v in lane `src` (wave-uniform) for every lane
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// acc += sign * A B^T for 16 x 16 blocks A, B (row-major, stride kLd)
template <typename PA, typename PB>
__device__ __forceinline__ d4 mma_abt(PA A, PB B, d4 acc, int lane, double sign) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int r = lane & 15, k = 4 * ks + (lane >> 4);
    acc = mfma(sign * A[r * kLd + k], B[r * kLd + k], acc);
  }
  return acc;
}

// acc += A B for 16 x 16 blocks A, B (row-major, stride kLd)
template <typename PA, typename PB>
__device__ __forceinline__ d4 mma_ab(PA A, PB B, d4 acc, int lane) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int r = lane & 15, k = 4 * ks + (lane >> 4);
    acc = mfma(A[r * kLd + k], B[k * kLd + r], acc);
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

// a lane's four operand values of a 16 x 16 block (row-major, stride kLd) for mma_frag: entry
// (lane % 16, 4 ks + lane / 16) for ks = 0 .. 3
template <typename Ptr>
__device__ __forceinline__ void load_frag(Ptr X, int lane, double f[4]) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) f[ks] = X[(lane & 15) * kLd + 4 * ks + (lane >> 4)];
}

// the inverse of load_frag: write a lane's four operand values of a 16 x 16 block
template <typename Ptr>
__device__ __forceinline__ void store_frag(Ptr X, const d4& f, int lane) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) X[(lane & 15) * kLd + 4 * ks + (lane >> 4)] = f[ks];
}

// acc += sign * A B^T from fragments loaded by load_frag (the same product as mma_abt)
__device__ __forceinline__ d4 mma_frag(const double a[4], const double b[4], d4 acc, double sign) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) acc = mfma(sign * a[ks], b[ks], acc);
  return acc;
}

// acc += sign sum_{c < n} A_c B_c^T over blocks A_c = A0 + c kBlk, B_c = B0 + c kBlk (1 <= n <= 4),
// added in the order c = 0, 1, ... like repeated mma_abt; every fragment is loaded before the
// first product (loads past n repeat block n - 1 and are not used)
template <typename PA, typename PB>
__device__ __forceinline__ d4 mma_abt_run4(PA A0, PB B0, int n, d4 acc, int lane, double sign) {
  double fa[4][4], fb[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int cc = c < n ? c : n - 1;
    load_frag(A0 + cc * kBlk, lane, fa[c]);
    load_frag(B0 + cc * kBlk, lane, fb[c]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (c < n) acc = mma_frag(fa[c], fb[c], acc, sign);
  return acc;
}

// ---------------------------------------------------------------------------------------
// K = A^T A (P x P, row-major; the lower blocks including full diagonal blocks are written)
// for A = rows x P, row-major, or column-major when kTrans (element (r, c) at c * rows + r).
// One workgroup of 16 waves per lower block; wave w takes the 4-row k-steps w, w + 16, ...
// (eight loads in flight) and the wave sums are added in the order 0, 1, ..., 15.
constexpr int kSyrkWaves = 16;
template <bool kTrans>
__global__ __launch_bounds__(64 * kSyrkWaves) void k_syrk(const double* __restrict__ A, int64_t rows, int P,
                                                          double* __restrict__ Kout, const int* status,
                                                          int* clear, int packed) {
  __shared__ double red[kSyrkWaves - 1][4][64];
  if (*status != kDevOk) return;
  if (clear && blockIdx.x == 0 && threadIdx.x == 0) *clear = 0;
  int bi, bj;
  slot_ij(blockIdx.x, bi, bj);
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loops
  const int r16 = lane & 15, k4 = lane >> 4;
  const int ci = 16 * bi + r16, cj = 16 * bj + r16;
  const int cic = ci < P ? ci : P - 1, cjc = cj < P ? cj : P - 1;
  const double mi = ci < P ? 1.0 : 0.0;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  const int64_t steps = (rows + 3) / 4;
  for (int64_t k0 = wave; k0 < steps; k0 += 8 * kSyrkWaves) {
    double va[8], vb[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = 4 * (k0 + (int64_t)u * kSyrkWaves) + k4;
      const int64_t rc = r < rows ? r : rows - 1;
      va[u] = (r < rows ? mi : 0.0) * (kTrans ? A[cic * rows + rc] : A[rc * P + cic]);
      vb[u] = kTrans ? A[cjc * rows + rc] : A[rc * P + cjc];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = mfma(va[u], vb[u], acc);
  }
  if (wave > 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wave - 1][q][lane] = acc[q];
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double v = acc[q];
    for (int w = 0; w < kSyrkWaves - 1; ++w) v += red[w][q][lane];
    const int row = 16 * bi + 4 * q + k4, col = 16 * bj + r16;
    if (packed) {
      // block-packed (P % 16 == 0): the blocked factorisation's work matrix, padding column zero
      double* blk = Kout + (int64_t)blockIdx.x * kBlk + (4 * q + k4) * kLd;
      blk[r16] = v;
      if (r16 == 0) blk[16] = 0.0;
    } else if (row < P && col < P) {
      Kout[(int64_t)row * P + col] = v;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Cholesky factorisation and inverse factor, one workgroup of kW waves (8 or 16).
//
// Right-looking over 16-column panels.  Panel K: the panel waves each hold the 16 rows of the
// diagonal block (lanes 0-15, identical copies) and three sub-diagonal block rows (lanes
// 16-63) in registers; pivot step k broadcasts column k of the diagonal block across the
// wave with lane reads (no LDS round trip), and every lane updates its row.  Then all waves
// apply the trailing update A_ij -= L_iK L_jK^T on matrix cores.  Afterwards the diagonal
// blocks are inverted (forward substitution per column) and W = L^{-1} is completed block
// row by block row: W_IK = -W_II sum_{J=K}^{I-1} L_IJ W_JK.
//
// kRegion = false: the whole P x P matrix (row-major H) in LDS, W to a.W.
// kRegion = true: the diagonal region of a.nb blocks starting at block a.b0 of the block-packed
// work matrix a.Lg (the large-P path below), tolerance from a.scal[0]; its inverse goes to the
// same blocks of a.W.
template <bool kRegion, int kW>
__device__ __forceinline__ bool chol_body(const CholArgs& a) {
  constexpr int kThr = 64 * kW, kGroups = kThr / 256;  // threads; 256-thread groups
  extern __shared__ double lds[];
  __shared__ int s_fail;
  __shared__ double s_tol;
  __shared__ double s_rdiag[16 * kMaxBlk];  // 1 / L_ii
  __shared__ double s_diag[16 * kLd];       // factored diagonal block of the current panel
  __shared__ double s_lt[16 * 16];          // transpose of the diagonal block being inverted
  if (*a.status != kDevOk || (a.fail && *a.fail)) return false;
  int* const fail_out = a.fail ? a.fail : a.status;
  const int P = a.P;
  const double* H = a.H;
  double* Wg = a.W;
  const int g0 = kRegion ? a.b0 : 0;  // global block index of local block 0
  const int nblk = kRegion ? a.nb : (P + 15) / 16;
  const int nslots = nblk * (nblk + 1) / 2;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loops
  double* Ls = lds;
  // region path: the previous step's inverse diagonal blocks W(pb0 + c, pb0 + c2), c2 <= c, and
  // the region's rows of its block columns A(g0 + bi, pb0 + c2), the operands of the panel below
  // (after the staging blocks and the panel blocks)
  const int nWp = kRegion ? a.pnb * (a.pnb + 1) / 2 : 0;
  double* const Wp = Ls + (nslots + nblk + nblk * (kRegion ? a.pnb : 0)) * kBlk;
  double* const Ap = Wp + nWp * kBlk;
  if (kRegion) {
    // the region's blocks and the panel operands, one wave per block (a lane takes four entries
    // of row lane / 4, lanes 0-15 the padding column too); every load of a wave is issued before
    // its first store
    constexpr int kPer = (10 + 10 + 16 + kW - 1) / kW;  // blocks per wave: four-block regions
    const int nall = nslots + nWp + nblk * a.pnb;
    const int r = lane >> 2, c0 = 4 * (lane & 3);
    double v[kPer][5];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = wave + kW * u;
      const double* src = a.Lg;
      int bi, bj;
      if (q < nslots) {
        slot_ij(q, bi, bj);
        src = a.Lg + (int64_t)slot(g0 + bi, g0 + bj) * kBlk;
      } else if (q < nslots + nWp) {
        slot_ij(q - nslots, bi, bj);
        src = a.W + (int64_t)slot(a.pb0 + bi, a.pb0 + bj) * kBlk;
      } else if (q < nall) {
        const int t = q - nslots - nWp;
        bi = t / a.pnb;
        src = a.Lg + (int64_t)slot(g0 + bi, a.pb0 + t - bi * a.pnb) * kBlk;
      }
      const bool in = q < nall;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[u][i] = in ? src[r * kLd + c0 + i] : 0.0;
      v[u][4] = in && lane < 16 ? src[lane * kLd + 16] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = wave + kW * u;
      if (q < nall) {
        double* dst = q < nslots ? Ls + q * kBlk : q < nslots + nWp ? Wp + (q - nslots) * kBlk : Ap + (q - nslots - nWp) * kBlk;
#pragma unroll
        for (int i = 0; i < 4; ++i) dst[r * kLd + c0 + i] = v[u][i];
        if (lane < 16) dst[lane * kLd + 16] = v[u][4];
      }
    }
  } else {
    // stage the lower blocks (full diagonal blocks; identity on the padded diagonal), eight
    // loads in flight per thread.  A wave covers four rows of one block: the block (bi, bj) is
    // wave-uniform and walks four slots per load (no per-element index arithmetic).
    constexpr int kB = 8;
    const int r = (threadIdx.x >> 4) & 15, c = threadIdx.x & 15;
    for (int base = 0; base < nslots; base += kGroups * kB) {
      int sl = __builtin_amdgcn_readfirstlane(base + ((int)threadIdx.x >> 8));
      int bi, bj;
      slot_ij(sl, bi, bj);
      double v[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int i = 16 * bi + r, j = 16 * bj + c;
        const bool in = sl < nslots && i < P && j < P;
        v[q] = in ? H[(int64_t)i * P + j] : (i == j ? 1.0 : 0.0);
        bj += kGroups;  // next slot of this wave: kGroups slots on
        while (bj > bi) {
          bj -= bi + 1;
          ++bi;
        }
        sl += kGroups;
      }
      sl -= kGroups * kB;
#pragma unroll
      for (int q = 0; q < kB; ++q)
        if (sl + kGroups * q < nslots) Ls[(sl + kGroups * q) * kBlk + r * kLd + c] = v[q];
    }
  }
  __syncthreads();
  if (kRegion) {
    if (a.prepacked && a.b0 == 0) {
      // the first step of a matrix a reduction packed (no k_big_init) takes the tolerance from
      // the largest diagonal entry itself, for the steps after it too
      if (wave == 0) {
        double mx = 0.0;
        for (int i = lane; i < P; i += 64)
          mx = fmax(mx, a.Lg[(int64_t)slot(i >> 4, i >> 4) * kBlk + (i & 15) * kLd + (i & 15)]);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
        if (lane == 0) {
          const double tol = (a.rel_tol > 0.0 ? a.rel_tol : (double)P * 2.220446049250313e-16) * mx;
          s_tol = tol;
          a.scal[0] = tol;
          s_fail = !(mx > 0.0) || !isfinite(mx);
        }
      }
    } else if (threadIdx.x == 0) {
      s_tol = a.scal[0];
      s_fail = 0;
    }
    // the previous step's panel for the rows of this region, L(i, pb0 + c) = sum_{c' <= c}
    // A(i, pb0 + c') W(pb0 + c, pb0 + c')^T (into LDS after the staging blocks, and into Lp),
    // then its trailing update A_ij -= sum_c L(i, pb0 + c) L(j, pb0 + c)^T
    if (a.pnb > 0) {
      double* Lsc = Ls + (nslots + nblk) * kBlk;  // nblk x pnb blocks
      // (the previous region has four blocks, pnb = 4 divides kW: odd rounds take the columns in
      // reverse, so that a wave's tasks c and 3 - c add up to five block products)
      for (int t = wave; t < nblk * a.pnb; t += kW) {
        const int bi = t / a.pnb, cr = t - bi * a.pnb;
        const int c = ((t / kW) & 1) ? a.pnb - 1 - cr : cr;
        d4 f = {0.0, 0.0, 0.0, 0.0};
        // blocks (c, c2), c2 = 0 .. c, are consecutive slots
        f = mma_abt_run4(Wp + slot(c, 0) * kBlk, Ap + bi * a.pnb * kBlk, c + 1, f, lane, 1.0);
        // f holds W L^T's block, i.e. L(g0 + bi, pb0 + c) in operand order
        store_frag(Lsc + (bi * a.pnb + c) * kBlk, f, lane);
        store_frag(a.Lp + (int64_t)slot(g0 + bi, a.pb0 + c) * kBlk, f, lane);
      }
      __syncthreads();
      for (int sl = wave; sl < nslots; sl += kW) {
        int bi, bj;
        slot_ij(sl, bi, bj);
        double* Ab = Ls + sl * kBlk;
        d4 acc = load_acc(Ab, lane);
        acc = mma_abt_run4(Lsc + bi * a.pnb * kBlk, Lsc + bj * a.pnb * kBlk, a.pnb, acc, lane, -1.0);
        store_acc(Ab, acc, lane);
      }
    }
  } else if (wave == 0) {
    double mx = 0.0;
    for (int i = lane; i < P; i += 64) mx = fmax(mx, Ls[slot(i >> 4, i >> 4) * kBlk + (i & 15) * kLd + (i & 15)]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if (lane == 0) {
      s_tol = (a.rel_tol > 0.0 ? a.rel_tol : (double)P * 2.220446049250313e-16) * mx;
      s_fail = !(mx > 0.0) || !isfinite(mx);
    }
  }
  __syncthreads();
  if (s_fail) {
    if (threadIdx.x == 0) *fail_out = kDevSingular;
    return false;
  }
  const double tol = s_tol;
  const int l = lane & 15, grp = lane >> 4;
  // W = L^{-1} is built while the factorisation proceeds.  Phase A of step K runs panel K on
  // waves [0, triples) and, on the other waves (counted from the top), the inverse of diagonal
  // block K-1 (wave 15, in place: slot (K-1, K-1) has no other reader after panel K-1) and the
  // off-diagonal blocks of W's block row K-2,
  //   W_IJ = -W_II sum_{M=J}^{I-1} L_IM W_MJ   (I = K-2, J < I),
  // held in registers.  Phase B stores the factored diagonal block, applies the trailing update
  // of column K and copies the block row of W into place from its staging blocks (nothing else
  // reads row K-2 any more).  Steps nblk and nblk+1 finish the last inverse and the last two
  // block rows.
  constexpr int kHelpers = kW - 1;  // waves taking W block-row tasks (stride)
  const int hw = kW - 1 - wave;     // 0: the inverse wave, 1.. : W block-row tasks
  double* Stg = Ls + nslots * kBlk;         // nblk staging blocks for one block row of W
  for (int K = 0; K <= nblk + 1; ++K) {
    const bool factor = K < nblk;
    const int below = nblk - 1 - K;
    const int triples = !factor ? 0 : below == 0 ? 1 : (below + 2) / 3;  // sub-diagonal triples
    // ---- phase A: panel K ----
    // The diagonal block stays unmodified in memory during the panel (each pass loads its own
    // copy); the factored block goes to s_diag and is stored after the panel barrier.
    for (int tri = wave; tri < triples; tri += kW) {
      int bi = grp == 0 ? K : K + 3 * tri + grp;
      const bool held = grp == 0 || bi < nblk;
      if (!held) bi = K;
      double* src = Ls + slot(bi, K) * kBlk + l * kLd;
      double v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = src[c];
      int bad = 0;
      double myil = 0.0;
      // l re-read here: keeps the sixteen lane == k masks from being hoisted out of the step
      // loop, where they would hold 32 scalar registers for the whole kernel
      int lme = l;
      asm volatile("" : "+v"(lme));
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const double pk = lane_bcast(v[k], k);
        // rows past P are padding (unit pivots), outside the tolerance test: it is relative to
        // the largest diagonal entry and can exceed 1.  Bitwise flags: no branch per pivot.
        const int ok = (int)(pk > tol) & (int)(pk < __builtin_huge_val());
        bad |= (int)(16 * (g0 + K) + k < P) & (ok ^ 1);
        const double il = rsqrt_f64(fmax(pk, 1e-300));
        const double t = v[k] * (il * il);
#pragma unroll
        for (int j = k + 1; j < 16; ++j) v[j] = fma(-t, lane_bcast(v[k], j), v[j]);
        v[k] *= il;
        if (lme == k) myil = il;
        // keep the update right-looking: each column is final when its pivot step starts, so
        // the compiler cannot defer the updates into a dependent chain at the pivot; the
        // breakdown flag and the lane's scale are settled in the step too (deferred past the
        // loop they keep sixteen pivots and scales live)
#pragma unroll
        for (int j = k + 1; j < 16; ++j) asm volatile("" : "+v"(v[j]));
        asm volatile("" : "+v"(myil), "+v"(bad));
      }
      if (grp == 0) {
        if (tri == 0) {
#pragma unroll
          for (int c = 0; c < 16; ++c) s_diag[l * kLd + c] = c <= l ? v[c] : 0.0;
          s_rdiag[16 * K + l] = myil;
          if (lane == 0 && bad) s_fail = 1;
        }
      } else if (held) {
#pragma unroll
        for (int c = 0; c < 16; ++c) src[c] = v[c];
      }
    }
    // ---- phase A: inverse of diagonal block K-1, column l by lane l (forward substitution) ----
    if (hw == 0 && K >= 1 && K <= nblk) {
      // lane l computes column l of the inverse by forward substitution; the block is first
      // transposed into s_lt so that column k of L is a contiguous (broadcast) read
      const int D = K - 1;
      double* Lb = Ls + slot(D, D) * kBlk;
      if (lane < 16)
#pragma unroll
        for (int c = 0; c < 16; ++c) s_lt[c * 16 + l] = Lb[l * kLd + c];
      double x[16];
      int lme = l;  // (as in the panel: no hoisted masks)
      asm volatile("" : "+v"(lme));
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = i == lme ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        x[k] *= s_rdiag[16 * D + k];
#pragma unroll
        for (int i = k + 1; i < 16; ++i) x[i] = fma(-s_lt[k * 16 + i], x[k], x[i]);
      }
      if (lane < 16)
#pragma unroll
        for (int i = 0; i < 16; ++i) Lb[i * kLd + l] = x[i];  // W_DD (lower; zeros above)
    }
    // ---- phase A: the rest of step K-1's trailing update (block columns K+1 and beyond; its
    // column K was updated before this panel), on the waves the panel leaves free ----
    if (K >= 1 && K < nblk && wave >= triples) {
      const int Kp = K - 1;
      const int rem = nblk - K - 1;  // rows and columns K+1 .. nblk-1
      for (int q = wave - triples; q < rem * (rem + 1) / 2; q += kW - triples) {
        int ii, jj;
        slot_ij(q, ii, jj);
        const int i = K + 1 + ii, j = K + 1 + jj;
        double* Aij = Ls + slot(i, j) * kBlk;
        d4 acc = load_acc(Aij, lane);
        acc = mma_abt(Ls + slot(i, Kp) * kBlk, Ls + slot(j, Kp) * kBlk, acc, lane, -1.0);
        store_acc(Aij, acc, lane);
      }
    }
    // ---- phase A: off-diagonal blocks of W's block row I = K-2 (into the staging blocks) ----
    const int I = K - 2;
    if (hw >= 1 && I >= 1) {
      const double* WII = Ls + slot(I, I) * kBlk;
      for (int J = hw - 1; J < I; J += kHelpers) {
        d4 sacc = {0.0, 0.0, 0.0, 0.0};
        for (int M = J; M < I; ++M) sacc = mma_ab(Ls + slot(I, M) * kBlk, Ls + slot(M, J) * kBlk, sacc, lane);
        d4 w = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) w = mfma(-WII[(lane & 15) * kLd + 4 * ks + (lane >> 4)], sacc[ks], w);
        store_acc(Stg + J * kBlk, w, lane);
      }
    }
    __syncthreads();
    if (factor && s_fail) {
      if (threadIdx.x == 0) *fail_out = kDevSingular;
      return false;
    }
    // ---- phase B ----
    if (factor) {
      // factored diagonal block into place (no one reads slot (K, K) during the trailing update)
      double* DK = Ls + slot(K, K) * kBlk;
      for (int e = threadIdx.x; e < 16 * kLd; e += kThr) DK[e] = s_diag[e];
      // trailing update A_ij -= L_iK L_jK^T, block column K+1 only (the next panel); the
      // columns beyond it are updated during the next panel
      for (int ii = wave; ii < below; ii += kW) {
        const int i = K + 1 + ii, j = K + 1;
        double* Aij = Ls + slot(i, j) * kBlk;
        d4 acc = load_acc(Aij, lane);
        acc = mma_abt(Ls + slot(i, K) * kBlk, Ls + slot(j, K) * kBlk, acc, lane, -1.0);
        store_acc(Aij, acc, lane);
      }
    }
    if (I >= 1) {
      // blocks (I, 0 .. I-1) are contiguous slots: one flat copy
      double* dst = Ls + slot(I, 0) * kBlk;
      for (int e = threadIdx.x; e < I * kBlk; e += kThr) dst[e] = Stg[e];
    }
    __syncthreads();
  }
  if (kRegion) {
    for (int e = threadIdx.x; e < nslots * kBlk; e += kThr) {
      int bi, bj;
      slot_ij(e / kBlk, bi, bj);
      Wg[(int64_t)slot(g0 + bi, g0 + bj) * kBlk + e % kBlk] = Ls[e];
    }
  } else {
    copy_batched<4>((double2*)Wg, (const double2*)Ls, (int64_t)nslots * kBlk / 2, threadIdx.x, kThr);
  }
  return true;
}

template <bool kRegion, int kW>
__global__ __launch_bounds__(64 * kW) void k_chol(CholArgs a) {
  chol_body<kRegion, kW>(a);
}

// workgroup 0: the factorisation (whole matrix in LDS); workgroups 1 ..: the fixed-order
// reduction of job jb (the right-hand sides, read by the solve after this launch), kW / 4
// 256-thread reduction blocks per workgroup.  The reduction does not read the status word:
// the factorisation may set it meanwhile, and its indexing does not depend on the data.
template <int kW>
__global__ __launch_bounds__(64 * kW) void k_chol_reduce(CholArgs a, ReduceJob jb, int nparts) {
  __shared__ double red[kW / 4][4][kRedElems];
  if (blockIdx.x == 0) {
    chol_body<false, kW>(a);
    return;
  }
  const int sub = threadIdx.x >> 8;
  reduce_block(jb, ((int64_t)blockIdx.x - 1) * (kW / 4) + sub, nparts, a.P, threadIdx.x & 255, red[sub]);
}

// ---------------------------------------------------------------------------------------
// Large P (more blocks than LDS holds): blocked over 64-column block columns (4 blocks), each
// step spread over many workgroups.  The block-packed work matrix Lg holds H, then L; W holds
// the inverse factor.  Step K: (1) one workgroup factors and inverts the diagonal region
// (W_KK); (2) the panel below it, L_iK = A_iK W_KK^T; (3) the trailing update A_ij -= L_iK
// L_jK^T, applied in the launch of step K + 1: to region K + 1 by its factorisation
// workgroup before it factors, to the blocks below by extra workgroups.  The block rows of W
// follow one 64-row band at a time,
// W_IJ = -W_II sum_{M=J}^{I-1} L_IM W_MJ; band I needs W_II and the bands above it only, so
// it runs beside the factorisation of diagonal region I + 1 (extra workgroups of that launch),
// and only the last band after the factorisation.

// Lg <- H in blocks (identity on the padded diagonal); scal[0] <- tol max_i H_ii (tol = rel_tol,
// or P eps when rel_tol is 0); a zero or non-finite diagonal is a breakdown (*fail_out).  Not
// launched when the producer of H wrote Lg itself (CholArgs.prepacked: the first step then sets
// scal[0] and checks the diagonal).
__global__ __launch_bounds__(256) void k_big_init(const double* __restrict__ H, int P, double* __restrict__ Lg,
                                                  double* scal, const int* status, int* fail_out, double rel_tol) {
  if (*status != kDevOk) return;
  const int nblk = (P + 15) / 16;
  const int64_t total = (int64_t)nblk * (nblk + 1) / 2 * kBlk;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int bi, bj;
    slot_ij((int)(e / kBlk), bi, bj);
    const int rc = (int)(e % kBlk), r = rc / kLd, c = rc % kLd;
    const int i = 16 * bi + r, j = 16 * bj + c;
    double v = 0.0;
    if (c < 16) v = (i < P && j < P) ? H[(int64_t)i * P + j] : (i == j ? 1.0 : 0.0);
    Lg[e] = v;
  }
  if (blockIdx.x == 0) {
    __shared__ double red[256];
    double mx = 0.0;
    for (int i = threadIdx.x; i < P; i += 256) mx = fmax(mx, H[(int64_t)i * P + i]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      mx = red[0];
      scal[0] = (rel_tol > 0.0 ? rel_tol : (double)P * 2.220446049250313e-16) * mx;
      if (!(mx > 0.0) || !isfinite(mx)) *fail_out = kDevSingular;
    }
  }
}

// Trailing block (i, j) after the step on the four blocks b0 .. b0 + 3 (i >= j beyond them), by
// one wave.  The panel rows it needs are formed here, L(x, b0 + c) = sum_{c' <= c}
// A(x, b0 + c') W(b0 + c, b0 + c')^T for x = i, j (every operand loaded before the first
// product); then A_ij -= sum_c L(i, b0 + c) L(j, b0 + c)^T.  The wave of the diagonal block
// (i, i) stores row i of the panel into Lp.  The products W A^T leave L in operand order, so no
// exchange between lanes is needed.
__device__ __forceinline__ void trail_block(double* __restrict__ Lg, double* __restrict__ Lp,
                                            const double* __restrict__ W, int i, int j, int b0, int lane) {
  double fw[10][4], fi[4][4], fj[4][4];
#pragma unroll
  for (int c = 0, t = 0; c < 4; ++c)
#pragma unroll
    for (int c2 = 0; c2 <= c; ++c2, ++t) load_frag(W + (int64_t)slot(b0 + c, b0 + c2) * kBlk, lane, fw[t]);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    load_frag(Lg + (int64_t)slot(i, b0 + c) * kBlk, lane, fi[c]);
    load_frag(Lg + (int64_t)slot(j, b0 + c) * kBlk, lane, fj[c]);
  }
  double* Aij = Lg + (int64_t)slot(i, j) * kBlk;
  d4 acc = load_acc(Aij, lane);
#pragma unroll
  for (int c = 0, t = 0; c < 4; ++c) {
    d4 li = {0.0, 0.0, 0.0, 0.0}, lj = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c2 = 0; c2 <= c; ++c2, ++t) {
      li = mma_frag(fw[t], fi[c2], li, 1.0);
      if (i != j) lj = mma_frag(fw[t], fj[c2], lj, 1.0);
    }
    if (i == j) {
      lj = li;
      store_frag(Lp + (int64_t)slot(i, b0 + c) * kBlk, li, lane);
    }
    const double a4[4] = {li[0], li[1], li[2], li[3]}, b4[4] = {lj[0], lj[1], lj[2], lj[3]};
    acc = mma_frag(a4, b4, acc, -1.0);
  }
  store_acc(Aij, acc, lane);
}

// band I (blocks 4I .. 4I + nbI - 1), four workgroups per band J < I, workgroup q taking the
// block column bj = 4J + q.  Its 8 waves share the nbI output blocks (4I + r, bj): each block's
// chain of products L(4I + r, bm) W(bm, bj), bm = bj .. 4I - 1, is cut into `parts` contiguous
// pieces (8 waves over nbI rows: 2, 4 or 8 pieces), one per wave, and the pieces' sums are added
// in order; then W(4I + r, bj) = -sum_{r2 <= r} W(4I + r, 4I + r2) S(4I + r2, bj).  One output
// per workgroup column keeps the chains short: a band's workgroups are otherwise the longest
// part of the last step.
__device__ __forceinline__ void wrow_body(const double* __restrict__ Lp, double* __restrict__ W, int nblk, int I,
                                          int J, int q) {
  extern __shared__ double lds[];
  double* const stage = lds;      // 8 partial blocks
  double* const sums = lds + 8 * kBlk;  // 4 summed blocks (kWrowLdsBytes: 16 blocks)
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loops
  const int nbI = nblk - 4 * I < 4 ? nblk - 4 * I : 4;
  const int rows = nbI > 2 ? 4 : nbI;  // row slots: 4, 2 or 1
  const int parts = kCholWaves / rows;
  const int r = wave / parts, part = wave - r * parts;
  const int bj = 4 * J + q;
  const int bi = 4 * I + r;
  const int n = 4 * I - bj;                // products of a chain (>= 1)
  const int len = (n + parts - 1) / parts;  // per piece
  {
    d4 sacc = {0.0, 0.0, 0.0, 0.0};
    if (r < nbI)
      for (int bm = bj + part * len; bm < bj + (part + 1) * len && bm < 4 * I; ++bm)
        sacc = mma_ab(Lp + (int64_t)slot(bi, bm) * kBlk, W + (int64_t)slot(bm, bj) * kBlk, sacc, lane);
    store_acc(stage + wave * kBlk, sacc, lane);
  }
  __syncthreads();
  if (part == 0 && r < nbI) {
    d4 v = load_acc(stage + wave * kBlk, lane);
    for (int p = 1; p < parts; ++p) {
      const d4 u = load_acc(stage + (wave + p) * kBlk, lane);
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += u[k];
    }
    store_acc(sums + r * kBlk, v, lane);
  }
  __syncthreads();
  if (part == 0 && r < nbI) {
    d4 w = {0.0, 0.0, 0.0, 0.0};
    for (int r2 = 0; r2 <= r; ++r2)
      w = mma_ab(W + (int64_t)slot(bi, 4 * I + r2) * kBlk, sums + r2 * kBlk, w, lane);
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = -w[k];
    store_acc(W + (int64_t)slot(bi, bj) * kBlk, w, lane);
  }
}

__global__ __launch_bounds__(64 * kCholWaves) void k_big_wrow(const double* __restrict__ Lp, double* __restrict__ W,
                                                              int nblk, int I, const int* status, const int* fail) {
  if (*status != kDevOk || (fail && *fail)) return;
  wrow_body(Lp, W, nblk, I, (int)blockIdx.x >> 2, (int)blockIdx.x & 3);
}

// Step a.b0 / 4 > 0 of the factorisation in one launch.  Workgroup 0 forms the previous step's
// panel for the rows of the diagonal region, applies that step's trailing update to the region,
// then factors and inverts it; workgroups 1 .. 4I take band I of W (I = 0: none); the rest apply
// the previous step's trailing update to the blocks below the region, one block per wave,
// forming the panel rows they need themselves.  Only workgroup 0 reads the status word: it may
// set it meanwhile, and the others' indexing does not depend on the data.
__global__ __launch_bounds__(64 * kCholWaves) void k_chol_step(CholArgs a, int I) {
  const int nblk = (a.P + 15) / 16;
  if (blockIdx.x == 0) {
    chol_body<true, kCholWaves>(a);
    return;
  }
  if ((int)blockIdx.x <= 4 * I) {
    wrow_body(a.Lp, a.W, nblk, I, ((int)blockIdx.x - 1) >> 2, ((int)blockIdx.x - 1) & 3);
    return;
  }
  const int q = ((int)blockIdx.x - 1 - 4 * I) * kCholWaves + (int)(threadIdx.x >> 6);
  const int rem = nblk - a.b0;  // the previous step's trailing blocks start at this region
  if (q >= rem * (rem + 1) / 2) return;
  int ii, jj;
  slot_ij(q, ii, jj);
  if (ii < a.nb) return;  // inside the region: workgroup 0 applies it
  trail_block(a.Lg, a.Lp, a.W, a.b0 + ii, a.b0 + jj, a.pb0, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------------------
// Right-hand sides in row form (row i = b_i, P doubles).  Workgroups [0, solve_groups) solve
// 16 rows each: z_i = W^T (W b_i), written as row i of the core (slice-major, FP64).
// Workgroups [solve_groups, +lev_groups) take 16 rows each of a core unfolding G_(2) and
// write the table weights Q_i = floor(||W g_i||^2 / P * 2^52).  Each of the NW waves takes
// the 16-row blocks K = wave, wave + NW, ...
template <int T, int NW>
__global__ __launch_bounds__(64 * NW) void k_trisolve(TriArgs a) {
  constexpr int kThr = 64 * NW;
  extern __shared__ double lds[];
  __shared__ double s_red[NW][16];
  if (*a.status != kDevOk) return;
  constexpr int kLdB = 17;
  const int P = a.P;
  const int nblk = (P + 15) / 16;
  const bool lev = (int)blockIdx.x >= a.solve_groups;
  const int grp = lev ? (int)blockIdx.x - a.solve_groups : (int)blockIdx.x;
  if (lev && a.lev_fail && *a.lev_fail) {
    // the Gram did not factor: the first table workgroup takes the whole table from the
    // pivoted QR of Blev (its dynamic LDS, 16 nblk rows of 17 doubles, holds the scratch), or,
    // without qr_work, a later launch takes it from elsewhere
    if (grp == 0 && a.qr_work)
      lev_qr_table(a.Blev, a.In_lev, P, a.qr_work, a.Q, a.status, (unsigned char*)lds, threadIdx.x, kThr);
    return;
  }
  const double* W = lev ? a.Wlev : a.Wsol;
  const double* Bsrc = lev ? a.Blev : a.Bsol;
  const int In = lev ? a.In_lev : a.In_sol;
  const int i0 = 16 * grp;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loops
  const int r16 = lane & 15, k4 = lane >> 4;
  double* Bs = lds;  // 16 nblk rows (p) x 16 columns (right-hand sides), stride kLdB
  // W operands.  Up to 8 blocks per row (P <= 128), all operands of a wave's products are held
  // in registers: the Y operands are loaded while the right-hand sides are staged (right after
  // their loads) and the Z operands before Y is exchanged, so that their memory latency overlaps
  // that work.  Larger P streams them one block ahead of the matrix cores.
  constexpr bool kHeld = T <= 2 && NW == 4;
  constexpr int kRing = 4;  // W blocks in flight per wave when streamed
  constexpr int kHB = kHeld ? 4 * T : 1;
  double wo[T][kHB][4];
  auto load_y_operands = [&]() {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int K = wave + NW * t;
      const double* Wr = W + (int64_t)slot(K < nblk ? K : 0, 0) * kBlk + r16 * kLd + k4;
#pragma unroll
      for (int J = 0; J < kHB; ++J)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) wo[t][J][ks] = (K < nblk && J <= K) ? Wr[(J <= K ? J : 0) * kBlk + 4 * ks] : 0.0;
    }
  };
  {
    // right-hand sides, transposed into Bs (one round of eight loads per thread up to P = 128);
    // all loads of a round are issued before any store.
    // W is read from memory by the products below: every workgroup shares it through L2, and
    // staging a copy per workgroup in LDS was measured slower (an extra round trip of up to 61 KB)
    const int cnt = 16 * nblk * 16;
    constexpr int kB = 8;
    for (int base = 0; base < cnt; base += kB * kThr) {
      double v[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int e = base + (int)threadIdx.x + kThr * q;
        const int j = e / (nblk * 16), p = e - j * (nblk * 16);
        const bool ok = e < cnt && i0 + j < In && p < P;
        v[q] = ok ? Bsrc[(int64_t)(i0 + j) * P + p] : 0.0;
      }
      // (one round when the operands are held: issued after the right-hand sides, whose
      // stores below then wait for those loads only)
      if constexpr (kHeld)
        if (base == 0) load_y_operands();
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int e = base + (int)threadIdx.x + kThr * q;
        const int j = e / (nblk * 16), p = e - j * (nblk * 16);
        if (e < cnt) Bs[p * kLdB + j] = v[q];
      }
    }
  }
  __syncthreads();
  // Y_K = sum_{J <= K} W_KJ B_J (blocks (K, 0 .. K) are consecutive slots)
  d4 Y[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int K = wave + NW * t;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    if (kHeld) {
#pragma unroll
      for (int J = 0; J < kHB; ++J)
        if (J <= K && K < nblk)
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) acc = mfma(wo[t][J][ks], Bs[(16 * J + 4 * ks + k4) * kLdB + r16], acc);
    } else if (K < nblk) {
      // blocks (K, 0 .. K) streamed through a ring of kRing blocks: kRing - 1 loads stay in
      // flight behind the block in use (clamped to block K past the end)
      const double* Wr = W + (int64_t)slot(K, 0) * kBlk + r16 * kLd + k4;
      double wb[kRing][4];
#pragma unroll
      for (int d = 0; d < kRing; ++d)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) wb[d][ks] = Wr[(d <= K ? d : K) * kBlk + 4 * ks];
      for (int J0 = 0; J0 <= K; J0 += kRing) {
#pragma unroll
        for (int d = 0; d < kRing; ++d) {
          const int J = J0 + d;
          if (J <= K)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) acc = mfma(wb[d][ks], Bs[(16 * J + 4 * ks + k4) * kLdB + r16], acc);
          const int Jn = J + kRing <= K ? J + kRing : K;
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) wb[d][ks] = Wr[Jn * kBlk + 4 * ks];
        }
      }
    }
    Y[t] = acc;
  }
  if (lev) {
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) s += Y[t][r] * Y[t][r];
    // lanes c, c + 16, c + 32, c + 48 hold four row groups of column c
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (lane < 16) s_red[wave][lane] = s;
    __syncthreads();
    if (threadIdx.x < 16 && i0 + (int)threadIdx.x < In) {
      const int j = threadIdx.x;
      double lv = s_red[0][j];
#pragma unroll
      for (int w = 1; w < NW; ++w) lv += s_red[w][j];  // in wave order
      a.Q[i0 + j] = (uint64_t)floor(lv / (double)P * 4503599627370496.0);  // 2^52
    }
    return;
  }
  // Z_K = sum_{J >= K} W_JK^T Y_J; blocks (J, K), J = K .. nblk-1, at slot(J + 1, K) =
  // slot(J, K) + J + 1
  const double* Wc = W + k4 * kLd + r16;
  if constexpr (kHeld) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int K = wave + NW * t;
      int sl = slot(K < nblk ? K : 0, K < nblk ? K : 0);
#pragma unroll
      for (int m = 0; m < kHB; ++m) {
        const bool in = K + m < nblk;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) wo[t][m][ks] = in ? Wc[(int64_t)sl * kBlk + 4 * ks * kLd] : 0.0;
        if (in) sl += K + m + 1;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int K = wave + NW * t;
    if (K < nblk)
#pragma unroll
      for (int r = 0; r < 4; ++r) Bs[(16 * K + 4 * r + k4) * kLdB + r16] = Y[t][r];
  }
  __syncthreads();
  const bool live = i0 + r16 < In;
  double* out = a.core + (int64_t)(i0 + r16) * P;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int K = wave + NW * t;
    if (K < nblk) {
      d4 acc = {0.0, 0.0, 0.0, 0.0};
      if (kHeld) {
#pragma unroll
        for (int m = 0; m < kHB; ++m)
          if (K + m < nblk)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
              acc = mfma(wo[t][m][ks], Bs[(16 * (K + m) + 4 * ks + k4) * kLdB + r16], acc);
      } else {
        // blocks (K .. nblk-1, K) through the same ring; block (J, K) is at slot(J, K), and
        // slot(J + 1, K) = slot(J, K) + J + 1
        double wb[kRing][4];
        int sl = slot(K, K), Jl = K;  // next block to load and its slot
#pragma unroll
        for (int d = 0; d < kRing; ++d) {
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) wb[d][ks] = Wc[(int64_t)sl * kBlk + 4 * ks * kLd];
          if (Jl + 1 < nblk) {
            sl += Jl + 1;
            ++Jl;
          }
        }
        for (int J0 = K; J0 < nblk; J0 += kRing) {
#pragma unroll
          for (int d = 0; d < kRing; ++d) {
            const int J = J0 + d;
            if (J < nblk)
#pragma unroll
              for (int ks = 0; ks < 4; ++ks)
                acc = mfma(wb[d][ks], Bs[(16 * J + 4 * ks + k4) * kLdB + r16], acc);
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) wb[d][ks] = Wc[(int64_t)sl * kBlk + 4 * ks * kLd];
            if (Jl + 1 < nblk) {
              sl += Jl + 1;
              ++Jl;
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = 16 * K + 4 * r + k4;
        if (live && p < P) out[p] = acc[r];
      }
    }
  }
  if (a.last_counter && *a.core_fail) {
    // The table's Gram broke down (known before this launch, the same for every workgroup): the
    // solve workgroup that finishes last (fence, then a counter: every other workgroup's rows are
    // written and visible) takes the new core's table from its pivoted QR and resets the counter.
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(a.last_counter, 1) == a.solve_groups - 1;
    __syncthreads();
    if (s_last) {
      __threadfence();
      lev_qr_table(a.core, a.In_sol, P, a.fallback_work, a.Q, a.status, (unsigned char*)lds, threadIdx.x, kThr);
      if (threadIdx.x == 0) *a.last_counter = 0;
    }
  }
}

// ---------------------------------------------------------------------------------------
// The solve for P > 128 in two launches.  On one compute unit a 16-row group's 2 nblk (nblk +
// 1) / 2 block products take longer than the FP64 matrix cores allow for the whole solve, and
// a few groups leave most units idle; here each group is spread over sp.n workgroups per half:
//   kZ = false: Y_K = sum_{J <= K} W_KJ B_J for the block rows K of the part, into Ys;
//   kZ = true:  Z_K = sum_{J >= K} W_JK^T Y_J for the block rows K of the part (Y_J from Ys),
//               written as rows of the core.
// Parts are contiguous ranges of K, [sp.lo[p], sp.lo[p + 1]), of about equal product counts;
// wave w takes K = lo + w, lo + w + 16, ...  Every block product and its order are those of
// k_trisolve.  Ys: group g's block K at (g nblk + K) 256 doubles, entry (i, j) = Y_K(i, j)
// (row i of the block row, right-hand side j).
struct SolveParts {
  int n;
  int lo[kMaxSolveParts + 1];
};

template <bool kZ>
__global__ __launch_bounds__(1024) void k_solve_half(TriArgs a, SolveParts sp) {
  constexpr int NW = 16, kThr = 64 * NW, kLdB = 17, kRing = 4;
  extern __shared__ double lds[];
  if (*a.status != kDevOk) return;
  const int P = a.P, nblk = (P + 15) / 16, In = a.In_sol;
  const int g = (int)blockIdx.x / sp.n, part = (int)blockIdx.x - g * sp.n;
  const int klo = sp.lo[part], khi = sp.lo[part + 1];
  const int i0 = 16 * g;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, k4 = lane >> 4;
  double* Bs = lds;  // 16 nblk rows (p) x 16 columns (right-hand sides), stride kLdB
  double* Ys = a.split_work + (int64_t)g * nblk * 256;
  const double* W = a.Wsol;
  // operands: B_J for J < khi (rows of B transposed), or Y_J for J >= klo (from Ys); all loads
  // of a round issued before any store
  {
    const int j0 = kZ ? klo : 0, j1 = kZ ? nblk : khi;
    const int cnt = 256 * (j1 - j0);
    constexpr int kB = 8;
    for (int base = 0; base < cnt; base += kB * kThr) {
      double v[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int e = base + (int)threadIdx.x + kThr * q;
        double x = 0.0;
        if (e < cnt) {
          if (kZ) {
            x = Ys[(int64_t)j0 * 256 + e];  // entry (i, j) of block j0 + e / 256
          } else {
            const int j = e / (16 * (j1 - j0)), p = e - j * (16 * (j1 - j0));  // row j of the group, column p
            if (i0 + j < In && p < P) x = a.Bsol[(int64_t)(i0 + j) * P + p];
          }
        }
        v[q] = x;
      }
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int e = base + (int)threadIdx.x + kThr * q;
        if (e < cnt) {
          if (kZ) {
            const int blk = j0 + e / 256, ij = e & 255;
            Bs[(16 * blk + (ij >> 4)) * kLdB + (ij & 15)] = v[q];
          } else {
            const int j = e / (16 * (j1 - j0)), p = e - j * (16 * (j1 - j0));
            Bs[p * kLdB + j] = v[q];
          }
        }
      }
    }
  }
  __syncthreads();
  for (int K = klo + wave; K < khi; K += NW) {
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    double wb[kRing][4];
    if (!kZ) {
      // blocks (K, 0 .. K) through a ring of kRing blocks (as in k_trisolve)
      const double* Wr = W + (int64_t)slot(K, 0) * kBlk + r16 * kLd + k4;
#pragma unroll
      for (int d = 0; d < kRing; ++d)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) wb[d][ks] = Wr[(d <= K ? d : K) * kBlk + 4 * ks];
      for (int J0 = 0; J0 <= K; J0 += kRing) {
#pragma unroll
        for (int d = 0; d < kRing; ++d) {
          const int J = J0 + d;
          if (J <= K)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) acc = mfma(wb[d][ks], Bs[(16 * J + 4 * ks + k4) * kLdB + r16], acc);
          const int Jn = J + kRing <= K ? J + kRing : K;
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) wb[d][ks] = Wr[Jn * kBlk + 4 * ks];
        }
      }
      // D(i, j) in lane j + 16 (i % 4), register i / 4
#pragma unroll
      for (int r = 0; r < 4; ++r) Ys[(int64_t)K * 256 + (4 * r + k4) * 16 + r16] = acc[r];
    } else {
      // blocks (K .. nblk-1, K); block (J, K) at slot(J, K), slot(J + 1, K) = slot(J, K) + J + 1
      const double* Wc = W + k4 * kLd + r16;
      int sl = slot(K, K), Jl = K;
#pragma unroll
      for (int d = 0; d < kRing; ++d) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) wb[d][ks] = Wc[(int64_t)sl * kBlk + 4 * ks * kLd];
        if (Jl + 1 < nblk) {
          sl += Jl + 1;
          ++Jl;
        }
      }
      for (int J0 = K; J0 < nblk; J0 += kRing) {
#pragma unroll
        for (int d = 0; d < kRing; ++d) {
          const int J = J0 + d;
          if (J < nblk)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) acc = mfma(wb[d][ks], Bs[(16 * J + 4 * ks + k4) * kLdB + r16], acc);
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) wb[d][ks] = Wc[(int64_t)sl * kBlk + 4 * ks * kLd];
          if (Jl + 1 < nblk) {
            sl += Jl + 1;
            ++Jl;
          }
        }
      }
      const bool live = i0 + r16 < In;
      double* out = a.core + (int64_t)(i0 + r16) * P;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int p = 16 * K + 4 * r + k4;
        if (live && p < P) out[p] = acc[r];
      }
    }
  }
}

// contiguous ranges of block rows with about equal product counts: block row K costs K + 1
// products in the first half, nblk - K in the second
SolveParts solve_parts(int nblk, int n, bool second) {
  SolveParts sp;
  sp.n = n;
  const int64_t total = (int64_t)nblk * (nblk + 1) / 2;
  int K = 0;
  int64_t acc = 0;
  sp.lo[0] = 0;
  for (int p = 1; p < n; ++p) {
    const int64_t target = total * p / n;
    while (K < nblk && acc + (second ? nblk - K : K + 1) <= target) acc += second ? nblk - K : K + 1, ++K;
    sp.lo[p] = K;
  }
  sp.lo[n] = nblk;
  return sp;
}

// ---------------------------------------------------------------------------------------
// Table of a wide core (I <= P) in one workgroup: the row Gram K = G G^T (lower blocks, into
// a.K), its factorisation in LDS with the table tolerance, then the uniform table if it
// factored, else the pivoted-QR table.
template <int kW>
__device__ __forceinline__ void lev_wide_body(const LevWideArgs& a, const CholArgs& ca) {
  extern __shared__ double lw_smem[];
  __shared__ int s_wide_fail;
  if (*a.status != kDevOk || (a.run_if && *a.run_if == 0)) return;
  const int I = a.I, P = a.P;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar loops
  const int r16 = lane & 15, k4 = lane >> 4;
  const int nb = (I + 15) / 16, nslots = nb * (nb + 1) / 2;
  if (threadIdx.x == 0) s_wide_fail = 0;
  // Gram blocks: with fewer blocks than waves, kparts waves share a block, each taking every
  // kparts-th 4-column k-step, and their sums are added in part order
  const int kparts = nslots >= kW ? 1 : kW / nslots;
  const int part = wave % kparts, nwork = (kW / kparts) * kparts;
  double* red = lw_smem;  // kW partial blocks (16 x 17 doubles each)
  for (int sl0 = 0; sl0 < nslots; sl0 += kW / kparts) {
    const int sl = sl0 + wave / kparts;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    int bi = 0, bj = 0;
    if (wave < nwork && sl < nslots) {
      slot_ij(sl, bi, bj);
      const int ri = 16 * bi + r16, rj = 16 * bj + r16;
      const double* gi = a.G + (int64_t)(ri < I ? ri : I - 1) * P;
      const double* gj = a.G + (int64_t)(rj < I ? rj : I - 1) * P;
      const double mi = ri < I ? 1.0 : 0.0;
      // D(i, j) = sum_p G(16 bi + i, p) G(16 bj + j, p): A(i, k) in lane i + 16 k, B(k, j) in
      // lane j + 16 k, both read along a row of G; four k-steps' loads in flight
      for (int p0 = 4 * part; p0 < P; p0 += 16 * kparts) {
        double va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int pp = p0 + 4 * kparts * u + k4;
          va[u] = pp < P ? mi * gi[pp] : 0.0;
          vb[u] = pp < P ? gj[pp] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = mfma(va[u], vb[u], acc);
      }
    }
    if (kparts > 1) {
      store_acc(red + wave * kBlk, acc, lane);
      __syncthreads();
      if (wave < nwork && part == 0 && sl < nslots) {
        for (int q2 = 1; q2 < kparts; ++q2) {
          const d4 o = load_acc(red + (wave + q2) * kBlk, lane);
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] += o[q];
        }
      }
      __syncthreads();
    }
    if (wave < nwork && part == 0 && sl < nslots)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * bi + 4 * q + k4, col = 16 * bj + r16;
        if (row < I && col < I) a.K[(int64_t)row * I + col] = acc[q];
      }
  }
  __syncthreads();
  CholArgs c = ca;
  c.fail = &s_wide_fail;
  const bool ok = chol_body<false, kW>(c);
  __syncthreads();
  if (ok) {
    const double pr = 1.0 / (double)I;  // full row rank: p_i = l_i / rank = 1 / I
    const uint64_t q = (uint64_t)floor(pr * 4503599627370496.0);
    for (int i = threadIdx.x; i < I; i += 64 * kW) a.Q[i] = q;
  } else if (a.qr_work) {
    lev_qr_table(a.G, I, P, a.qr_work, a.Q, a.status, (unsigned char*)lw_smem, threadIdx.x, 64 * kW);
  }
  // without qr_work the breakdown is only reported (a later launch takes the table)
  if (!a.qr_work && threadIdx.x == 0) *a.fail = ok ? 0 : 1;
}

template <int kW>
__global__ __launch_bounds__(64 * kW) void k_lev_wide(LevWideArgs a, CholArgs ca) {
  lev_wide_body<kW>(a, ca);
}

// Two independent single-workgroup jobs in one launch: workgroup 0 factors a0; workgroup 1
// factors a1, or (wide = 1) takes the table of the wide matrix of lw as k_lev_wide does.
template <int kW>
__global__ __launch_bounds__(64 * kW) void k_chol_pair(CholArgs a0, CholArgs a1, LevWideArgs lw, int wide,
                                                        int* clear) {
  if (clear && blockIdx.x == 0 && threadIdx.x == 0) *clear = 0;
  if (blockIdx.x == 1 && wide) {
    lev_wide_body<kW>(lw, a1);
    return;
  }
  chol_body<false, kW>(blockIdx.x == 0 ? a0 : a1);
}

// Table from the breakdown word of a factorisation run before: uniform if it factored (a wide
// core's row Gram), else the pivoted QR of G.
__global__ __launch_bounds__(1024) void k_lev_fallback(const double* __restrict__ G, int I, int P,
                                                       double* __restrict__ qr_work, uint64_t* __restrict__ Q,
                                                       const int* fail, int* status) {
  extern __shared__ unsigned char lf_smem[];
  if (*status != kDevOk) return;
  if (*fail == 0) {
    const double pr = 1.0 / (double)I;
    const uint64_t q = (uint64_t)floor(pr * 4503599627370496.0);
    for (int i = threadIdx.x; i < I; i += 1024) Q[i] = q;
    return;
  }
  lev_qr_table(G, I, P, qr_work, Q, status, lf_smem, threadIdx.x, 1024);
}

hipError_t trisolve_dispatch(const TriArgs& a, int nblk, unsigned grid, size_t lds, hipStream_t s) {
  // four waves with every W operand in registers up to 8 blocks; beyond, sixteen waves (one or
  // a few block rows each: the chains of dependent block products are spread over the CU)
  if (nblk <= 4) k_trisolve<1, 4><<<grid, 256, lds, s>>>(a);
  else if (nblk <= 8) k_trisolve<2, 4><<<grid, 256, lds, s>>>(a);
  else if (nblk <= 16) k_trisolve<1, 16><<<grid, 1024, lds, s>>>(a);
  else if (nblk <= 32) k_trisolve<2, 16><<<grid, 1024, lds, s>>>(a);
  else k_trisolve<4, 16><<<grid, 1024, lds, s>>>(a);
  return hipGetLastError();
}

}  // namespace

size_t chol_factor_doubles(int P) {
  const int nblk = (P + 15) / 16;
  return (size_t)nblk * (nblk + 1) / 2 * kBlk;
}

size_t chol_work_doubles(int P) {
  const int nblk = (P + 15) / 16;
  if (nblk <= kLdsBlocks) return chol_factor_doubles(P) + (size_t)nblk * kBlk;  // W + staging blocks
  return 3 * chol_factor_doubles(P) + 8;  // W, work matrix, panel blocks L, tolerance
}

hipError_t launch_syrk(const double* A, int64_t rows, int P, double* Kout, const int* status, hipStream_t s,
                       bool trans, int* clear, bool packed) {
  const int nblk = (P + 15) / 16;
  if (nblk > kMaxBlk || rows < 1 || (packed && P % 16)) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)(nblk * (nblk + 1) / 2);
  if (trans)
    k_syrk<true><<<grid, 64 * kSyrkWaves, 0, s>>>(A, rows, P, Kout, status, clear, packed ? 1 : 0);
  else
    k_syrk<false><<<grid, 64 * kSyrkWaves, 0, s>>>(A, rows, P, Kout, status, clear, packed ? 1 : 0);
  return hipGetLastError();
}

bool chol_single_workgroup(int P) { return (P + 15) / 16 <= kLdsBlocks; }

hipError_t launch_chol(const CholArgs& args, hipStream_t s, const ReduceJob* beside, int nparts) {
  const int nblk = (args.P + 15) / 16;
  if (nblk > kMaxBlk) return hipErrorInvalidValue;
  if (beside && !chol_single_workgroup(args.P)) return hipErrorInvalidValue;
  if (nblk <= kLdsBlocks) {
    const size_t lds = chol_work_doubles(args.P) * sizeof(double);
    // eight waves for up to four blocks (the panel steps dominate; fewer waves share a SIMD
    // with the panel wave), sixteen above
    const bool small = nblk <= 4;
    if (beside && beside->count > 0) {
      const int64_t nred = reduce_blocks(*beside, args.P, nparts);
      if (small)
        k_chol_reduce<8><<<(unsigned)(1 + (nred + 1) / 2), 512, lds, s>>>(args, *beside, nparts);
      else
        k_chol_reduce<16><<<(unsigned)(1 + (nred + 3) / 4), 1024, lds, s>>>(args, *beside, nparts);
    } else if (small) {
      k_chol<false, 8><<<1, 512, lds, s>>>(args);
    } else {
      k_chol<false, 16><<<1, 1024, lds, s>>>(args);
    }
    return hipGetLastError();
  }
  CholArgs a = args;
  a.Lg = a.W + chol_factor_doubles(a.P);
  a.Lp = a.W + 2 * chol_factor_doubles(a.P);
  a.scal = a.W + 3 * chol_factor_doubles(a.P);
  const int nslots = nblk * (nblk + 1) / 2;
  if (a.prepacked && !chol_prepack_ok(a.P)) return hipErrorInvalidValue;
  if (!a.prepacked)
    k_big_init<<<(unsigned)((nslots * kBlk + 255) / 256 < 1024 ? (nslots * kBlk + 255) / 256 : 1024), 256, 0, s>>>(
        a.H, a.P, a.Lg, a.scal, a.status, a.fail ? a.fail : a.status, a.rel_tol);
  const int nb64 = (nblk + 3) / 4;
  for (int K = 0; K < nb64; ++K) {
    a.b0 = 4 * K;
    a.nb = nblk - a.b0 < 4 ? nblk - a.b0 : 4;
    a.pb0 = K > 0 ? a.b0 - 4 : 0;  // every region but the last has four blocks
    a.pnb = K > 0 ? 4 : 0;
    // region blocks, staging blocks, the previous step's panel rows of the region, and that
    // panel's operands (the step's inverse diagonal blocks, the region's rows of its columns)
    size_t lds = ((size_t)a.nb * (a.nb + 1) / 2 + a.nb + 2 * (size_t)a.nb * a.pnb + (size_t)a.pnb * (a.pnb + 1) / 2) *
                 kBlk * sizeof(double);  // at most kRegionLdsBytes
    if (K == 0) {
      k_chol<true, kCholWaves><<<1, 64 * kCholWaves, lds, s>>>(a);
    } else {
      // band K - 1 of W: 4 (K - 1) workgroups (none when only the factor's regions are needed)
      const int band = (K >= 2 && !a.factor_only) ? K - 1 : 0;
      if (band > 0 && lds < kWrowLdsBytes) lds = kWrowLdsBytes;
      const int rem = nblk - a.b0;
      const int tgroups = (rem * (rem + 1) / 2 + kCholWaves - 1) / kCholWaves;
      k_chol_step<<<(unsigned)(1 + 4 * band + tgroups), 64 * kCholWaves, lds, s>>>(a, band);
    }
  }
  if (nb64 >= 2 && !a.factor_only)
    k_big_wrow<<<(unsigned)(4 * (nb64 - 1)), 64 * kCholWaves, kWrowLdsBytes, s>>>(a.Lp, a.W, nblk, nb64 - 1, a.status,
                                                                               a.fail);
  return hipGetLastError();
}

hipError_t launch_lev_fallback(const double* G, int I, int P, double* qr_work, uint64_t* Q, const int* fail,
                               int* status, hipStream_t s) {
  k_lev_fallback<<<1, 1024, lev_qr_smem_bytes(P), s>>>(G, I, P, qr_work, Q, fail, status);
  return hipGetLastError();
}

namespace {

// the row-Gram factorisation of a wide table: only the breakdown matters, not W's bands
CholArgs wide_chol_args(const LevWideArgs& a) {
  CholArgs ca;
  memset(&ca, 0, sizeof(ca));
  ca.P = a.I;
  ca.H = a.K;
  ca.W = a.F;
  ca.status = a.status;
  ca.fail = a.fail;
  ca.rel_tol = a.rel_tol;
  ca.factor_only = 1;
  return ca;
}

// dynamic LDS of a single-workgroup wide table with kW waves
size_t wide_lds(const LevWideArgs& a, int kW) {
  const size_t need = chol_work_doubles(a.I) * sizeof(double);
  const size_t qr = lev_qr_smem_bytes(a.P);
  const size_t red = (size_t)kW * kBlk * sizeof(double);  // Gram partial blocks
  size_t lds = need > qr ? need : qr;
  return lds > red ? lds : red;
}

}  // namespace

hipError_t launch_chol_pair(const CholArgs& a0, const CholArgs* a1, const LevWideArgs* lw, hipStream_t s,
                            int* clear) {
  if ((a1 == nullptr) == (lw == nullptr) || !chol_single_workgroup(a0.P)) return hipErrorInvalidValue;
  if (a1 && !chol_single_workgroup(a1->P)) return hipErrorInvalidValue;
  if (lw && (lw->I > lw->P || lw->I < 1 || !chol_single_workgroup(lw->I) || (lw->P + 15) / 16 > kMaxBlk))
    return hipErrorInvalidValue;
  const int n0 = (a0.P + 15) / 16, n1 = a1 ? (a1->P + 15) / 16 : (lw->I + 15) / 16;
  const int kW = (n0 <= 4 && n1 <= 4) ? 8 : 16;
  size_t lds = chol_work_doubles(a0.P) * sizeof(double);
  CholArgs c1;
  LevWideArgs l1;
  memset(&l1, 0, sizeof(l1));
  if (a1) {
    c1 = *a1;
    const size_t b = chol_work_doubles(a1->P) * sizeof(double);
    lds = b > lds ? b : lds;
  } else {
    l1 = *lw;
    c1 = wide_chol_args(*lw);
    const size_t b = wide_lds(*lw, kW);
    lds = b > lds ? b : lds;
  }
  if (kW == 8)
    k_chol_pair<8><<<2, 512, lds, s>>>(a0, c1, l1, lw ? 1 : 0, clear);
  else
    k_chol_pair<16><<<2, 1024, lds, s>>>(a0, c1, l1, lw ? 1 : 0, clear);
  return hipGetLastError();
}

hipError_t launch_lev_wide(const LevWideArgs& a, hipStream_t s) {
  if (a.I > a.P || a.I < 1 || (a.P + 15) / 16 > kMaxBlk) return hipErrorInvalidValue;
  const CholArgs ca = wide_chol_args(a);
  if (chol_single_workgroup(a.I)) {
    const bool small = (a.I + 15) / 16 <= 4;
    const size_t lds = wide_lds(a, small ? 8 : 16);
    if (small)
      k_lev_wide<8><<<1, 512, lds, s>>>(a, ca);
    else
      k_lev_wide<16><<<1, 1024, lds, s>>>(a, ca);
    return hipGetLastError();
  }
  // K = G G^T (G's storage read as the column-major P x I matrix G^T), blocked factorisation
  // with the breakdown word, then the table
  hipError_t e = launch_syrk(a.G, a.P, a.I, a.K, a.status, s, /*trans=*/true, a.fail);
  if (e != hipSuccess) return e;
  e = launch_chol(ca, s);
  if (e != hipSuccess) return e;
  return launch_lev_fallback(a.G, a.I, a.P, a.qr_work, a.Q, a.fail, a.status, s);
}

bool chol_prepack_ok(int P) { return !chol_single_workgroup(P) && P % 16 == 0 && (P + 15) / 16 <= kMaxBlk; }
double* chol_packed_input(double* W, int P) { return W + chol_factor_doubles(P); }

size_t solve_split_doubles(int In, int P) { return (size_t)((In + 15) / 16) * ((P + 15) / 16) * 256; }

hipError_t launch_trisolve(const TriArgs& args, hipStream_t s) {
  TriArgs a = args;
  const int nblk = (a.P + 15) / 16;
  if (nblk > kMaxBlk) return hipErrorInvalidValue;
  if (a.split_work && a.Wsol && !a.Wlev && !a.last_counter && nblk > 8 && a.In_sol > 0) {
    // about 1.5 workgroups per compute unit in each half (measured best over 1, 1.5, 2 and 4 at
    // P = 400, 2000 rows), at most kMaxSolveParts per group
    const int groups = (a.In_sol + 15) / 16;
    int n = (3 * kPlanCUs / 2 + groups - 1) / groups;
    n = n < 1 ? 1 : n > kMaxSolveParts ? kMaxSolveParts : n > nblk ? nblk : n;
    const unsigned grid = (unsigned)(groups * n);
    const SolveParts p1 = solve_parts(nblk, n, false), p2 = solve_parts(nblk, n, true);
    // staged blocks are indexed by their block row: room for all nblk (at most 139 KB)
    const size_t lds = (size_t)nblk * 16 * 17 * sizeof(double);
    k_solve_half<false><<<grid, 1024, lds, s>>>(a, p1);
    k_solve_half<true><<<grid, 1024, lds, s>>>(a, p2);
    return hipGetLastError();
  }
  a.solve_groups = a.Wsol ? (a.In_sol + 15) / 16 : 0;
  a.lev_groups = a.Wlev ? (a.In_lev + 15) / 16 : 0;
  const unsigned grid = (unsigned)(a.solve_groups + a.lev_groups);
  if (grid == 0) return hipSuccess;
  const size_t lds = (size_t)nblk * 16 * 17 * sizeof(double);
  return trisolve_dispatch(a, nblk, grid, lds, s);
}

}  // namespace trals
