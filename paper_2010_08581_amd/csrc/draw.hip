// Sampler and sketch of one core update, fused (Algorithm 3 draws, Definition 5 rescaling,
// Algorithm 4 / eq. (5) subchain rows).  The same kernel forms the rows for given index tuples
// (the true-core rows of a generated source) and, enumerating every tuple, the full design
// matrix G^{!=n}_[2] of Algorithm 1 (exact TR-ALS).
//
// Tables.  The device tables hold either the integer weights Q_i (then every workgroup forms
// the inclusive sums C in LDS while staging them) or the sums C themselves (problems whose
// tables exceed the LDS budget; searched in global memory).
//
// Draws.  Sample j, mode draw k (mode m = (n+1+k) mod N) takes 64-bit word (k mod 4) of the
// Philox4x64-10 block with key (seed, stream_id) and counter (j, k/4, u, 0), u the update
// number.  With the mode's inclusive integer table C (total T = C[I-1]) the draw is
// t = floor(r T / 2^64) (high word of the 128-bit product) and i = min{i : t < C_i}, found by
// binary search; zero-weight entries are never drawn.  The rescaling is w = 1/sqrt(J q) with
// q = prod_k Q_{i_k} / T_k the exact probability of the tuple, multiplied in FP64 in k order.
//
// Sketch.  Row j is w_j times the product of the sampled lateral slices
// G^(m_0)(:, i_{m_0}, :) ... G^(m_{N-2})(:, i_{m_{N-2}}, :) (an R_n x R_{n-1} matrix M_j),
// stored with column a*R_n + b holding w_j M_j(b, a).  (This column order is a permutation
// of the paper's a + R_{n-1} b; it makes the solution columns the lateral slices of the new
// core in slice-major storage.)  FP64 and FP32 sketches: products in FP64 from the FP64 cores,
// the row rounded once to the sketch type.  BF16 sketch (the BF16 form): products on BF16
// matrix cores with FP32 accumulation, every operand (slice or partial product) a pair of BF16
// values, hi + lo, so that each product carries about 16 bits.
//
// A workgroup stages the tables once (in LDS when they fit) and then takes batches of jb
// samples, gridDim.x batches apart: one thread per sample and table draws, then thread (s, b)
// carries row b of M_s through the chain, the slices of all jb samples staged in LDS (loads
// batched, one round trip per kB per thread), and the finished rows leave through LDS as one
// contiguous store.
#include <type_traits>

#include "kernels.h"

namespace trals {

namespace {

constexpr int kThreads = 256;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// BF16 form: chain products on BF16 matrix cores.  One wave per sample keeps D = M^T of its
// chain as kT x kT tiles of 16 x 16 FP32 accumulators (kT = 1 for ranks up to 16, 2 up to 32);
// at most kChainSPW(RM) samples per wave, so a workgroup holds 4 kChainSPW(RM) samples.
__host__ __device__ constexpr int kChainT(int rm) { return rm <= 16 ? 1 : 2; }
__host__ __device__ constexpr int kChainSPW(int rm) { return rm <= 16 ? 8 : 4; }
constexpr size_t kDrawLdsBytes = 160 * 1024;  // LDS per compute unit

// inclusive prefix sums of t[0, n) in place (kThreads threads: contiguous chunks per thread,
// a shuffle scan of the chunk sums per wave, then the wave totals)
__device__ void lds_scan_u64(uint64_t* t, int n, uint64_t* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = (n + kThreads - 1) / kThreads;
  const int b0 = tid * c < n ? tid * c : n, b1 = b0 + c < n ? b0 + c : n;
  uint64_t s = 0;
  for (int i = b0; i < b1; ++i) s += t[i];
  uint64_t x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint64_t pre = x - s;
  for (int w = 0; w < wave; ++w) pre += wsum[w];
  for (int i = b0; i < b1; ++i) {
    pre += t[i];
    t[i] = pre;
  }
  __syncthreads();
}

// Staged slices: row stride kRowLd(RM) (even, >= RM) and one slot of kSliceLd(RM) doubles per
// sample (even, so every row starts on 16 bytes; slots RM^2 + 2 doubles apart fall on distinct
// LDS banks for the instance sizes).
__host__ __device__ constexpr int kRowLd(int RM) { return (RM + 1) & ~1; }
__host__ __device__ constexpr int kSliceLd(int RM) { return RM * kRowLd(RM) + 2; }

template <typename TA, int RM, bool CHAIN>
__global__ __launch_bounds__(kThreads) void k_draw(DrawArgs a) {
  __shared__ uint64_t s_wsum[kThreads / 64];
  extern __shared__ __align__(16) double lds[];
  if (*a.status != kDevOk) return;
  const int N = a.ring.N;
  const int K = N - 1;
  const int n = a.n;
  const int jb = a.jb;
  constexpr int kSlice = kSliceLd(RM), kLdR = kRowLd(RM);
  static_assert(RM % 2 == 0, "slice rows are read as pairs");
  constexpr int kB = 16;               // loads in flight per thread while staging
  double* S = lds;                                    // jb * kSlice
  double* s_w = S + (size_t)jb * kSlice;              // jb
  int32_t* s_idx = (int32_t*)(s_w + jb);              // jb * K (padded to even)
  double* s_p = s_w + jb + (jb * K + 1) / 2;          // jb * K: probability of each draw
  uint64_t* tab = (uint64_t*)(s_p + jb * K);
  const int tid = threadIdx.x;

  // ---- draws ----
  int off[kMaxOrder];
  if (a.draw && a.tables_in_lds) {
    // The K tables are concatenated in LDS (table k at off[k]).  A wave copies 64-entry pieces,
    // table and offset wave-uniform, eight pieces in flight, so all tables cost about one
    // memory round trip.  With weights, one inclusive scan over the concatenation gives every
    // table's sums offset by the total of the tables before it (exact in integers); the search
    // below subtracts that base.
    int o = 0, pieces = 0;
    int first_piece[kMaxOrder];
    for (int k = 0; k < K; ++k) {
      int m = n + 1 + k;
      if (m >= N) m -= N;
      off[k] = o;
      first_piece[k] = pieces;
      o += a.ring.dims[m];
      pieces += (a.ring.dims[m] + 63) / 64;
    }
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    constexpr int kQ = 8;
    for (int p0 = wave; p0 < pieces; p0 += 4 * kQ) {
      uint64_t v[kQ];
      int dst[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int pc = p0 + 4 * q;
        int k = 0;
        while (k + 1 < K && pc >= first_piece[k + 1]) ++k;
        int m = n + 1 + k;
        if (m >= N) m -= N;
        const int e = (pc - first_piece[k]) * 64 + lane;
        const bool ok = pc < pieces && e < a.ring.dims[m];
        v[q] = ok ? a.cdf.p[m][ok ? e : 0] : 0ull;
        dst[q] = ok ? off[k] + e : -1;
      }
#pragma unroll
      for (int q = 0; q < kQ; ++q)
        if (dst[q] >= 0) tab[dst[q]] = v[q];
    }
    __syncthreads();
    if (a.weights) lds_scan_u64(tab, o, s_wsum);
  }
  // batches of jb samples, gridDim.x apart (the tables above are staged once per workgroup)
  const int64_t nbatch = (a.J + jb - 1) / jb;
  for (int64_t batch = blockIdx.x; batch < nbatch; batch += gridDim.x) {
  const int64_t j0 = batch * jb;
  if (tid < jb && !a.draw) {
    // given samples (same rows, no rescaling), or every index tuple in panel-row order
    const int64_t j = j0 + tid;
    for (int k = 0; k < K; ++k) {
      int v = 0;
      if (j < a.J) {
        if (a.enumerate) {
          int m = n + 1 + k;
          if (m >= N) m -= N;
          v = (int)((j / a.en_stride[k]) % a.ring.dims[m]);
        } else {
          v = a.idx[j * K + k];
        }
      }
      s_idx[tid * K + k] = v;
    }
    s_w[tid] = j < a.J ? 1.0 : 0.0;
    if (a.enumerate && j < a.J) a.w[j] = 1.0;
  } else if (a.draw) {
    // one thread per (sample, table), consecutive threads on consecutive samples of one table:
    // draw k of sample j is word k mod 4 of Philox block (j, k / 4); its probability goes to
    // s_p, and the weight is formed after the next barrier, in table order
    for (int e = tid; e < jb * K; e += kThreads) {
      const int sl = e % jb, k = e / jb;
      const int64_t j = j0 + sl;
      if (j >= a.J) {
        s_idx[sl * K + k] = 0;
        continue;
      }
      {
        uint64_t x[4] = {(uint64_t)j, (uint64_t)(k >> 2), a.u, 0};
        philox4x64_10(x, a.seed, a.stream_id);
        const int word = k & 3;
        const uint64_t r = word == 0 ? x[0] : word == 1 ? x[1] : word == 2 ? x[2] : x[3];
        int m = n + 1 + k;
        if (m >= N) m -= N;
        const uint64_t* C = a.tables_in_lds ? tab + off[k] : a.cdf.p[m];
        // base: the total of the tables before table k in the concatenated scan (else 0)
        const uint64_t base = (a.tables_in_lds && a.weights && k > 0) ? C[-1] : 0ull;
        const int I = a.ring.dims[m];
        const uint64_t T = C[I - 1] - base;
        const uint64_t t = __umul64hi(r, T) + base;
        int lo = 0, hi = I - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (C[mid] > t) hi = mid;
          else lo = mid + 1;
        }
        const uint64_t Qi = C[lo] - (lo > 0 ? C[lo - 1] : base);
        s_p[sl * K + k] = (double)Qi / (double)T;
        s_idx[sl * K + k] = lo;
        a.idx[j * K + k] = lo;
      }
    }
  }

  // ---- subchain rows ----
  const int Rn = a.ring.ranks[n];
  const int sj = tid / Rn, b = tid - sj * Rn;
  const bool live = sj < jb;
  double row[RM];
#pragma unroll
  for (int c = 0; c < RM; ++c) row[c] = 0.0;
  // BF16 form: the transposed chain D_0 = S_0^T, D_k = S_k^T D_{k-1} on BF16 matrix cores with
  // FP32 accumulation (D_{K-1} = M^T).  A D tile's accumulator layout, row 4 (lane / 16) + r and
  // column lane % 16, is the B operand of the next product when the 32 reduction slots of the
  // 16 x 16 x 32 instruction are numbered so that lane group g's eight slots are rows 4g .. 4g + 3
  // and 16 + 4g .. 16 + 4g + 3; the A operand (the slice, transposed) takes the same numbering.
  constexpr bool kMfmaChain = CHAIN && std::is_same<TA, __bf16>::value;
  constexpr int kT = kChainT(RM), kSPW = kMfmaChain ? kChainSPW(RM) : 1;
  const int lane = tid & 63, wave = tid >> 6, l16 = lane & 15, l4 = lane >> 4;
  f4 D[kSPW][kT][kT];
#pragma unroll
  for (int q = 0; q < kSPW; ++q)
#pragma unroll
    for (int tr = 0; tr < kT; ++tr)
#pragma unroll
      for (int tc = 0; tc < kT; ++tc) D[q][tr][tc] = f4{0.f, 0.f, 0.f, 0.f};
  int rin = Rn;
  for (int k = 0; k < K; ++k) {
    int m = n + 1 + k;
    if (m >= N) m -= N;
    const int rout = a.ring.ranks[m];
    const int ssz = rin * rout;
    const double* core = a.cores.p[m];
    __syncthreads();  // draws visible / previous slices consumed
    if (k == 0 && a.draw && tid < jb) {
      // w = 1 / sqrt(J q), q the product of the sample's draw probabilities in table order
      // (s_w is read by the sketch store only)
      const int64_t j = j0 + tid;
      double q = 1.0;
      for (int kk = 0; kk < K; ++kk) q = q * s_p[tid * K + kk];
      const double w = j < a.J ? 1.0 / sqrt((double)a.J * q) : 0.0;
      s_w[tid] = w;
      if (j < a.J) a.w[j] = w;
    }
    // stage the jb slices (rin x rout each, contiguous in slice-major storage) with row stride
    // kLdR.  Element e is sample e / ssz, entry o = e mod ssz, row o / rout; the quotients come
    // from float reciprocals, exact here (e < 256 ssz and o < 32^2: the rounding stays below
    // the distance of (e + 1/2)/ssz, (o + 1/2)/rout from an integer; checked for every ssz <= 32^2)
    const int tot = jb * ssz;
    const float rs = 1.0f / (float)ssz, rr = 1.0f / (float)rout;
    for (int base = 0; base < tot; base += kB * kThreads) {
      double v[kB];
      int dst[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        v[q] = 0.0;
        dst[q] = -1;
        // a sub-round wholly past the end is skipped (the test is uniform across the workgroup)
        if (base + kThreads * q < tot) {
          const int e = base + tid + kThreads * q;
          const int ec = e < tot ? e : tot - 1;  // clamped: every load is in bounds
          const int smp = (int)(((float)ec + 0.5f) * rs), o = ec - smp * ssz;
          const int orow = (int)(((float)o + 0.5f) * rr);
          v[q] = core[(int64_t)s_idx[smp * K + k] * ssz + o];
          dst[q] = e < tot ? smp * kSlice + orow * kLdR + (o - orow * rout) : -1;
        }
      }
#pragma unroll
      for (int q = 0; q < kB; ++q)
        if (dst[q] >= 0) S[dst[q]] = v[q];
    }
    __syncthreads();
    if constexpr (kMfmaChain) {
#pragma unroll
      for (int q = 0; q < kSPW; ++q) {
        const int sq = wave + 4 * q;
        if (sq >= jb) continue;  // wave-uniform
        const double* Sj = S + sq * kSlice;  // rin x rout, row-major, row stride kLdR
        if (k == 0) {
          // D_0 = S_0^T (rout x Rn): entry (i, j) = S_0(j, i)
#pragma unroll
          for (int tr = 0; tr < kT; ++tr)
#pragma unroll
            for (int tc = 0; tc < kT; ++tc)
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int i = 16 * tr + 4 * l4 + r, j = 16 * tc + l16;
                D[q][tr][tc][r] = (i < rout && j < rin) ? (float)Sj[j * kLdR + i] : 0.f;
              }
        } else {
          // B operand: D_{k-1} (rin x Rn), slots as above; A operand: S_k^T (rout x rin).  Each
          // operand is a BF16 pair, hi = bf16(v) and lo = bf16(v - hi), and the product is
          // hi hi + hi lo + lo hi in FP32 (the dropped lo lo term and the pair's residue are
          // below 2^-16 of the operands)
          bf8 bh[kT], bl[kT];
#pragma unroll
          for (int tc = 0; tc < kT; ++tc)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const float v = (t < 4 || kT == 2) ? D[q][t < 4 ? 0 : kT - 1][tc][t & 3] : 0.f;
              bh[tc][t] = (__bf16)v;
              bl[tc][t] = (__bf16)(v - (float)bh[tc][t]);
            }
          f4 Dn[kT][kT];
#pragma unroll
          for (int tr = 0; tr < kT; ++tr) {
            bf8 ah, al;
            const int i = 16 * tr + l16;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const int kk = t < 4 ? 4 * l4 + t : 16 + 4 * l4 + (t - 4);
              const double v = (i < rout && kk < rin) ? Sj[kk * kLdR + i] : 0.0;
              ah[t] = (__bf16)v;
              al[t] = (__bf16)(v - (double)ah[t]);
            }
#pragma unroll
            for (int tc = 0; tc < kT; ++tc) {
              f4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[tc], f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[tc], acc, 0, 0, 0);
              Dn[tr][tc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[tc], acc, 0, 0, 0);
            }
          }
#pragma unroll
          for (int tr = 0; tr < kT; ++tr)
#pragma unroll
            for (int tc = 0; tc < kT; ++tc) D[q][tr][tc] = Dn[tr][tc];
        }
      }
    } else if (live) {
      // rin, rout are uniform (the copy's guard is a scalar branch)
      const double* Sj = S + sj * kSlice;
      if (k == 0) {
#pragma unroll
        for (int c = 0; c < RM; ++c)
          if (c < rout) row[c] = Sj[b * kLdR + c];
      } else {
        double nr[RM];
#pragma unroll
        for (int co = 0; co < RM; ++co) nr[co] = 0.0;
        // Rows past rin read the last row (finite) and add 0; columns past rout read the row's
        // padding or unstaged entries of the sample's slot (at most index RM kLdR - 1 < kSlice:
        // any value) and land only in entries of nr that are never read.  No branches and no
        // clamped column index: each row is RM / 2 aligned 16-byte LDS reads, all of a step in
        // flight together.
#pragma unroll
        for (int ci = 0; ci < RM; ++ci) {
          const double v = ci < rin ? row[ci] : 0.0;
          const double2* Sr = (const double2*)(Sj + (ci < rin ? ci : rin - 1) * kLdR);
#pragma unroll
          for (int co = 0; co < RM / 2; ++co) {
            const double2 sv = Sr[co];
            nr[2 * co] = fma(v, sv.x, nr[2 * co]);
            nr[2 * co + 1] = fma(v, sv.y, nr[2 * co + 1]);
          }
        }
#pragma unroll
        for (int c = 0; c < RM; ++c) row[c] = nr[c];
      }
    }
    rin = rout;
  }
  // rin == R_{n-1}: row b of M_s is row[0 .. R_{n-1})
  const int Rp = rin;
  const int P = Rn * Rp;
  __syncthreads();
  const int64_t rows = a.J - j0 < jb ? a.J - j0 : jb;
  if constexpr (kMfmaChain) {
    // BF16 pair, transposed: column col = c R_n + b holds its jb samples contiguously; entry
    // (c, b) of M^T sits in tile (c / 16, b / 16), row 4 (lane / 16) + r, column lane % 16
    __bf16* o1 = (__bf16*)S;  // P x jb each (2 P jb bf16 <= jb * kSlice doubles)
    __bf16* o2 = o1 + P * jb;
#pragma unroll
    for (int q = 0; q < kSPW; ++q) {
      const int sq = wave + 4 * q;
      if (sq >= jb) continue;
      const double w = s_w[sq];
#pragma unroll
      for (int tr = 0; tr < kT; ++tr)
#pragma unroll
        for (int tc = 0; tc < kT; ++tc)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = 16 * tr + 4 * l4 + r, bb = 16 * tc + l16;
            if (c < Rp && bb < Rn) {
              const int col = c * Rn + bb;
              const double v = (double)D[q][tr][tc][r];
              o1[col * jb + sq] = (__bf16)(w * v);
              o2[col * jb + sq] = (__bf16)(w * (w * v));
            }
          }
    }
    __syncthreads();
    __bf16* T1 = (__bf16*)a.A + j0;
    __bf16* T2 = (__bf16*)a.A2 + j0;
    for (int64_t e = tid; e < rows * P; e += kThreads) {
      const int col = (int)(e / rows), q = (int)(e - (int64_t)col * rows);
      T1[col * a.ldt + q] = o1[col * jb + q];
      T2[col * a.ldt + q] = o2[col * jb + q];
    }
  } else if constexpr (std::is_same<TA, __bf16>::value) {
    // BF16 pair, transposed: column col = c R_n + b holds its jb samples contiguously
    __bf16* o1 = (__bf16*)S;  // P x jb each (2 P jb bf16 <= jb * kSlice doubles)
    __bf16* o2 = o1 + P * jb;
    if (live) {
      const double w = s_w[sj];
#pragma unroll
      for (int c = 0; c < RM; ++c)
        if (c < Rp) {
          const int col = c * Rn + b;
          o1[col * jb + sj] = (__bf16)(w * row[c]);
          o2[col * jb + sj] = (__bf16)(w * (w * row[c]));
        }
    }
    __syncthreads();
    __bf16* T1 = (__bf16*)a.A + j0;
    __bf16* T2 = (__bf16*)a.A2 + j0;
    for (int64_t e = tid; e < rows * P; e += kThreads) {
      const int col = (int)(e / rows), q = (int)(e - (int64_t)col * rows);
      T1[col * a.ldt + q] = o1[col * jb + q];
      T2[col * a.ldt + q] = o2[col * jb + q];
    }
  } else {
    TA* out = (TA*)S;  // jb x P staging (jb * P <= 256 * RM < jb * kSlice doubles)
    if (live) {
      const double w = s_w[sj];
#pragma unroll
      for (int c = 0; c < RM; ++c)
        if (c < Rp) out[sj * P + c * Rn + b] = (TA)(w * row[c]);
    }
    __syncthreads();
    TA* A = (TA*)a.A + j0 * P;
    for (int64_t e = tid; e < rows * P; e += kThreads) A[e] = out[e];
  }
  __syncthreads();  // the next batch reuses the LDS
  }
}

// the BF16 sketch has both chain forms; the others form their rows in FP64 only
template <typename TA, int R>
void launch_rm(const DrawArgs& a, unsigned blocks, size_t lds, hipStream_t s) {
  if constexpr (std::is_same<TA, __bf16>::value) {
    if (a.mfma_chain) {
      k_draw<TA, R, true><<<blocks, kThreads, lds, s>>>(a);
      return;
    }
  }
  k_draw<TA, R, false><<<blocks, kThreads, lds, s>>>(a);
}

template <typename TA>
hipError_t draw_dispatch(DrawArgs a, hipStream_t s) {
  int rmax = 0;
  for (int m = 0; m < a.ring.N; ++m) rmax = a.ring.ranks[m] > rmax ? a.ring.ranks[m] : rmax;
  const int RM = rmax <= 4 ? 4 : rmax <= 6 ? 6 : rmax <= 8 ? 8 : rmax <= 10 ? 10 : rmax <= 12 ? 12 : rmax <= 16 ? 16
                 : rmax <= 20 ? 20 : rmax <= 24 ? 24 : 32;
  if (rmax > 32) return hipErrorInvalidValue;
  const int Rn = a.ring.ranks[a.n];
  // samples per workgroup: one thread per (sample, row b); slice staging within 64 KB
  int jb = kThreads / Rn;
  const int cap = (int)((64 * 1024) / (kSliceLd(RM) * sizeof(double)));
  jb = jb < cap ? jb : cap;
  // BF16 form: the chain tiles of at most kChainSPW samples per wave live in registers
  if (std::is_same<TA, __bf16>::value && a.mfma_chain && jb > 4 * kChainSPW(RM)) jb = 4 * kChainSPW(RM);
  if (jb < 1) return hipErrorInvalidValue;
  a.jb = jb;
  const int K = a.ring.N - 1;
  size_t tbytes = 0;
  for (int k = 0; k < K; ++k) tbytes += (size_t)a.ring.dims[(a.n + 1 + k) % a.ring.N] * 8;
  a.tables_in_lds = tbytes <= kDrawTableBytes;
  if (a.draw && a.weights && !a.tables_in_lds) return hipErrorInvalidValue;
  const size_t head = ((size_t)jb * kSliceLd(RM) + jb + (jb * K + 1) / 2 + (size_t)jb * K) * sizeof(double);
  const size_t lds = head + (a.draw && a.tables_in_lds ? tbytes : 0);
  // a resident round of workgroups (LDS-bound, at most four per compute unit), each looping
  // over its batches
  const int64_t nbatch = (a.J + jb - 1) / jb;
  int64_t per_cu = (int64_t)(kDrawLdsBytes / lds);
  per_cu = per_cu < 1 ? 1 : per_cu > 4 ? 4 : per_cu;
  const unsigned blocks = (unsigned)(nbatch < per_cu * kPlanCUs ? nbatch : per_cu * kPlanCUs);
#define TRALS_DRAW_CASE(R)                        \
  case R:                                         \
    launch_rm<TA, R>(a, blocks, lds, s);          \
    break;
  switch (RM) {
    TRALS_DRAW_CASE(4)
    TRALS_DRAW_CASE(6)
    TRALS_DRAW_CASE(8)
    TRALS_DRAW_CASE(10)
    TRALS_DRAW_CASE(12)
    TRALS_DRAW_CASE(16)
    TRALS_DRAW_CASE(20)
    TRALS_DRAW_CASE(24)
    default: TRALS_DRAW_CASE(32)
  }
#undef TRALS_DRAW_CASE
  return hipGetLastError();
}

}  // namespace

hipError_t launch_draw(const DrawArgs& a, int sketch_dtype, hipStream_t s) {
  if (sketch_dtype == 0) return draw_dispatch<double>(a, s);
  if (sketch_dtype == 1) return draw_dispatch<float>(a, s);
  if (sketch_dtype == 2) {
    if (!a.A2 || a.ldt < a.J || a.ldt % 64) return hipErrorInvalidValue;
    return draw_dispatch<__bf16>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace trals
