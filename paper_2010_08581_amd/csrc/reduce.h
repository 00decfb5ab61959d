// Fixed-order sums of split-K partial arrays (ReduceJob), shared by the reduction launch and by
// the factorisation launch that reduces the right-hand sides beside the factorisation.
#pragma once

#include "kernels.h"

namespace trals {

constexpr int kRedElems = 64;  // elements per set (a 256-thread block takes one set, or four)

// Reduction block blk of job jb, run by the 256 threads t = 0..255 of one block (red: its own
// 4 x 64 doubles of LDS; every thread of the workgroup must reach this call, it may hold a
// barrier).  An element set is 64 elements: [64 e, 64 e + 64) for modes 0 and 1, the 8 x 8
// tile (p, i) in [8 tp, 8 tp + 8) x [8 ti, 8 ti + 8) for mode 2.  out = sum over s of
// parts[s * count + e], in a fixed order: with more than four partials, a block takes one set
// and four threads per element sum the partials s = g, g + 4, ... (g = 0..3), the four sums
// added in the order g = 0, 1, 2, 3; with at most four, a block takes four sets (one per
// 64-thread group g) and each thread adds its element's partials in the order s = 0, 1, ...,
// the same sums (mode 3: the partials are P x P each, element e of the output is the packed
// entry (slot, r, c) of the symmetric matrix, its column 16 zero).  mode 0: out[e] = sum.  mode 1: P x P matrix symmetrised from its lower
// triangle, out(i, j) = sum_s parts_s(max(i, j), min(i, j)), for the entries its readers (the
// factorisations: lower 16 x 16 blocks, diagonal blocks whole) use; entries in blocks strictly
// above the diagonal are not written.  mode 2: the P x n partials are
// written transposed, out[i * P + p] = sum_s parts_s[p * n + i] (n = count / P), a tile read as
// 8 runs of 8 consecutive i and written as 8 runs of 8 consecutive p.
__host__ __device__ inline int64_t reduce_sets(const ReduceJob& jb, int P) {
  if (jb.count <= 0) return 0;
  if (jb.mode == 2) {
    const int64_t n = jb.count / P;
    return (int64_t)((P + 7) / 8) * ((n + 7) / 8);
  }
  return (jb.count + kRedElems - 1) / kRedElems;
}
// reduction blocks of job jb (launch sizing)
__host__ __device__ inline int64_t reduce_blocks(const ReduceJob& jb, int P, int nparts) {
  const int64_t sets = reduce_sets(jb, P);
  return nparts <= 4 ? (sets + 3) / 4 : sets;
}

__device__ __forceinline__ void reduce_block(const ReduceJob& jb, int64_t blk, int nparts, int P, int t,
                                             double (*red)[kRedElems]) {
  const double* __restrict__ parts = jb.parts;
  double* __restrict__ out = jb.out;
  const int64_t count = jb.count;
  const int mode = jb.mode;
  const int g = t / kRedElems, el = t % kRedElems;
  const bool few = nparts <= 4;
  const int64_t set = few ? 4 * blk + g : blk;  // this thread's element set
  const bool live = set < reduce_sets(jb, P);
  const int s0 = few ? 0 : g, ds = few ? 1 : 4;  // partials of this thread: s0, s0 + ds, ...
  const int row = few ? g : 0;                   // the LDS row its set is read back from
  if (mode == 2) {
    const int64_t n = count / P, tiles_i = (n + 7) / 8;
    const int64_t tp = set / tiles_i, ti = set - tp * tiles_i;
    const int64_t p = 8 * tp + (el >> 3), i = 8 * ti + (el & 7);
    double acc = 0.0;
    if (live && p < P && i < n) {
#pragma unroll 4
      for (int s = s0; s < nparts; s += ds) acc += parts[s * count + p * n + i];
    }
    red[g][el] = acc;
    __syncthreads();
    if (live && (few || g == 0)) {
      const int ep = el & 7, ei = el >> 3;  // element (ep, ei) of the tile, at red index 8 ep + ei
      const int64_t p2 = 8 * tp + ep, i2 = 8 * ti + ei;
      const int e2 = 8 * ep + ei;
      if (p2 < P && i2 < n)
        out[i2 * P + p2] = few ? red[row][e2] : ((red[0][e2] + red[1][e2]) + red[2][e2]) + red[3][e2];
    }
    return;
  }
  const int64_t e = set * kRedElems + el;
  bool use = live && e < count;
  int64_t src = e, stride = count;
  if (mode == 1 && use) {
    const int i = (int)(e / P), j = (int)(e % P);
    use = j / 16 <= i / 16;
    src = i >= j ? e : (int64_t)j * P + i;
  }
  bool pad = false;
  if (mode == 3) {
    stride = (int64_t)P * P;
    if (use) {
      int bi, bj;
      slot_ij((int)(e / kPackBlk), bi, bj);
      const int rc = (int)(e % kPackBlk), r = rc / kPackLd, c = rc % kPackLd;
      pad = c == 16;
      const int i = 16 * bi + r, j = 16 * bj + c;
      src = i >= j ? (int64_t)i * P + j : (int64_t)j * P + i;
    }
  }
  double acc = 0.0;
  if (use && !pad) {
#pragma unroll 4
    for (int s = s0; s < nparts; s += ds) acc += parts[s * stride + src];
  }
  if (few) {
    if (use) out[e] = acc;
    return;
  }
  red[g][el] = acc;
  __syncthreads();
  if (g == 0 && use) {
    out[e] = ((red[0][el] + red[1][el]) + red[2][el]) + red[3][el];
  }
}

}  // namespace trals
