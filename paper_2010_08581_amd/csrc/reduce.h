// Fixed-order sums of split-K partial arrays (ReduceJob), shared by the reduction launch and by
// the factorisation launch that reduces the right-hand sides beside the factorisation.
#pragma once

#include "kernels.h"

namespace trals {

constexpr int kRedElems = 64;  // elements per 256-thread reduction block

// Elements [64 blk, 64 blk + 64) of job jb, by the 256 threads t = 0..255 of one reduction
// block (red: its own 4 x 64 doubles of LDS; every thread of the workgroup must reach this
// call, it holds a barrier).  out = sum over s of parts[s * count + e], in a fixed order: four
// threads per element sum the partials s = g, g + 4, ... (g = 0..3) and the four sums are added
// in the order g = 0, 1, 2, 3.  mode 0: out[e] = sum.  mode 1: P x P matrix symmetrised from
// its lower triangle, out(i, j) = sum_s parts_s(max(i, j), min(i, j)).  mode 2: the P x n
// partials are written transposed, out[i * P + p] = sum_s parts_s[p * n + i] (n = count / P);
// there block blk is the 8 x 8 tile (p, i) in [8 tp, 8 tp + 8) x [8 ti, 8 ti + 8), read as 8
// runs of 8 consecutive i and written as 8 runs of 8 consecutive p.
// reduction blocks of job jb (launch sizing)
__host__ __device__ inline int64_t reduce_blocks(const ReduceJob& jb, int P) {
  if (jb.count <= 0) return 0;
  if (jb.mode == 2) {
    const int64_t n = jb.count / P;
    return (int64_t)((P + 7) / 8) * ((n + 7) / 8);
  }
  return (jb.count + kRedElems - 1) / kRedElems;
}

__device__ __forceinline__ void reduce_block(const ReduceJob& jb, int64_t blk, int nparts, int P, int t,
                                             double (*red)[kRedElems]) {
  const double* __restrict__ parts = jb.parts;
  double* __restrict__ out = jb.out;
  const int64_t count = jb.count;
  const int mode = jb.mode;
  const int g = t / kRedElems, el = t % kRedElems;
  if (mode == 2) {
    const int64_t n = count / P, tiles_i = (n + 7) / 8;
    const int64_t tp = blk / tiles_i, ti = blk - tp * tiles_i;
    const int64_t p = 8 * tp + (el >> 3), i = 8 * ti + (el & 7);
    double acc = 0.0;
    if (p < P && i < n) {
#pragma unroll 4
      for (int s = g; s < nparts; s += 4) acc += parts[s * count + p * n + i];
    }
    red[g][el] = acc;
    __syncthreads();
    if (g == 0) {
      const int ep = el & 7, ei = el >> 3;  // element (ep, ei) of the tile, at red index 8 ep + ei
      const int64_t p2 = 8 * tp + ep, i2 = 8 * ti + ei;
      const int e2 = 8 * ep + ei;
      if (p2 < P && i2 < n) out[i2 * P + p2] = ((red[0][e2] + red[1][e2]) + red[2][e2]) + red[3][e2];
    }
    return;
  }
  const int64_t e = blk * kRedElems + el;
  double acc = 0.0;
  if (e < count) {
    int64_t src = e;
    if (mode == 1) {
      const int i = (int)(e / P), j = (int)(e % P);
      src = i >= j ? e : (int64_t)j * P + i;
    }
#pragma unroll 4
    for (int s = g; s < nparts; s += 4) acc += parts[s * count + src];
  }
  red[g][el] = acc;
  __syncthreads();
  if (g == 0 && e < count) {
    out[e] = ((red[0][el] + red[1][el]) + red[2][el]) + red[3][el];
  }
}

}  // namespace trals
