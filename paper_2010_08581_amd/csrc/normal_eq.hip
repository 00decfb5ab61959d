// Normal equations of the sampled least-squares problem (Algorithm 2, LS step) on matrix
// cores, fused with the fiber gather (Algorithm 2, "sample X"):
//
//     [ H | B ] = A^T [ A | X~ ],   A = J x P sketched design rows,  X~(j, :) = w_j X(..., :, ...)
//
// One launch covers both products.  The extended column space holds the P Gram columns (read
// from A, padded to a multiple of 64) followed by the I_n data columns (gathered from the
// mode-n panel, where row j's fiber is contiguous).  A workgroup owns a (16 MB) x 64 output
// tile and one chunk of sample rows; each group of four waves takes every KG-th 32-row stage
// of the chunk, each wave owning 16 columns and all MB row blocks.  Gram tiles strictly above
// the diagonal are skipped; consumers read H's lower triangle.  Each lane takes the FP64 row
// factors of its eight k-steps once per stage (w_j for data tiles, 1 for Gram tiles, 0 for
// padding rows) and applies them to its B operand.  Partial tiles per sample chunk are
// reduced afterwards in a fixed order (deterministic).
//
// Arithmetic: v_mfma_f64_16x16x4 with FP64 accumulation for FP64 and FP32 data alike (FP32
// operands widen exactly).  Rounding partial sums of H to FP32 would be an unstructured
// perturbation of the normal equations, amplified by cond(A)^2 in the solution rather than the
// cond(A) that FP32 storage of A and X costs.
//   v_mfma_f64_16x16x4 layouts: A(i, k) lane i + 16 k; B(k, j) lane j + 16 k;
//     D(i, j) lane j + 16 (i % 4), register i / 4.
#include <hip/hip_ext.h>

#include "kernels.h"
#include "reduce.h"

namespace trals {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kColTile = 64;
constexpr int kX3ColTile = 128;  // column tile of the three-slice kernel (eight waves of 16)
constexpr int kKB = 32;          // sample rows per LDS stage (8 MFMA k-steps)
constexpr int kMaxChunk = 1024;  // sample rows per split, padding included (row offsets and weights in LDS)
constexpr int kLdsBytes = 160 * 1024;
constexpr int kX1PerCU = 2;  // workgroups of the one-slice (BF16) products per CU (register bound)

// LDS bytes of the FP64 / FP32 kernel: KG groups x double-buffered A and B stages.
constexpr size_t ne_dyn_lds(int mb, int kg, int esz) {
  return (size_t)kg * 2 * (kKB * (16 * mb + 1) + kKB * (kColTile + 1)) * esz;
}

template <typename Real, int MB, int KG>
__global__ __launch_bounds__(256 * KG) void k_normal_eq(NormalEqArgs a) {
  constexpr int RT = 16 * MB;
  constexpr int NA = kKB * RT / 256;          // A elements per thread per stage (= 2 MB)
  constexpr int NB = kKB * kColTile / 256;    // B elements per thread per stage (= 8)
  constexpr int LA = RT + 1, LB = kColTile + 1;
  constexpr int kStageA = kKB * LA, kStageB = kKB * LB;
  extern __shared__ __align__(16) unsigned char ne_smem[];
  __shared__ int64_t s_roff[kMaxChunk];
  __shared__ double s_w[kMaxChunk];
  if (*a.status != kDevOk) return;
  const int P = a.P, In = a.In;
  // the tiles of one split (same sketch rows) are consecutive logical blocks on one XCD
  const int lb = xcd_linear_block(blockIdx.x, gridDim.x);
  const int s = lb / a.tiles, t = lb - s * a.tiles;
  const int ct = t % a.col_tiles, rt = t / a.col_tiles;
  const int row0 = rt * RT;
  const bool gram = ct < a.gram_tiles;
  const int col0 = gram ? ct * kColTile : (ct - a.gram_tiles) * kColTile;
  if (gram && col0 >= row0 + RT) return;  // strictly upper Gram tile
  const int64_t r0 = (int64_t)s * a.chunk;
  const int64_t r1 = r0 + a.chunk < a.J ? r0 + a.chunk : a.J;
  const int nrows = (int)(r1 - r0);
  const int stages = (nrows + kKB - 1) / kKB;
  const int rounds = (stages + KG - 1) / KG;
  const int npad = rounds * KG * kKB;
  const Real* A = (const Real*)a.A;
  const Real* X = (const Real*)a.panel;
  const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 8), tl = threadIdx.x & 255;
  const int lane = tl & 63, wave = __builtin_amdgcn_readfirstlane(tl >> 6);  // uniform per wave
  Real* As = (Real*)ne_smem + (size_t)g * 2 * (kStageA + kStageB);
  Real* Bs = As + 2 * kStageA;
  // per chunk row: panel-row offset (data tiles) and the row factor (w_j for data tiles, 1 for
  // Gram tiles, 0 for the padding rows of the last stage)
  for (int r = threadIdx.x; r < npad; r += 256 * KG) {
    const bool v = r < nrows;
    if (gram) {
      s_w[r] = v ? 1.0 : 0.0;
    } else {
      int64_t off = 0;
      if (v) {
        if (a.direct) {
          off = r0 + r;
        } else {
          const int32_t* ij = a.idx + (r0 + r) * a.K;
          for (int k = 0; k < a.K; ++k) off += (int64_t)ij[k] * a.stride[k];
        }
      }
      s_roff[r] = off * In;
      s_w[r] = v ? a.w[r0 + r] : 0.0;
    }
  }
  __syncthreads();
  // Loads are unguarded: rows past the chunk read the following rows of the sketch buffer,
  // which holds kSketchPadRows finite rows past row J (their row factor is 0); columns past P
  // or I_n are clamped to the last column (those outputs are not stored).
  Real ra[NA], rb[NB];
  const int gcb = gram ? (col0 + lane < P ? col0 + lane : P - 1) : (col0 + lane < In ? col0 + lane : In - 1);
  auto load_stage = [&](int base) {
    const Real* Ab = A + (r0 + base) * P;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tl + 256 * q;
      const int r = e / RT, c = e - r * RT;
      ra[q] = Ab[r * P + (row0 + c < P ? row0 + c : P - 1)];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int r = wave + 4 * q;
      rb[q] = gram ? Ab[r * P + gcb] : X[s_roff[base + r] + gcb];
    }
  };
  auto store_stage = [&](int buf) {
    Real* as = As + buf * kStageA;
    Real* bs = Bs + buf * kStageB;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tl + 256 * q;
      const int r = e / RT, c = e - r * RT;
      as[r * LA + c] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) bs[(wave + 4 * q) * LB + lane] = rb[q];
  };
  d4 acc[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
  const int r16 = lane & 15, k4 = lane >> 4;
  // Pipeline: round u computes on LDS buffer u & 1; between its first and second half of
  // k-steps every wave stores the (already loaded) stage of round u + 1 into the other buffer
  // and issues the loads of round u + 2, so those memory operations overlap the matrix-core
  // work of the other wave on the SIMD instead of running between barriers.  The other
  // buffer was last read in round u - 1, which every wave finished before round u's barrier.
  auto mfma_steps = [&](const Real* as, const Real* bs, const double* wv, int ks0) {
#pragma unroll
    for (int kq = 0; kq < kKB / 8; ++kq) {
      const int ks = ks0 + kq;
      const int kr = ks * 4 + k4;
      const double b = (double)bs[kr * LB + wave * 16 + r16] * wv[ks];
#pragma unroll
      for (int m = 0; m < MB; ++m)
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)as[kr * LA + m * 16 + r16], b, acc[m], 0, 0, 0);
    }
  };
  load_stage(g * kKB);
  store_stage(0);
  if (rounds > 1) load_stage((KG + g) * kKB);
  for (int u = 0; u < rounds; ++u) {
    const int buf = u & 1;
    const int base = (u * KG + g) * kKB;
    __syncthreads();
    // A last round holding a single stage (group 0's; the other groups' would be padding) is
    // shared: group 0 takes its first half of k-steps, group 1 the second half from group 0's
    // buffer (the groups' sums are added below).
    const bool lone = KG == 2 && u == rounds - 1 && (stages & 1);
    const int sbase = lone ? u * KG * kKB : base;  // rows of the stage this group works on
    const Real* as = As + buf * kStageA;
    const Real* bs = Bs + buf * kStageB;
    const Real* as2 = lone ? (const Real*)ne_smem + buf * kStageA : as;
    const Real* bs2 = lone ? (const Real*)ne_smem + 2 * kStageA + buf * kStageB : bs;
    double wv[kKB / 4];
#pragma unroll
    for (int ks = 0; ks < kKB / 4; ++ks) wv[ks] = s_w[sbase + ks * 4 + k4];
    if (!lone || g == 0) mfma_steps(as, bs, wv, 0);
    __builtin_amdgcn_sched_barrier(0);
    if (u + 1 < rounds) {
      store_stage(buf ^ 1);
      if (u + 2 < rounds) load_stage(base + 2 * KG * kKB);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (!lone || g == 1) mfma_steps(as2, bs2, wv, kKB / 8);
  }
  if constexpr (KG > 1) {
    // fixed-order sum of the groups' accumulators (group 0 + group 1 + ...)
    double* red = (double*)ne_smem;
    __syncthreads();
    if (g > 0)
#pragma unroll
      for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[((size_t)((g - 1) * MB + m) * 4 + r) * 256 + tl] = acc[m][r];
    __syncthreads();
    if (g > 0) return;
    for (int h = 1; h < KG; ++h)
#pragma unroll
      for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[m][r] += red[((size_t)((h - 1) * MB + m) * 4 + r) * 256 + tl];
  }
  const int col = col0 + wave * 16 + r16;
  if (gram) {
    double* H = a.Hpart + (int64_t)s * P * P;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + m * 16 + 4 * r + k4;
        if (row < P && col <= row) H[(int64_t)row * P + col] = acc[m][r];
      }
  } else {
    double* B = a.Bpart + (int64_t)s * P * In;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + m * 16 + 4 * r + k4;
        if (row < P && col < In) B[(int64_t)row * In + col] = acc[m][r];
      }
  }
}

// BF16 form of the same products (k_normal_eq_x3 with one slice).  The draw kernel writes the
// sketch twice in BF16 and transposed (column c's samples contiguous): bf16(w_j M_j) for the Gram
// tiles and bf16(w_j^2 M_j) for the data tiles, so that B = sum_j w_j^2 M_j^T x_j meets the raw
// BF16 panel rows (x~_j = w_j x_j, Definition 5) unmodified; a gather pass (k_x1_gather) writes
// the sampled fibers transposed beside them.  Products are accumulated in FP32 over each
// 64-sample block and the block sums added in FP64.
//   v_mfma_f32_16x16x32_bf16 layouts: A(i, k) at lane i + 16 (k / 8), element k % 8;
//   B(k, j) at lane j + 16 (k / 8), element k % 8; D(i, j) at lane j + 16 (i / 4), register i % 4.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------------------
// FP32 path on BF16 matrix cores with products exact to 2^-34 of the block maxima (ne_dtype 3).
//
// Every operand value v of a 64-sample block is written as v = 2^(e-8) (s0 + 2^-8 s1 + 2^-16 s2)
// + r with integers |s0| <= 256, |s1|, |s2| <= 128 (exact in BF16) and |r| <= 2^(e-25), e the
// block exponent of its column (max |v| < 2^e): a relative truncation of at most 2^-24 of the
// column's block maximum, the size of FP32 rounding.  A product of two such values is the sum
// of nine slice products s_s t_t 2^(-8(s+t)); the eight of levels l = s + t <= 3 are formed
// (kX3Levels), and the dropped s2 t2 is below 2^-34 of the product of the block maxima.
// Each level's sum over the 64 samples is an integer below 2^24, so the FP32 accumulation of
// the BF16 matrix cores is exact.  After each block the level sums are combined and scaled by
// 2^(e_row + e_col - 16) in FP64 and added to FP64 accumulators.
//
// The sketch side has one representation (sketch_split_tile), used both as the row operand
// and, in the Gram tiles, as the column operand: H is exactly R(A)^T R(A).  The data side is the
// weighted fiber w_j X(j, i), split the same way by the split pass (fiber_split_tile) with the
// block maximum of its column.  So
// B = R(A)^T R(diag(w) X) up to the dropped levels: both products are those of one slightly
// perturbed problem, whose solution moves by cond(A) times the perturbation, as with FP32
// storage alone.
//   v_mfma_f32_16x16x32_bf16 layouts: A(i, k) at lane i + 16 (k / 8), element k % 8;
//   B(k, j) at lane j + 16 (k / 8), element k % 8; D(i, j) at lane j + 16 (i / 4), register i % 4.

__device__ __forceinline__ int block_exponent(double m) {
  int e = 0;
  if (m > 0.0) (void)frexp(m, &e);  // m = f 2^e, f in [0.5, 1): every |v| <= m is below 2^e
  return e;
}

// three 8-bit slices of y = v 2^(8 - e), |y| < 256, of an FP32 value v: the power-of-two
// scaling, the differences y - rint(y) (|.| <= 1/2, within y's precision) and the products by
// 256 are exact in FP32, so the slices reproduce y down to 2^-17 (y carries 24 bits)
struct Slices3 {
  __bf16 s[3];
};
__device__ __forceinline__ Slices3 split3(float v, int e) {
  const float y = ldexpf(v, 8 - e);
  const float a0 = rintf(y);
  const float r1 = (y - a0) * 256.f;
  const float a1 = rintf(r1);
  const float a2 = rintf((r1 - a1) * 256.f);
  return Slices3{{(__bf16)a0, (__bf16)a1, (__bf16)a2}};
}

// One 64 x 64 tile (bx, by) of the sketch per workgroup, no LDS.
// Wave w takes columns 16 w .. 16 w + 15 of the tile; lane (li, q) = (lane % 16, lane / 16)
// holds samples 16 q .. 16 q + 15 of column li, so a column's 64 samples sit in four lanes of one
// wave: its block maximum takes two lane exchanges, and each lane stores its 16 samples of each
// slice as 32 contiguous bytes (the four lanes of a column fill its 128-byte run).
__device__ __forceinline__ void sketch_split_tile(const float* __restrict__ A, int64_t J, int P,
                                                  __bf16* __restrict__ S3, int64_t ld, int* __restrict__ E, int bx,
                                                  int by) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, q = lane >> 4;
  const int p = bx * 64 + 16 * wave + li;
  const int64_t j0 = (int64_t)by * kSplitBlock + 16 * q;
  const bool pin = p < P;
  float v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = (pin && j0 + r < J) ? A[(j0 + r) * P + p] : 0.f;
  float mx = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) mx = fmaxf(mx, fabsf(v[r]));
  mx = fmaxf(mx, __shfl_xor(mx, 16));
  mx = fmaxf(mx, __shfl_xor(mx, 32));
  const int e = block_exponent((double)mx);
  if (q == 0 && pin) E[(int64_t)by * P + p] = e;
  bf8 o[3][2];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const Slices3 x = split3(v[r], e);
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) o[sl][r >> 3][r & 7] = x.s[sl];
  }
  if (pin)
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      bf8* dst = (bf8*)(S3 + ((int64_t)sl * P + p) * ld + j0);
      dst[0] = o[sl][0];
      dst[1] = o[sl][1];
    }
}

// Tile (bx, by) of the weighted fibers w_j X(j, :) (FP32 product of the FP32 weight and the
// panel entry): one 64-sample block and 64 columns, gathered and split as the sketch is.  Lane
// (li, q) of wave w holds samples 16 q .. 16 q + 15 of column 16 w + li (the 16 lanes of one q
// read 64 contiguous bytes of a fiber), the column's exponent takes two lane exchanges, and each
// lane stores 32 contiguous bytes per slice.  Samples past J have weight 0 and row 0.
__device__ __forceinline__ void fiber_split_tile(const NormalEqArgs& a, int bx, int by) {
  __shared__ int64_t s_off[kSplitBlock];
  __shared__ float s_w[kSplitBlock];
  const int64_t jb = (int64_t)by * kSplitBlock;
  const int In = a.In;
  if (threadIdx.x < kSplitBlock) {
    const int64_t j = jb + threadIdx.x;
    int64_t off = 0;
    float w = 0.f;
    if (j < a.J) {
      if (a.direct) {
        off = j;
      } else {
        const int32_t* ij = a.idx + j * a.K;
        for (int k = 0; k < a.K; ++k) off += (int64_t)ij[k] * a.stride[k];
      }
      w = (float)a.w[j];
    }
    s_off[threadIdx.x] = off * In;
    s_w[threadIdx.x] = w;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, q = lane >> 4;
  const int i = bx * 64 + 16 * wave + li;
  const bool in = i < In;
  const int ic = in ? i : In - 1;
  const float* X = (const float*)a.panel;
  float v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = s_w[16 * q + r] * X[s_off[16 * q + r] + ic];
  float mx = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) mx = fmaxf(mx, fabsf(v[r]));
  mx = fmaxf(mx, __shfl_xor(mx, 16));
  mx = fmaxf(mx, __shfl_xor(mx, 32));
  const int e = block_exponent((double)mx);
  if (q == 0 && in) a.ED[(int64_t)by * In + i] = e;
  bf8 o[3][2];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const Slices3 x = split3(v[r], e);
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) o[sl][r >> 3][r & 7] = x.s[sl];
  }
  if (in)
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      bf8* dst = (bf8*)((__bf16*)a.D3 + ((int64_t)sl * In + i) * a.ld + jb + 16 * q);
      dst[0] = o[sl][0];
      dst[1] = o[sl][1];
    }
}

// Both split passes of an update in one launch: workgroups [0, sk_tiles) take the sketch's
// tiles (ceil(P / 64) per 64-sample block), the rest the fibers' (ceil(I_n / 64) per block).
__global__ __launch_bounds__(256) void k_x3_split(NormalEqArgs a, int sk_tiles) {
  if (*a.status != kDevOk) return;
  const int b = blockIdx.x;
  if (b < sk_tiles) {
    const int cx = (a.P + 63) / 64;
    sketch_split_tile((const float*)a.A, a.J, a.P, a.S3, a.ld, a.E, b % cx, b / cx);
  } else {
    const int cx = (a.In + 63) / 64, t = b - sk_tiles;
    fiber_split_tile(a, t % cx, t / cx);
  }
}

// The BF16 form's gather pass: workgroups [0, fb_tiles) gather the raw BF16 fibers of one
// 64-sample block and 64 columns into D3 (I_n x ld, samples contiguous per column; zero past J),
// lane (li, q) of wave w taking samples 16 q .. 16 q + 15 of column 16 w + li.  With x1_rows the
// rest take one 64 x 64 tile each of the FP32 rows A = w M (J x P): S3 gets bf16(w M) and
// S3 + P ld gets bf16(w^2 M), transposed (zero past J); without, the last workgroup zeroes the
// columns J .. ld - 1 of the transposed sketches the draw wrote (row p of bf16(w M) and
// bf16(w^2 M) at p ld), which the draw does not write.
__global__ __launch_bounds__(256) void k_x1_gather(NormalEqArgs a, int fb_tiles) {
  __shared__ int64_t s_off[kSplitBlock];
  if (*a.status != kDevOk) return;
  const int In = a.In;
  if ((int)blockIdx.x >= fb_tiles && a.x1_rows) {
    const int cx = (a.P + 63) / 64, t = (int)blockIdx.x - fb_tiles;
    const int bx = t % cx, by = t / cx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, q = lane >> 4;
    const int p = bx * 64 + 16 * wave + li;
    if (p >= a.P) return;
    const int64_t j0 = (int64_t)by * kSplitBlock + 16 * q;
    const float* A = (const float*)a.A;
    bf8 o1[2], o2[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const bool in = j0 + r < a.J;
      const float v = in ? A[(j0 + r) * a.P + p] : 0.f;
      const double w = in ? a.w[j0 + r] : 0.0;
      o1[r >> 3][r & 7] = (__bf16)v;
      o2[r >> 3][r & 7] = (__bf16)(w * (double)v);
    }
    bf8* d1 = (bf8*)(a.S3 + (int64_t)p * a.ld + j0);
    bf8* d2 = (bf8*)(a.S3 + ((int64_t)a.P + p) * a.ld + j0);
    d1[0] = o1[0];
    d1[1] = o1[1];
    d2[0] = o2[0];
    d2[1] = o2[1];
    return;
  }
  if ((int)blockIdx.x == fb_tiles) {
    const int pad = (int)(a.ld - a.J);
    __bf16* A = (__bf16*)a.A;
    __bf16* A2 = (__bf16*)a.A2;
    for (int e = threadIdx.x; e < a.P * pad; e += 256) {
      const int p = e / pad;
      const int64_t j = a.J + (e - p * pad);
      A[(int64_t)p * a.ld + j] = (__bf16)0.f;
      A2[(int64_t)p * a.ld + j] = (__bf16)0.f;
    }
    return;
  }
  const int cx = (In + 63) / 64;
  const int bx = (int)blockIdx.x % cx, by = (int)blockIdx.x / cx;
  const int64_t jb = (int64_t)by * kSplitBlock;
  if (threadIdx.x < kSplitBlock) {
    const int64_t j = jb + threadIdx.x;
    int64_t off = -1;
    if (j < a.J) {
      off = 0;
      if (a.direct) {
        off = j;
      } else {
        const int32_t* ij = a.idx + j * a.K;
        for (int k = 0; k < a.K; ++k) off += (int64_t)ij[k] * a.stride[k];
      }
      off *= In;
    }
    s_off[threadIdx.x] = off;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, q = lane >> 4;
  const int i = bx * 64 + 16 * wave + li;
  if (i >= In) return;
  const __bf16* X = (const __bf16*)a.panel;
  bf8 o[2];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t off = s_off[16 * q + r];
    o[r >> 3][r & 7] = off >= 0 ? X[off + i] : (__bf16)0.f;
  }
  bf8* dst = (bf8*)((__bf16*)a.D3 + (int64_t)i * a.ld + jb + 16 * q);
  dst[0] = o[0];
  dst[1] = o[1];
}

// Workgroup of 8 waves on a (16 MB) x 128 tile: wave c owns tile columns 16c .. 16c + 15, all
// MB row blocks and both 32-sample halves (matrix-core k-steps) of every 64-sample block, so
// that its level sums cover 64 samples between FP64 flushes (each stays below 2^23 in
// magnitude, exact in FP32).  The sketch rows of the tile (three slices, both halves) are staged
// in LDS by the whole workgroup, double-buffered with one barrier per block; each wave loads the
// column operand of its own columns directly into the matrix-core registers, one block ahead:
// Gram tiles read the sketch slices, data tiles the fiber slices (both written by k_x3_split).
constexpr int kX3Ld = 72;  // LDS row stride of a staged slice (64 samples + 8: 16-byte reads
                           // of 16 rows fall on distinct banks)
// Slice products kept: level l = si + ti of s_si t_ti weighs 2^(-8 l) against the leading
// product, and levels 0 .. kX3Levels - 1 are multiplied (eight products of nine).  The dropped
// level 4 (s2 t2, an integer below 2^14) is below 2^-34 of the product of the two block maxima,
// far under the FP32 inputs' own rounding (2^-24).  Dropping level 3 as well (six products) was
// measured 2% faster but a perturbation of that size (2^-25) in H and B separately is amplified
// by cond(A)^2 in the solution (video cores 4.8e-7 -> 9.8e-6 against the oracle).
constexpr int kX3Levels = 4;

// One tile of k_normal_eq_x3; GRAM selects the column operand (sketch or fiber slices) and the
// output (H or B partials).  NS = 3: the FP32 path's slices (S3 / D3, block exponents); NS = 1:
// the BF16 form, whose operands are BF16 values already (row operand bf16(w M) for Gram tiles,
// bf16(w^2 M) for data tiles, P x ld; column operand bf16(w M) or the gathered raw fibers D3,
// I_n x ld), one product per k-step, no exponents.
template <int MB, bool GRAM, int NS>
__device__ __forceinline__ void x3_tile(const NormalEqArgs& a, int s, int row0, int col0, int (*s_ea)[16 * MB],
                                        unsigned char* smem) {
  static_assert(NS == 1 || NS == 3, "three slices (FP32 path) or one (BF16 form)");
  constexpr int NL = NS == 3 ? kX3Levels : 1;           // level sums per output
  constexpr int RT = 16 * MB;
  constexpr int kBufElems = NS * RT * kX3Ld;            // one buffer of staged row operands
  constexpr int kChunks = NS * RT * (kSplitBlock / 8);  // 16-byte pieces of a buffer
  constexpr int kCPT = (kChunks + 511) / 512;          // per thread
  const int P = a.P, In = a.In;
  const int64_t r0 = (int64_t)s * a.chunk;  // a multiple of kSplitBlock
  const int64_t r1 = r0 + a.chunk < a.J ? r0 + a.chunk : a.J;
  const int nrows = (int)(r1 - r0);
  const int nblk = (nrows + kSplitBlock - 1) / kSplitBlock;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wave
  const int li = lane & 15, lg = lane >> 4;
  __bf16* Ab = (__bf16*)smem;  // [2][NS][RT][kX3Ld]
  const __bf16* S3 = NS == 3     ? (const __bf16*)a.S3
                     : a.x1_rows ? (const __bf16*)a.S3 + (GRAM ? 0 : (int64_t)a.P * a.ld)
                     : GRAM      ? (const __bf16*)a.A
                                 : (const __bf16*)a.A2;
  const int64_t ld = a.ld, sstride = (int64_t)P * ld;
  const int64_t eb0 = r0 / kSplitBlock;
  // staging of the sketch rows: piece q = (slice, row, 8-sample group)
  bf8 stg[kCPT];
  int stg_ea = 0;
  auto load_a = [&](int b) {
    const int64_t base = r0 + (int64_t)b * kSplitBlock;
#pragma unroll
    for (int u = 0; u < kCPT; ++u) {
      const int q = tid + 512 * u;
      const int qc = q < kChunks ? q : kChunks - 1;
      const int sl = qc / (RT * 8), rem = qc - sl * (RT * 8), r = rem >> 3, c8 = rem & 7;
      const int pr = row0 + r < P ? row0 + r : P - 1;
      stg[u] = *(const bf8*)(S3 + sl * sstride + (int64_t)pr * ld + base + 8 * c8);
    }
    if (NS == 3 && tid < RT) stg_ea = a.E[(eb0 + b) * P + (row0 + tid < P ? row0 + tid : P - 1)];
  };
  auto store_a = [&](int buf) {
    __bf16* dst = Ab + buf * kBufElems;
#pragma unroll
    for (int u = 0; u < kCPT; ++u) {
      const int q = tid + 512 * u;
      if (q < kChunks) {
        const int sl = q / (RT * 8), rem = q - sl * (RT * 8), r = rem >> 3, c8 = rem & 7;
        *(bf8*)(dst + (sl * RT + r) * kX3Ld + 8 * c8) = stg[u];
      }
    }
    if (NS == 3 && tid < RT) s_ea[buf][tid] = stg_ea;
  };
  // column operand of this wave: sketch column (Gram tiles) or fiber column (data tiles) bcc
  const int bc = col0 + 16 * wave + li;
  const int ncols = GRAM ? P : In;
  const int bcc = bc < ncols ? bc : ncols - 1;
  const __bf16* C3 = GRAM ? S3 : (const __bf16*)a.D3;
  const int* CE = GRAM ? a.E : a.ED;  // (NS = 3)
  const int64_t cstride = (int64_t)ncols * ld;
  const __bf16* brow = C3 + (int64_t)bcc * ld + r0;
  bf8 nb3[2][NS];  // next block's column slices, both halves
  int ncol_e = 0;
  auto load_b = [&](int b) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k0 = b * kSplitBlock + 32 * h + 8 * lg;  // this lane's 8 samples of half h
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) nb3[h][sl] = *(const bf8*)(brow + sl * cstride + k0);
    }
    if (NS == 3) ncol_e = CE[(eb0 + b) * ncols + bcc];
  };
  f4 acc[MB][NL];
  double out[MB][4];
#pragma unroll
  for (int m = 0; m < MB; ++m) {
#pragma unroll
    for (int l = 0; l < NL; ++l) acc[m][l] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < 4; ++q) out[m][q] = 0.0;
  }
  load_a(0);
  load_b(0);
  store_a(0);
  __syncthreads();
  for (int b = 0; b < nblk; ++b) {
    const int buf = b & 1;
    const bool more = b + 1 < nblk;
    bf8 cb[2][NS];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) cb[h][sl] = nb3[h][sl];
    const int fcol = ncol_e;
    if (more) {
      load_a(b + 1);
      load_b(b + 1);
    }
    const __bf16* As = Ab + buf * kBufElems;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        bf8 av[NS];
#pragma unroll
        for (int sl = 0; sl < NS; ++sl)
          av[sl] = *(const bf8*)(As + (sl * RT + 16 * m + li) * kX3Ld + 32 * h + 8 * lg);
#pragma unroll
        for (int si = 0; si < NS; ++si)
#pragma unroll
          for (int ti = 0; ti < NS; ++ti)
            if (si + ti < NL)
              acc[m][si + ti] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[si], cb[h][ti], acc[m][si + ti], 0, 0, 0);
      }
    }
    // block sums into FP64: sum_l acc_l 2^(-8 l), times 2^(e_row + e_col - 16) (NS = 3); the
    // BF16 form's FP32 block sums as they are
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (NS == 3) {
          double v = (double)acc[m][NL - 1][q];
#pragma unroll
          for (int l = NL - 2; l >= 0; --l) v = fma(v, 0.00390625, (double)acc[m][l][q]);
          out[m][q] += ldexp(v, s_ea[buf][16 * m + 4 * lg + q] + fcol - 16);
        } else {
          out[m][q] += (double)acc[m][0][q];
        }
      }
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int l = 0; l < NL; ++l) acc[m][l] = f4{0.f, 0.f, 0.f, 0.f};
    if (more) store_a(buf ^ 1);
    __syncthreads();
  }
  const int col = col0 + wave * 16 + li;
  if (GRAM) {
    double* H = a.Hpart + (int64_t)s * P * P;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + m * 16 + 4 * lg + q;
        if (row < P && col < P && col <= row) H[(int64_t)row * P + col] = out[m][q];
      }
  } else {
    double* B = a.Bpart + (int64_t)s * P * In;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + m * 16 + 4 * lg + q;
        if (row < P && col < In) B[(int64_t)row * In + col] = out[m][q];
      }
  }
}

template <int MB, int NS>
__global__ __launch_bounds__(512) void k_normal_eq_x3(NormalEqArgs a) {
  constexpr int RT = 16 * MB;
  extern __shared__ __align__(16) unsigned char x3_smem[];
  __shared__ int s_ea[2][RT];
  if (*a.status != kDevOk) return;
  const int lb = xcd_linear_block(blockIdx.x, gridDim.x);  // a split's tiles share an XCD
  const int s = lb / a.tiles;
  int t = lb - s * a.tiles;
  // the grid holds only the tiles on or below the diagonal, so that every workgroup computes
  // and the rounds of workgroups per XCD are the ones the planner counted.  Row tiles vary
  // fastest: the row tiles of one column tile (which gather the same fibers) run side by side on
  // one XCD and share them through its L2.  Gram column tile c keeps the row tiles from
  // floor(128 c / RT) on (those reaching column 128 c).
  const int row_tiles = a.row_tiles;
  for (int c = 0; c < a.gram_tiles; ++c) {
    const int first = (c * kX3ColTile) / RT < row_tiles ? (c * kX3ColTile) / RT : row_tiles;
    const int n = row_tiles - first;
    if (t < n) {
      x3_tile<MB, true, NS>(a, s, (first + t) * RT, c * kX3ColTile, s_ea, x3_smem);
      return;
    }
    t -= n;
  }
  const int rt = t % row_tiles, ct = t / row_tiles;
  x3_tile<MB, false, NS>(a, s, rt * RT, ct * kX3ColTile, s_ea, x3_smem);
}

// Tiles one split of the three-slice kernel computes: every data tile and the Gram tiles on or
// below the diagonal.
int x3_live_tiles(const NormalEqPlan& pl) {
  const int RT = 16 * pl.mb;
  int n = pl.row_tiles * pl.data_tiles;
  for (int c = 0; c < pl.gram_tiles; ++c) {
    const int first = (c * kX3ColTile) / RT;
    n += pl.row_tiles - (first < pl.row_tiles ? first : pl.row_tiles);
  }
  return n;
}

size_t x3_dyn_lds(int mb, int ns) {
  return (size_t)2 * ns * 16 * mb * kX3Ld * 2;  // two buffers of staged row operands
}

// Two reductions in one launch: blocks [0, nb0) take job 0, the rest job 1.
__global__ __launch_bounds__(256) void k_reduce_parts(ReduceJob j0, ReduceJob j1, int64_t nb0, int nparts, int P,
                                                      const int* status) {
  __shared__ double red[4][kRedElems];
  if (*status != kDevOk) return;
  const bool first = (int64_t)blockIdx.x < nb0;
  reduce_block(first ? j0 : j1, (int64_t)blockIdx.x - (first ? 0 : nb0), nparts, P, threadIdx.x, red);
}

// e0/e1 (optional): events the runtime stamps at the kernel's own start and end
template <typename Real, int KG>
hipError_t dispatch(const NormalEqArgs& a, int mb, unsigned grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const size_t lds = ne_dyn_lds(mb, KG, sizeof(Real));
  switch (mb) {
#define TRALS_NE_CASE(MB)                                                                              \
  case MB:                                                                                             \
    if (e0)                                                                                            \
      hipExtLaunchKernelGGL((k_normal_eq<Real, MB, KG>), dim3(grid), dim3(256 * KG), lds, s, e0, e1, 0, a); \
    else                                                                                               \
      k_normal_eq<Real, MB, KG><<<grid, 256 * KG, lds, s>>>(a);                                          \
    break;
    TRALS_NE_CASE(1)
    TRALS_NE_CASE(2)
    TRALS_NE_CASE(3)
    TRALS_NE_CASE(4)
    TRALS_NE_CASE(5)
    TRALS_NE_CASE(6)
    TRALS_NE_CASE(7)
    TRALS_NE_CASE(8)
#undef TRALS_NE_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// Splits of the slice-operand kernel.  Its workgroups hold a CU (per_cu of them) for the whole
// split, so a launch takes ceil(workgroups on an XCD / their slots per XCD) rounds, each as long as one
// split's 64-sample blocks; every split adds its FP64 partials of H and B, written once and read
// once by the reduction.  The split count minimises
//     rounds * (blocks per split + 1) + splits * partial bytes / 12 MB
// (12 MB: what the reduction moves in about the time of one block; the 1 a workgroup's prologue
// and epilogue), ties to fewer splits.
static NormalEqPlan plan_x3_splits(NormalEqPlan pl, int64_t J, int num_cu, int per_cu) {
  const int live = x3_live_tiles(pl);
  const int P = 16 * pl.mb * pl.row_tiles;  // bound on the partial rows, padding included
  const double part_blocks = 16.0 * ((double)P * (P + 1) / 2 + (double)P * 128 * pl.data_tiles) / 12e6;
  const int per_xcd = per_cu * (num_cu / kXcds > 0 ? num_cu / kXcds : 1);
  const int64_t s_lo = 1;
  int64_t s_hi = 4 * (int64_t)per_cu * num_cu / live + 2;
  if (s_hi > (J + kSplitBlock - 1) / kSplitBlock) s_hi = (J + kSplitBlock - 1) / kSplitBlock;
  if (s_hi < s_lo) s_hi = s_lo;
  double best = 1e300;
  int64_t best_chunk = 0;
  for (int64_t S = s_lo; S <= s_hi; ++S) {
    const int64_t chunk = ((J + S - 1) / S + kSplitBlock - 1) / kSplitBlock * kSplitBlock;
    const int64_t splits = (J + chunk - 1) / chunk;
    const int64_t grid = splits * live;
    const int64_t rounds = ((grid + kXcds - 1) / kXcds + per_xcd - 1) / per_xcd;
    const double cost = (double)rounds * (double)(chunk / kSplitBlock + 1) + part_blocks * (double)splits;
    if (cost < best - 1e-9) {
      best = cost;
      best_chunk = chunk;
    }
  }
  pl.chunk = best_chunk;
  pl.splits = (int)((J + best_chunk - 1) / best_chunk);
  return pl;
}

NormalEqPlan plan_normal_eq(int P, int In, int64_t J, int ne_dtype, int num_cu) {
  NormalEqPlan pl;
  // row tile of 16 * mb rows: one tile when P <= 128, else the mb in [4, 8] with least padding.
  // The slice-operand kernel (FP32 three-slice path, BF16 form) holds its accumulators without
  // spilling up to mb = 4: one tile when P <= 64, else the mb in [3, 4] with the fewest row
  // tiles (each reads the column operand again), then the least padding.
  const bool x3 = ne_dtype == 2 || ne_dtype == 3;  // the slice-operand products (k_normal_eq_x3)
  const int mb_max = x3 ? 4 : 8, mb_min = x3 ? 3 : 4;
  if (P <= 16 * mb_max) {
    pl.mb = (P + 15) / 16;
  } else {
    int best = mb_max, best_pad = 1 << 30, best_tiles = 1 << 30;
    for (int mb = mb_max; mb >= mb_min; --mb) {
      const int rt = 16 * mb;
      const int tiles = (P + rt - 1) / rt;
      const int pad = tiles * rt - P;
      const bool better = x3 ? (tiles < best_tiles || (tiles == best_tiles && pad < best_pad)) : pad < best_pad;
      if (better) {
        best_pad = pad;
        best_tiles = tiles;
        best = mb;
      }
    }
    pl.mb = best;
  }
  pl.row_tiles = (P + 16 * pl.mb - 1) / (16 * pl.mb);
  const int ctile = x3 ? kX3ColTile : kColTile;
  pl.gram_tiles = (P + ctile - 1) / ctile;
  pl.data_tiles = (In + ctile - 1) / ctile;
  if (x3) return plan_x3_splits(pl, J, num_cu, ne_dtype == 2 ? kX1PerCU : 1);
  const int64_t tiles = (int64_t)pl.row_tiles * (pl.gram_tiles + pl.data_tiles);
  // workgroups resident per CU (LDS-bound) and the rows one split must be a multiple of
  const int kg = ne_dtype == 1 ? 2 : 1;
  const int esz = ne_dtype == 1 ? 4 : 8;
  const size_t lds = ne_dyn_lds(pl.mb, kg, esz) + (size_t)kMaxChunk * 16;
  int per_cu = (int)(kLdsBytes / lds);
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 2) per_cu = 2;
  const int quantum = kg * kKB;
  // one round of workgroups over the chip: splits = resident slots / tiles, at least one
  // quantum of rows per split and at most kMaxChunk rows with the padding of the last round
  int64_t S = ((int64_t)per_cu * num_cu) / tiles;
  if (S < 1) S = 1;
  if (S > J / quantum) S = J / quantum;
  if (S < 1) S = 1;
  const int64_t maxchunk = kMaxChunk - quantum;
  if ((J + S - 1) / S > maxchunk) S = (J + maxchunk - 1) / maxchunk;
  const int64_t chunk = (J + S - 1) / S;
  pl.chunk = chunk;
  pl.splits = (int)((J + chunk - 1) / chunk);
  return pl;
}

hipError_t launch_normal_eq(const NormalEqArgs& args, const NormalEqPlan& pl, int ne_dtype, hipStream_t s,
                            hipEvent_t e0, hipEvent_t e1) {
  NormalEqArgs a = args;
  a.col_tiles = pl.gram_tiles + pl.data_tiles;
  a.row_tiles = pl.row_tiles;
  a.tiles = ne_dtype >= 2 ? x3_live_tiles(pl) : pl.row_tiles * a.col_tiles;
  a.splits = pl.splits;
  if ((int64_t)pl.splits * a.tiles > 0x7fffffff) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)(pl.splits * a.tiles);
  if (ne_dtype == 0) return dispatch<double, 1>(a, pl.mb, grid, s, e0, e1);
  if (ne_dtype == 1) return dispatch<float, 2>(a, pl.mb, grid, s, e0, e1);
  if (ne_dtype == 2 || ne_dtype == 3) {
    const int ns = ne_dtype == 3 ? 3 : 1;
    if (!a.A || !a.D3 || a.ld % kSplitBlock || a.ld < a.J) return hipErrorInvalidValue;
    if (ns == 3 && (!a.S3 || !a.E || !a.ED)) return hipErrorInvalidValue;
    if (ns == 1 && (a.x1_rows ? !a.S3 || !a.w : !a.A2)) return hipErrorInvalidValue;
    const int64_t jb = (a.J + kSplitBlock - 1) / kSplitBlock;
    const int64_t sk = ns == 3 || a.x1_rows ? (int64_t)((a.P + 63) / 64) * jb : 0;
    const int64_t fb = (int64_t)((a.In + 63) / 64) * jb;
    if (sk + fb + 1 > 0x7fffffff) return hipErrorInvalidValue;
    // the split pass (FP32 path) or the gather pass (BF16 form), then the products
    if (ns == 3) {
      if (e0)
        hipExtLaunchKernelGGL(k_x3_split, dim3((unsigned)(sk + fb)), dim3(256), 0, s, e0, nullptr, 0, a, (int)sk);
      else
        k_x3_split<<<(unsigned)(sk + fb), 256, 0, s>>>(a, (int)sk);
    } else {
      const unsigned g1 = (unsigned)(fb + (a.x1_rows ? sk : 1));
      if (e0)
        hipExtLaunchKernelGGL(k_x1_gather, dim3(g1), dim3(256), 0, s, e0, nullptr, 0, a, (int)fb);
      else
        k_x1_gather<<<g1, 256, 0, s>>>(a, (int)fb);
    }
    switch (pl.mb * 4 + ns) {
#define TRALS_NE3_CASE(MB, NS)                                                                     \
  case MB * 4 + NS:                                                                                \
    if (e1)                                                                                        \
      hipExtLaunchKernelGGL((k_normal_eq_x3<MB, NS>), dim3(grid), dim3(512), x3_dyn_lds(MB, NS), s, nullptr, e1, \
                            0, a);                                                                 \
    else                                                                                           \
      k_normal_eq_x3<MB, NS><<<grid, 512, x3_dyn_lds(MB, NS), s>>>(a);                             \
    break;
      TRALS_NE3_CASE(1, 3)
      TRALS_NE3_CASE(2, 3)
      TRALS_NE3_CASE(3, 3)
      TRALS_NE3_CASE(4, 3)
      TRALS_NE3_CASE(1, 1)
      TRALS_NE3_CASE(2, 1)
      TRALS_NE3_CASE(3, 1)
      TRALS_NE3_CASE(4, 1)
#undef TRALS_NE3_CASE
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}


hipError_t launch_reduce_parts(const ReduceJob& a, const ReduceJob& b, int nparts, int P, const int* status,
                               hipStream_t s) {
  const int64_t na = reduce_blocks(a, P, nparts), nb = reduce_blocks(b, P, nparts);
  if (na + nb == 0) return hipSuccess;
  k_reduce_parts<<<(unsigned)(na + nb), 256, 0, s>>>(a, b, na, nparts, P, status);
  return hipGetLastError();
}

}  // namespace trals
