// Normal equations of the sampled least-squares problem (Algorithm 2, LS step) on FP64 matrix
// cores, fused with the fiber gather (Algorithm 2, "sample X"):
//
//     [ H | B ] = A^T [ A | X~ ],   A = J x P sketched design rows,  X~(j, :) = w_j X(..., :, ...)
//
// One launch covers both products.  The extended column space holds the P Gram columns (read
// from A, padded to a multiple of 64) followed by the I_n data columns (gathered from the
// mode-n panel, where row j's fiber is contiguous).  A workgroup owns a (16 MB) x 64 output
// tile and one chunk of sample rows; its four waves each own 16 columns and all MB row blocks
// and run v_mfma_f64_16x16x4 on FP64 operands (FP32 storage is widened exactly on the way into
// LDS).  Gram tiles strictly above the diagonal are skipped; consumers read H's lower triangle.
// Partial tiles per sample chunk are reduced afterwards in a fixed order (deterministic).
#include "kernels.h"

namespace trals {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kColTile = 64;
constexpr int kKB = 32;         // sample rows per LDS stage (8 MFMA k-steps)
constexpr int kMaxChunk = 512;  // sample rows per split (row offsets and weights cached in LDS)

template <typename Real, int MB>
__global__ __launch_bounds__(256) void k_normal_eq(NormalEqArgs a) {
  constexpr int RT = 16 * MB;
  constexpr int NA = (kKB * RT + 255) / 256;        // A elements per thread per stage
  constexpr int NB = (kKB * kColTile + 255) / 256;  // B elements per thread per stage
  __shared__ Real As[2][kKB][RT + 1];
  __shared__ Real Bs[2][kKB][kColTile + 1];
  __shared__ int64_t s_roff[kMaxChunk];
  __shared__ double s_w[kMaxChunk];
  if (*a.status != kDevOk) return;
  const int P = a.P, In = a.In;
  const int ct = blockIdx.x, rt = blockIdx.y, s = blockIdx.z;
  const int row0 = rt * RT;
  const bool gram = ct < a.gram_tiles;
  const int col0 = gram ? ct * kColTile : (ct - a.gram_tiles) * kColTile;
  if (gram && col0 >= row0 + RT) return;  // strictly upper Gram tile
  const int64_t r0 = (int64_t)s * a.chunk;
  const int64_t r1 = r0 + a.chunk < a.J ? r0 + a.chunk : a.J;
  const int nrows = (int)(r1 - r0);
  const Real* A = (const Real*)a.A;
  const Real* X = (const Real*)a.panel;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // weights and panel-row offsets of the whole chunk (data tiles)
  if (!gram) {
    for (int r = threadIdx.x; r < nrows; r += 256) {
      const int32_t* ij = a.idx + (r0 + r) * a.K;
      int64_t off = 0;
      for (int k = 0; k < a.K; ++k) off += (int64_t)ij[k] * a.stride[k];
      s_roff[r] = off * In;
      s_w[r] = a.w[r0 + r];
    }
    __syncthreads();
  }
  Real ra[NA], rb[NB];
  auto load_stage = [&](int base) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int r = e / RT, c = e % RT;
      ra[q] = (e < kKB * RT && base + r < nrows && row0 + c < P) ? A[(r0 + base + r) * P + row0 + c] : Real(0);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int r = e / kColTile, c = e % kColTile;
      Real v = Real(0);
      if (base + r < nrows) {
        if (gram) {
          if (col0 + c < P) v = A[(r0 + base + r) * P + col0 + c];
        } else {
          if (col0 + c < In) v = X[s_roff[base + r] + col0 + c];
        }
      }
      rb[q] = v;
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < kKB * RT) As[buf][e / RT][e % RT] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = threadIdx.x + 256 * q;
      Bs[buf][e / kColTile][e % kColTile] = rb[q];
    }
  };
  d4 acc[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
  const int stages = (nrows + kKB - 1) / kKB;
  load_stage(0);
  for (int t = 0; t < stages; ++t) {
    const int buf = t & 1;
    store_stage(buf);
    __syncthreads();
    if (t + 1 < stages) load_stage((t + 1) * kKB);
#pragma unroll
    for (int ks = 0; ks < kKB / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      double b = (double)Bs[buf][kr][wave * 16 + (lane & 15)];
      if (!gram) b *= s_w[t * kKB + kr < nrows ? t * kKB + kr : 0];
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const double av = (double)As[buf][kr][m * 16 + (lane & 15)];
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[m], 0, 0, 0);
      }
    }
  }
  // D(i, j) of each 16 x 16 block sits in lane j + 16 (i % 4), register i / 4
  const int col = col0 + wave * 16 + (lane & 15);
  if (gram) {
    double* H = a.Hpart + (int64_t)s * P * P;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + m * 16 + 4 * r + (lane >> 4);
        if (row < P && col < P && col <= row) H[(int64_t)row * P + col] = acc[m][r];
      }
  } else {
    double* B = a.Bpart + (int64_t)s * P * In;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + m * 16 + 4 * r + (lane >> 4);
        if (row < P && col < In) B[(int64_t)row * In + col] = acc[m][r];
      }
  }
}

// BF16 form of the same products on v_mfma_f32_16x16x32_bf16: operands rounded to BF16
// (round to nearest even), products accumulated in FP32 within a sample chunk, partial tiles
// written in FP64.  Gram tiles use bf16(A) on both sides; data tiles use bf16(w_j A_j) against
// the raw BF16 panel rows (w_j folded into the sketch side, so the gathered fibers feed the
// matrix cores unmodified).  LDS tiles are stored k-major ([column][sample]) so that each lane
// reads its 8 consecutive k values of an operand with one 16-byte load.
//   v_mfma_f32_16x16x32_bf16 layouts: A(i, k) at lane i + 16 (k / 8), element k % 8;
//   B(k, j) at lane j + 16 (k / 8), element k % 8; D(i, j) at lane j + 16 (i / 4), register i % 4.
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kKB16 = 64;  // sample rows per stage (two MFMA k-steps of 32)
constexpr int kPadK = 8;   // k padding of the LDS rows (bf16 elements)

template <int MB>
__global__ __launch_bounds__(256) void k_normal_eq_bf16(NormalEqArgs a) {
  constexpr int RT = 16 * MB;
  constexpr int LK = kKB16 + kPadK;
  constexpr int NA = (kKB16 * RT + 255) / 256;
  constexpr int NB = (kKB16 * kColTile + 255) / 256;
  __shared__ __bf16 As[2][RT][LK];
  __shared__ __bf16 Bs[2][kColTile][LK];
  __shared__ int64_t s_roff[kMaxChunk];
  __shared__ float s_w[kMaxChunk];
  if (*a.status != kDevOk) return;
  const int P = a.P, In = a.In;
  const int ct = blockIdx.x, rt = blockIdx.y, s = blockIdx.z;
  const int row0 = rt * RT;
  const bool gram = ct < a.gram_tiles;
  const int col0 = gram ? ct * kColTile : (ct - a.gram_tiles) * kColTile;
  if (gram && col0 >= row0 + RT) return;
  const int64_t r0 = (int64_t)s * a.chunk;
  const int64_t r1 = r0 + a.chunk < a.J ? r0 + a.chunk : a.J;
  const int nrows = (int)(r1 - r0);
  const float* A = (const float*)a.A;
  const __bf16* X = (const __bf16*)a.panel;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (!gram) {
    for (int r = threadIdx.x; r < nrows; r += 256) {
      const int32_t* ij = a.idx + (r0 + r) * a.K;
      int64_t off = 0;
      for (int k = 0; k < a.K; ++k) off += (int64_t)ij[k] * a.stride[k];
      s_roff[r] = off * In;
      s_w[r] = (float)a.w[r0 + r];
    }
    __syncthreads();
  }
  float ra[NA];
  __bf16 rb[NB];
  auto load_stage = [&](int base) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int r = e / RT, c = e % RT;
      float v = 0.f;
      if (e < kKB16 * RT && base + r < nrows && row0 + c < P) {
        v = A[(r0 + base + r) * P + row0 + c];
        if (!gram) v *= s_w[base + r];
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = threadIdx.x + 256 * q;
      const int r = e / kColTile, c = e % kColTile;
      __bf16 v = (__bf16)0.f;
      if (base + r < nrows) {
        if (gram) {
          if (col0 + c < P) v = (__bf16)A[(r0 + base + r) * P + col0 + c];
        } else {
          if (col0 + c < In) v = X[s_roff[base + r] + col0 + c];
        }
      }
      rb[q] = v;
    }
  };
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q;
      if (e < kKB16 * RT) As[buf][e % RT][e / RT] = (__bf16)ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = threadIdx.x + 256 * q;
      Bs[buf][e % kColTile][e / kColTile] = rb[q];
    }
  };
  f4 acc[MB];
#pragma unroll
  for (int m = 0; m < MB; ++m) acc[m] = f4{0.f, 0.f, 0.f, 0.f};
  const int stages = (nrows + kKB16 - 1) / kKB16;
  load_stage(0);
  for (int t = 0; t < stages; ++t) {
    const int buf = t & 1;
    store_stage(buf);
    __syncthreads();
    if (t + 1 < stages) load_stage((t + 1) * kKB16);
#pragma unroll
    for (int ks = 0; ks < kKB16 / 32; ++ks) {
      const int k0 = ks * 32 + 8 * (lane >> 4);
      const bf8 b = *(const bf8*)&Bs[buf][wave * 16 + (lane & 15)][k0];
#pragma unroll
      for (int m = 0; m < MB; ++m) {
        const bf8 av = *(const bf8*)&As[buf][m * 16 + (lane & 15)][k0];
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, acc[m], 0, 0, 0);
      }
    }
  }
  const int col = col0 + wave * 16 + (lane & 15);
  if (gram) {
    double* H = a.Hpart + (int64_t)s * P * P;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + m * 16 + 4 * (lane >> 4) + r;
        if (row < P && col < P && col <= row) H[(int64_t)row * P + col] = (double)acc[m][r];
      }
  } else {
    double* B = a.Bpart + (int64_t)s * P * In;
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + m * 16 + 4 * (lane >> 4) + r;
        if (row < P && col < In) B[(int64_t)row * In + col] = (double)acc[m][r];
      }
  }
}

// out[e] = sum_s parts[s * count + e] in a fixed order.  With lower != 0 the P x P matrix is
// symmetrised from its lower triangle: out(i, j) = sum_s parts_s(max(i,j), min(i,j)).
__global__ __launch_bounds__(256) void k_reduce_parts(const double* __restrict__ parts, int nparts, int64_t count,
                                                      int P, int lower, double* __restrict__ out,
                                                      const int* status) {
  if (*status != kDevOk) return;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t src = e;
    if (lower) {
      const int i = (int)(e / P), j = (int)(e % P);
      src = i >= j ? e : (int64_t)j * P + i;
    }
    double acc = 0.0;
#pragma unroll 8
    for (int s = 0; s < nparts; ++s) acc += parts[s * count + src];
    out[e] = acc;
  }
}

template <typename Real>
hipError_t dispatch(const NormalEqArgs& a, int mb, dim3 grid, hipStream_t s) {
  switch (mb) {
#define TRALS_NE_CASE(MB) \
  case MB: k_normal_eq<Real, MB><<<grid, 256, 0, s>>>(a); break;
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

NormalEqPlan plan_normal_eq(int P, int In, int64_t J, int panel_bytes, int num_cu) {
  NormalEqPlan pl;
  // row tile of 16 * mb rows: one tile when P <= 128, else the mb in [4, 8] with least padding
  if (P <= 128) {
    pl.mb = (P + 15) / 16;
  } else {
    int best = 8, best_pad = 1 << 30;
    for (int mb = 8; mb >= 4; --mb) {
      const int rt = 16 * mb;
      const int pad = (P + rt - 1) / rt * rt - P;
      if (pad < best_pad) {
        best_pad = pad;
        best = mb;
      }
    }
    pl.mb = best;
  }
  pl.row_tiles = (P + 16 * pl.mb - 1) / (16 * pl.mb);
  pl.gram_tiles = (P + kColTile - 1) / kColTile;
  pl.data_tiles = (In + kColTile - 1) / kColTile;
  const int64_t tiles = (int64_t)pl.row_tiles * (pl.gram_tiles + pl.data_tiles);
  // split the samples so that the launch holds ~3 workgroups per CU, but keep the FP64 partial
  // traffic below the gathered bytes and every chunk at least one LDS stage long
  int64_t S = (3 * (int64_t)num_cu + tiles - 1) / tiles;
  if (In > 0) {
    const int64_t cap_bytes = (2 * J * In * panel_bytes) / (8 * (int64_t)P * (P + In)) + 1;
    if (S > cap_bytes) S = cap_bytes;
  }
  if (S > J / kKB) S = J / kKB;
  if (S < (J + kMaxChunk - 1) / kMaxChunk) S = (J + kMaxChunk - 1) / kMaxChunk;
  if (S < 1) S = 1;
  if (S > 65535) S = 65535;
  int64_t chunk = (J + S - 1) / S;
  chunk = (chunk + kKB - 1) / kKB * kKB;
  pl.chunk = chunk;
  pl.splits = (int)((J + chunk - 1) / chunk);
  return pl;
}

hipError_t launch_normal_eq(const NormalEqArgs& a, const NormalEqPlan& pl, int real_dtype, hipStream_t s) {
  dim3 grid(pl.gram_tiles + pl.data_tiles, pl.row_tiles, pl.splits);
  if (real_dtype == 0) return dispatch<double>(a, pl.mb, grid, s);
  if (real_dtype == 1) return dispatch<float>(a, pl.mb, grid, s);
  if (real_dtype == 2) {
    switch (pl.mb) {
#define TRALS_NE16_CASE(MB) \
  case MB: k_normal_eq_bf16<MB><<<grid, 256, 0, s>>>(a); break;
      TRALS_NE16_CASE(1)
      TRALS_NE16_CASE(2)
      TRALS_NE16_CASE(3)
      TRALS_NE16_CASE(4)
      TRALS_NE16_CASE(5)
      TRALS_NE16_CASE(6)
      TRALS_NE16_CASE(7)
      TRALS_NE16_CASE(8)
#undef TRALS_NE16_CASE
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_parts(const double* parts, int nparts, int64_t count, int P, int lower, double* out,
                               const int* status, hipStream_t s) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  k_reduce_parts<<<(unsigned)blocks, 256, 0, s>>>(parts, nparts, count, P, lower, out, status);
  return hipGetLastError();
}

}  // namespace trals
