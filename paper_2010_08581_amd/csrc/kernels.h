// Launch wrappers of the gfx950 kernels (host side).  Each returns the launch's hipError_t.
#pragma once

#include "common.h"

namespace trals {

// ---- setup (one-time passes at handle creation) ----
// Mode-n panel: X viewed as [A][I_n][B] (A = prod_{k<n} I_k, B = prod_{k>n} I_k) is written
// as panel[a*B + b][i] = X[a][i][b], i.e. mode n contiguous, other modes in C order.
hipError_t launch_panel(const void* X, int x_dtype, void* panel, int p_dtype, int64_t A, int64_t In,
                        int64_t B, hipStream_t s);
// sum of squares (FP64) and count of non-finite entries of X; results in out[0] (double bits), out[1].
hipError_t launch_scan_x(const void* X, int x_dtype, int64_t n, double* partial, int nblocks,
                         unsigned long long* nonfinite, hipStream_t s);
hipError_t launch_sum_partials(const double* partial, int n, double* out, hipStream_t s);
// core import/export between C-order (Rp, I, Rn) and slice-major (I, Rp, Rn) storage.
hipError_t launch_core_import(const void* src, int src_dtype, void* dst, int dst_dtype, int Rp, int I,
                              int Rn, hipStream_t s);
hipError_t launch_core_export(const void* src, int src_dtype, void* dst, int dst_dtype, int Rp, int I,
                              int Rn, hipStream_t s);
hipError_t launch_core_normal(void* dst, int dst_dtype, int64_t count, uint64_t seed, uint64_t stream_id,
                              int core, hipStream_t s);

// ---- per update ----
struct SampleArgs {
  Ring ring;
  int n;
  int64_t J;
  uint64_t seed, stream_id, u;
  PerMode<const uint64_t> cdf;
  int32_t* idx;
  double* w;
  const int* status;
};
hipError_t launch_sample(const SampleArgs& a, hipStream_t s);

struct SketchArgs {
  Ring ring;
  int n;
  int64_t J;
  PerMode<const void> cores;  // slice-major cores in the compute type
  const int32_t* idx;
  const double* w;
  void* A;                    // J x P sketched design rows, column a*R_n + b
  const int* status;
};
hipError_t launch_sketch(const SketchArgs& a, int real_dtype, hipStream_t s);

// Fused normal equations [H | B] = A^T [A | X~] on FP64 matrix cores (split-K partials).
struct NormalEqArgs {
  const void* A;              // J x P sketched rows (compute type)
  const void* panel;          // mode-n panel (compute type)
  const int32_t* idx;         // J x (N-1)
  const double* w;
  int64_t stride[kMaxOrder];  // panel-row stride of the k-th sampled mode
  int K;                      // N-1
  int64_t J;
  int64_t chunk;              // sample rows per split
  int P, In;
  int gram_tiles;             // 64-wide column tiles of the Gram part
  double* Hpart;              // splits x P x P (lower triangle written)
  double* Bpart;              // splits x P x I_n
  const int* status;
};
struct NormalEqPlan {
  int mb;          // row tile = 16 * mb rows of P
  int row_tiles, gram_tiles, data_tiles;
  int splits;
  int64_t chunk;
};
constexpr int kPlanCUs = 256;  // MI355X compute units (launch sizing)
NormalEqPlan plan_normal_eq(int P, int In, int64_t J, int panel_bytes, int num_cu);
// real_dtype 0: FP64 sketch and panel; 1: FP32 sketch and panel (FP64 matrix cores);
// 2: BF16 form (FP32 sketch, BF16 panel, BF16 matrix cores with FP32 accumulation).
hipError_t launch_normal_eq(const NormalEqArgs& a, const NormalEqPlan& pl, int real_dtype, hipStream_t s);
// out = fixed-order sum of nparts partial arrays of count doubles (lower != 0: symmetrise a
// P x P matrix from its lower triangle).
hipError_t launch_reduce_parts(const double* parts, int nparts, int64_t count, int P, int lower, double* out,
                               const int* status, hipStream_t s);

// Blocked FP64 Cholesky of the SPD P x P matrix H (full storage, P <= 1024) into the factor
// buffer F (chol_factor_doubles(P) doubles).  A non-positive pivot sets *status = kDevSingular.
size_t chol_factor_doubles(int P);
hipError_t launch_chol_factor(int P, const double* H, double* F, int* status, hipStream_t s);
// With the factor F of H: mode 0 solves H Z = B (P x I_n) and writes lateral slice i of the
// core as column i of Z (compute type); mode 1 writes the leverage weights
// Q_i = floor(||L^{-1} g_i||^2 / P * 2^52) of the rows g_i of the core (B unused).
hipError_t launch_chol_solve(int P, int In, const double* F, const double* B, void* core, int real_dtype,
                             uint64_t* Q, int mode, const int* status, hipStream_t s);

// ---- leverage tables (eq. (3)) ----
hipError_t launch_lev_uniform(int In, uint64_t* Q, const int* status, hipStream_t s);
hipError_t launch_scan_u64(uint64_t* Q, int In, const int* status, hipStream_t s);

// ---- fit error ----
struct FitArgs {
  Ring ring;
  PerMode<const void> cores;  // slice-major
  const void* X;              // C-order data (= panel of mode N-1)
  int64_t rows;               // prod_{k<N-1} I_k
  double* partial;            // one per block
};
hipError_t launch_fit(const FitArgs& a, int real_dtype, int x_dtype, int* nblocks_out, hipStream_t s);

}  // namespace trals
