// Launch wrappers of the gfx950 kernels (host side).  Each returns the launch's hipError_t.
#pragma once

#include "common.h"

namespace trals {

// ---- setup (one-time passes at handle creation) ----
// Mode-n panel: X viewed as [A][I_n][B] (A = prod_{k<n} I_k, B = prod_{k>n} I_k) is written
// as panel[a*B + b][i] = X[a][i][b], i.e. mode n contiguous, other modes in C order.
hipError_t launch_panel(const void* X, int x_dtype, void* panel, int p_dtype, int64_t A, int64_t In,
                        int64_t B, hipStream_t s);
// sum of squares (FP64, finite entries) into nblocks partials, and the count of non-finite
// entries added to *nonfinite (skipped when nonfinite is NULL).
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
// Fused sampler and sketch: draws J tuples (indices idx[j * (N-1) + k], rescaling w[j]) and
// writes the J x P sketched rows A (column a*R_n + b = w_j M_j(b, a)).
struct DrawArgs {
  Ring ring;
  int n;
  int64_t J;
  uint64_t seed, stream_id, u;
  PerMode<const uint64_t> cdf;
  PerMode<const double> cores;  // slice-major FP64 cores
  int32_t* idx;
  double* w;
  void* A;                      // sketch type: FP64 (0) or FP32 (1): J x P rows; BF16 pair (2):
                                // bf16(w M) transposed, P x ldt (samples contiguous per column)
  void* A2;                     // BF16 pair only: bf16(w^2 M), same layout
  int64_t ldt;                  // BF16 pair only: row length (a multiple of 64 samples)
  const int* status;
  int weights;                  // 1: cdf holds the weights Q (scanned in LDS); 0: inclusive sums C
  int mfma_chain;               // BF16 sketch: 1 = subchain products on BF16 matrix cores
  int draw;                     // 1: draw the samples; 0: take idx as given, rows without weights
  // with draw == 0: 1 = row j is the j-th index tuple in the order of the mode-n panel's rows
  // (digit k = (j / en_stride[k]) mod I of the k-th mode after n; idx is not read) and
  // w[j] = 1 is written (the full design matrix of Algorithm 1)
  int enumerate;
  int64_t en_stride[kMaxOrder];
  int jb;                       // samples per workgroup (set by launch_draw)
  int tables_in_lds;            // set by launch_draw
};
constexpr size_t kDrawTableBytes = 48 * 1024;  // sampling tables staged per draw workgroup
hipError_t launch_draw(const DrawArgs& a, int sketch_dtype, hipStream_t s);

// Fused normal equations [H | B] = A^T [A | X~] on matrix cores (split-K partials).
struct NormalEqArgs {
  const void* A;              // J x P sketched rows (compute type); BF16: bf16(w M), P x ld
  const void* A2;             // BF16 only: bf16(w^2 M), P x ld
  int64_t ld;                 // BF16 only: row length of A, A2 (a multiple of 64)
  const void* panel;          // mode-n panel (compute type)
  const int32_t* idx;         // J x (N-1)
  const double* w;
  int64_t stride[kMaxOrder];  // panel-row stride of the k-th sampled mode
  int K;                      // N-1
  int64_t J;
  int64_t chunk;              // sample rows per split
  int P, In;
  int gram_tiles;             // column tiles of the Gram part (64 wide; 128, ne_dtype 2 and 3)
  int col_tiles, tiles, splits;  // filled in by launch_normal_eq (ne_dtype 2 and 3: tiles = the
  int row_tiles;                 // tiles a split computes, strictly upper Gram tiles left out)
  double* Hpart;              // splits x P x P (lower triangle written)
  double* Bpart;              // splits x P x I_n
  int direct;                 // 1: the fiber of sample j is row j of `panel` (I_n wide)
  const int* status;
  // FP32 path (ne_dtype 3): the sketch rows A (FP32, J x P row-major) in three BF16 slices per
  // 64-sample block and column, slice s of column p at S3 + (s P + p) ld (ld samples per
  // column, a multiple of 64), with block exponents E[b P + p]; the weighted fibers w_j X(j, i)
  // in the same form, slice s of column i at D3 + (s I_n + i) ld, exponents ED[b I_n + i].
  // launch_normal_eq writes all four (split pass) before the contraction reads them.  The BF16
  // form uses D3 for the gathered raw BF16 fibers, I_n x ld, and, with x1_rows, S3 for its two
  // sketches bf16(w M) and bf16(w^2 M) (P x ld each, one after the other), rounded and
  // transposed by the gather pass from the FP32 rows A = w M (J x P); without x1_rows the draw
  // wrote them transposed into A and A2.
  __bf16* S3;
  int* E;
  void* D3;
  int* ED;
  int x1_rows;
};
struct NormalEqPlan {
  int mb;          // row tile = 16 * mb rows of P
  int row_tiles, gram_tiles, data_tiles;
  int splits;
  int64_t chunk;
};
constexpr int kPlanCUs = 256;  // MI355X compute units (launch sizing)
// rows of finite padding the sketch buffer keeps past row J (the contraction reads up to one
// split quantum past the end of a chunk without bounds checks)
constexpr int kSketchPadRows = 64;
// ne_dtype 0: FP64 sketch and panel (FP64 matrix cores); 1: FP32 sketch and panel, widened
// exactly to FP64 and multiplied on the FP64 matrix cores (FP64 accumulation); 2: BF16 form
// (two transposed BF16 sketches A = bf16(w M), A2 = bf16(w^2 M), P x ld, BF16 panel, BF16
// matrix cores with FP32 accumulation over each 64-sample block, FP64 across blocks); 3: FP32
// path on BF16 matrix cores with exact products: the FP32 sketch and the weighted FP32 fibers
// in three 8-bit slices per 64-sample block and column (one exponent each), slice products
// exact in FP32, block sums added in FP64.  For ne_dtype 2 and 3 the launch is two kernels: the
// gather pass (the raw BF16 fibers into D3, I_n x ld) or the split pass (slices of the sketch
// into S3 / E and of the gathered weighted fibers w_j X(j, :) into D3 / ED), then the products;
// e0 stamps the first one's start, e1 the second one's end.
NormalEqPlan plan_normal_eq(int P, int In, int64_t J, int ne_dtype, int num_cu);
// e0/e1 (optional, for measurement): events stamped at the kernel's own start and end
hipError_t launch_normal_eq(const NormalEqArgs& a, const NormalEqPlan& pl, int ne_dtype, hipStream_t s,
                            hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Three-slice form of an FP32 operand (the sketch rows, the weighted fibers) for ne_dtype 3:
// per block b of 64 samples and column p, e = E[b ncols + p] with max_j |V(j, p)| < 2^e over
// the block, and V(j, p) = 2^(e-8) (s0 + 2^-8 s1 + 2^-16 s2) + r, |r| <= 2^(e-25), with
// integers |s0| <= 256, |s1|, |s2| <= 128 stored as BF16 (exact).  Samples past J are zero.
constexpr int kSplitBlock = 64;  // samples per exponent block of the three-slice sketch

// out = fixed-order sum of nparts partial arrays of count doubles.  mode 0: as is; mode 1:
// symmetrise a P x P matrix from its lower triangle; mode 2: transpose P x (count / P) to
// (count / P) x P; mode 3: P x P partials (P % 16 == 0, lower triangle read) into the
// block-packed lower blocks of the symmetric matrix (count = its packed doubles, padding column
// zero).  Two independent reductions share one launch.
struct ReduceJob {
  const double* parts;
  int64_t count;
  int mode;
  double* out;
};
hipError_t launch_reduce_parts(const ReduceJob& a, const ReduceJob& b, int nparts, int P, const int* status,
                               hipStream_t s);

// K = A^T A (P x P row-major, lower blocks incl. full diagonal blocks) of an FP64 rows x P
// matrix A, row-major (trans = false) or column-major (trans = true: then K = G G^T of the
// row-major P x rows matrix G that A's storage holds).  clear (optional): a word the launch
// sets to 0 (the failure word of the factorisation that follows).  packed (P % 16 == 0): K is
// written block-packed instead (kPackBlk doubles per lower block, padding column zero), as the
// blocked factorisation's work matrix (chol_packed_input, CholArgs.prepacked).
hipError_t launch_syrk(const double* A, int64_t rows, int P, double* K, const int* status, hipStream_t s,
                       bool trans = false, int* clear = nullptr, bool packed = false);

// Cholesky factorisation of an SPD P x P matrix H (full storage, lower triangle read,
// P <= 1024) into the inverse factor W = L^{-1} (chol_factor_doubles(P) doubles,
// block-packed).  A pivot of row k < P at or below the tolerance (rel_tol, or P eps when
// rel_tol is 0, times the largest diagonal entry of H) is a breakdown: it sets *fail if fail is
// given (the handle goes on: a table factorisation then falls back), else *status.
// Block-packed lower-triangular storage of the factorisations: 16 x 16 blocks of kPackLd
// doubles per row (column 16 is padding), block (i, j), i >= j, at slot i (i + 1) / 2 + j.
constexpr int kPackLd = 17;
constexpr int kPackBlk = 16 * kPackLd;
__host__ __device__ __forceinline__ int slot(int i, int j) { return i * (i + 1) / 2 + j; }
__device__ __forceinline__ void slot_ij(int sl, int& i, int& j) {
  int r = (int)((sqrtf(8.0f * (float)sl + 1.0f) - 1.0f) * 0.5f);
  while ((r + 1) * (r + 2) / 2 <= sl) ++r;
  while (r * (r + 1) / 2 > sl) --r;
  i = r;
  j = sl - r * (r + 1) / 2;
}

struct CholArgs {
  int P;
  const double* H;  // P x P, row-major (lower triangle and diagonal read)
  double* W;        // chol_work_doubles(P): the block-packed inverse factor first
  int* status;
  int* fail;         // optional breakdown word (kernels after a breakdown skip their work)
  double rel_tol;    // 0: P eps
  int factor_only;   // 1: only the factor's diagonal regions of W are needed (large P: the
                     // off-diagonal bands of W are skipped)
  int prepacked;     // large P with P % 16 == 0: the work matrix (chol_packed_input(W, P))
                     // already holds H block-packed; the first step takes the tolerance
  // set by launch_chol for large P: work matrix, panel blocks of L, tolerance, and the diagonal
  // region of a step
  double* Lg;
  double* Lp;
  double* scal;
  int b0, nb;
  int pb0, pnb;  // the previous step's region (pnb = 0: none), whose trailing update of this
                 // region the step applies first
};
size_t chol_factor_doubles(int P);  // the block-packed factor W
size_t chol_work_doubles(int P);    // W plus the staging blocks k_chol uses (size of CholArgs.W)
// beside (optional, single-workgroup factorisations only): a reduction run by extra
// workgroups of the same launch, independent of the factorisation
hipError_t launch_chol(const CholArgs& a, hipStream_t s, const ReduceJob* beside = nullptr, int nparts = 0);
bool chol_single_workgroup(int P);  // the factorisation runs as one workgroup (P <= 144)
// large P: where the blocked factorisation keeps its block-packed work matrix inside W (the
// destination of a reduction of H in mode 3, CholArgs.prepacked), and whether it may be used
bool chol_prepack_ok(int P);
double* chol_packed_input(double* W, int P);

// With inverse factors: solve rows z_i = W^T W b_i of Bsol (In_sol x P) into core (row i), and
// table weights Q_i = floor(||W g_i||^2 / P * 2^52) of the rows of Blev (In_lev x P, a core
// unfolding).  Either part is skipped when its W is NULL.  When *lev_fail is set (the core
// Gram's factorisation broke down) the table comes from the pivoted QR of Blev instead
// (levqr.h), with qr_work (In_lev * P doubles) as its work memory; with qr_work NULL the
// table is left to a later launch.
struct TriArgs {
  int P, In_sol, In_lev;
  const double* Wsol;
  const double* Wlev;
  const double* Bsol;
  const double* Blev;
  double* core;
  uint64_t* Q;
  int solve_groups, lev_groups;  // set by launch_trisolve
  int* status;
  const int* lev_fail;
  double* qr_work;
  // optional: the solve workgroup that finishes last (counted on *last_counter, which must be 0
  // at launch and is left 0) takes the table Q of the new core (core, In_sol x P) from its
  // pivoted QR when *core_fail is set, with fallback_work (In_sol * P doubles)
  int* last_counter;
  const int* core_fail;
  double* fallback_work;
  // optional, a solve without leverage rows for P > 128: work memory of
  // solve_split_doubles(In_sol, P) doubles; the solve then runs as two launches, each spread
  // over several workgroups per 16-row group (the same block products in the same order)
  double* split_work;
};
hipError_t launch_trisolve(const TriArgs& a, hipStream_t s);
size_t solve_split_doubles(int In, int P);

// Sampling table of a wide core (I <= P: G_(2) is I x P, slice-major).  The row Gram G G^T is
// factored with tolerance rel_tol; if it factors, G_(2) has full row rank and p_i = 1/I
// exactly; otherwise the table comes from the pivoted QR of G_(2) (levqr.h).  For I <= 144 one
// launch does all of it (Gram into K, factorisation in LDS, table); above, the Gram and the
// blocked factorisation are separate launches (CholArgs with fail) and launch_lev_fallback
// writes the table.  K: I x I doubles, F: chol_work_doubles(I), qr_work: I * P doubles.
// Without qr_work a breakdown only sets *fail (cleared otherwise) and Q is not written.
struct LevWideArgs {
  const double* G;
  int I, P;
  double* K;
  double* F;
  double* qr_work;
  uint64_t* Q;
  int* status;
  int* fail;
  double rel_tol;
  const int* run_if;  // optional: the launch does nothing unless *run_if != 0
};
hipError_t launch_lev_wide(const LevWideArgs& a, hipStream_t s);
// table from *fail: uniform (1/I) if it is clear, else the pivoted QR of G (one workgroup)
hipError_t launch_lev_fallback(const double* G, int I, int P, double* qr_work, uint64_t* Q, const int* fail,
                               int* status, hipStream_t s);
constexpr double kTableRelTol = 1e-8;  // pivot tolerance of the table factorisations
// Two independent single-workgroup jobs in one launch (both sizes must satisfy
// chol_single_workgroup): the factorisation a0, beside either the factorisation *a1 or the
// whole table of the wide matrix *lw (exactly one of a1, lw non-null).
// clear (optional): an int the launch sets to 0 first (the solve's completion counter below)
hipError_t launch_chol_pair(const CholArgs& a0, const CholArgs* a1, const LevWideArgs* lw, hipStream_t s,
                            int* clear = nullptr);

// ---- generated data source and transfer-matrix inner products ----
// Sampled fibers of X = TR(G*) + sigma Z: out[j][i] = sum_p G*_n[i][p] T[j][p] + sigma z(lin),
// T[j] the true-core subchain product of sample j (column order of the sketch), lin the C-order
// linear index of the entry (lin_stride[k] of the k-th sampled mode, lin_stride_n of mode n).
struct FiberArgs {
  int64_t J;
  int P, In, K;
  const double* T;
  const int32_t* idx;
  int64_t lin_stride[kMaxOrder];
  int64_t lin_stride_n;
  const double* true_core;    // slice-major I_n x P, FP64
  const double* sigma;        // device scalar
  uint64_t noise_seed, noise_stream;
  void* out;                  // J x I_n, panel type
  const int* status;
};
hipError_t launch_fibers(const FiberArgs& a, int out_dtype, hipStream_t s);
// *sigma = noise_rel sqrt(*t2 / entries) (*status = kDevSingular if *t2 is not positive and finite)
hipError_t launch_source_scale(const double* t2, double noise_rel, double entries, double* sigma, int* status,
                               hipStream_t s);
// *fit = sqrt(max(0, r[0] - 2 r[1] + r[2]) / r[2]) (distance of two rings relative to the second)
hipError_t launch_clean_fit(const double* r, double* fit, hipStream_t s);
// *fit = sqrt(*r2 / x2)
hipError_t launch_dense_fit(const double* r2, double x2, double* fit, hipStream_t s);
// *fit = sqrt(*r2 / *x2) (both on the device)
hipError_t launch_dense_fit_dev(const double* r2, const double* x2, double* fit, hipStream_t s);
// *out = <TR(A), TR(B)> for two rings with equal mode sizes (FP64 slice-major cores); work:
// ring_inner_doubles(ra, rb) doubles.
size_t ring_inner_doubles(const Ring& ra, const Ring& rb);
hipError_t launch_ring_inner(const Ring& ra, PerMode<const double> A, const Ring& rb, PerMode<const double> B,
                             double* work, double* out, hipStream_t s);

// ---- leverage tables (eq. (3)) ----
// Normalisation of core n after its update: G_n <- Q, G_{n+1} <- R G_{n+1} with G_n = Q R (the
// (I_n R_{n-1}) x R_n unfolding, R upper with positive diagonal).  S: R x R scratch for the
// Gram; work: gauge_work_doubles() doubles.  A singular Gram sets *status = kDevSingular.
size_t gauge_work_doubles();
hipError_t launch_gauge(double* core, int64_t In, int Rp, int R, double* next, int64_t In_next, int Rnext,
                        double* S, double* work, int* status, hipStream_t s);
hipError_t launch_lev_uniform(int In, uint64_t* Q, const int* status, hipStream_t s);
hipError_t launch_scan_u64(uint64_t* Q, int In, const int* status, hipStream_t s);
// One workgroup: Q <- Qalt (In entries) if *status is clear and *fail is set, and *redo = kDevOk
// in that case, kDevIdle otherwise
hipError_t launch_table_settle(const int* fail, const int* status, const uint64_t* Qalt, uint64_t* Q, int In, int* redo,
                               hipStream_t s);

// ---- fit error ----
constexpr int kFitRows = 8;       // rows of X (C order, last mode contiguous) per fit block
constexpr int kScanBlocks = 1024; // blocks (partial sums) of the ||X||^2 scan
struct FitArgs {
  Ring ring;
  PerMode<const void> cores;  // slice-major
  const void* X;              // C-order data (= panel of mode N-1)
  int64_t rows;               // prod_{k<N-1} I_k
  double* partial;            // one per block
};
hipError_t launch_fit(const FitArgs& a, int real_dtype, int x_dtype, int* nblocks_out, hipStream_t s);

// Sampled squared residual (estimate of the fit error from S uniform entries, Philox counter
// (s, tag, 0, 1), index floor(r E / 2^64)): per-block sums into partial (at most
// kFitSampleBlocks of them; *nblocks_out receives the count).  Cores FP64 slice-major.
struct FitSampleArgs {
  Ring ring;
  PerMode<const void> cores;
  const void* X;  // C order (= panel of mode N-1)
  int64_t E, S;
  uint64_t seed, stream_id, tag;
  double* partial;
};
constexpr int kFitSampleBlocks = 256;
hipError_t launch_fit_sample(const FitSampleArgs& a, int x_dtype, int* nblocks_out, hipStream_t s);

}  // namespace trals
