/*
 * trals.h -- C ABI of the MI355X (gfx950) sampled tensor-ring ALS library.
 *
 * The library fits a tensor ring (TR) decomposition X ~ TR(G^(0..N-1)) to a
 * dense N-way tensor by leverage-score-sampled alternating least squares
 * (Malik & Becker, ICML 2021, Algorithm 2 "TR-ALS-Sampled").  Per core update
 * n it draws J index tuples from the product of the other cores' leverage
 * distributions (Algorithm 3, eqs. (3)-(4)), forms the J sampled rows of the
 * design matrix from lateral-slice products (Algorithm 4, eq. (5)), gathers
 * the J sampled mode-n fibers of X (Algorithm 2, "sample X"), solves the
 * sampled least-squares problem (Algorithm 2, LS step) and recomputes the
 * leverage distribution of the new core (eq. (3)).  The cores are held in FP64
 * in every precision; the precision selects the storage of the data panels and
 * the sketched rows and the arithmetic of their products.
 *
 * Conventions
 *  - Indices are 0-based.  X is a C-order array X[i_0, ..., i_{N-1}] (last
 *    index fastest), which differs from the paper's first-index-fastest
 *    linearisation (Section 2); only the row order of the sampled systems
 *    depends on it, not their solution.
 *  - Core n has shape (R[(n+N-1)%N], I[n], R[n]) (Section 2.1: ring closure
 *    R_0 = R_N).  The cores exchanged through this ABI are stored one after
 *    the other, each in C order.
 *  - All pointers named *_dev are device pointers on the current HIP device.
 *    Host arrays are read during the call only.
 *  - Every call returns a trals_status (0 on success) and never throws.
 *  - Asynchrony: trals_create, trals_sweep and trals_step enqueue work on the
 *    caller's stream.  trals_sweep/trals_step synchronise that stream once at
 *    the end to report a failed solve; trals_fit_error, trals_get_cores and
 *    trals_get_last_samples synchronise it as well.
 *  - A handle must not be used from two threads at once.
 *  - The workspace is owned by the caller, must stay allocated until
 *    trals_destroy, and is used for everything the handle keeps on the GPU
 *    (data panels, cores, sampling tables, samples, partial sums).  The
 *    library itself allocates no device memory.
 */
#ifndef TRALS_H
#define TRALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct trals_ctx* trals_handle;

typedef enum {
  TRALS_OK = 0,
  TRALS_EINVAL = -1,     /* bad argument: shape, rank, J, dtype, NaN/Inf in X, small workspace */
  TRALS_ENOMEM = -2,     /* host allocation failed */
  TRALS_ESINGULAR = -3,  /* sampled normal equations not positive definite, or an all-zero
                            core (no sampling distribution); the core being updated is left
                            unchanged */
  TRALS_EHIP = -4,       /* a HIP runtime call failed */
  TRALS_ESTATE = -5,     /* handle is in a failed state (reset it with trals_set_cores) */
  TRALS_ERANGE = -6,     /* trals_fit_error_noalloc: the problem's scratch exceeds the library's
                            fixed scratch array (TRALS_NOALLOC_SCRATCH_BYTES) */
  TRALS_PENDING = 1      /* trals_query: work still running on the stream */
} trals_status;

typedef enum {
  TRALS_F64 = 0,   /* IEEE double */
  TRALS_F32 = 1,   /* IEEE single */
  TRALS_BF16 = 2,  /* bfloat16 (precision TRALS_BF16 selects the BF16 form: BF16 data panels
                      and sketch on matrix cores with FP32 accumulation, FP64 Gram/Cholesky;
                      the subchain rows formed in FP64 and rounded once to BF16) */
  TRALS_BF16_CHAINS = 3  /* precision only: the BF16 form with the subchain products (Algorithm 4)
                            also on BF16 matrix cores, FP32 accumulation, each operand a pair of
                            BF16 values (about 16 bits) */
  /* TRALS_F32: FP32 data panels and sketch with FP64 sums: multiplied on the FP64 matrix cores
     (FP32 operands widen exactly) when every R[n-1]R[n] <= 128, else on the BF16 matrix cores as
     three 8-bit slices per operand (exact products); TRALS_F64: FP64 throughout. */
} trals_dtype;

typedef enum {
  TRALS_LEVERAGE = 0,  /* Algorithm 2: samples drawn from the leverage-score distributions (3) */
  TRALS_UNIFORM = 1,   /* Algorithm 2 with every p^(m) uniform (Section 4's uniform-sampling
                          comparison): same draws, sketch and solve, no leverage computation */
  TRALS_EXACT = 2      /* Algorithm 1 (TR-ALS): every update solves against the full design
                          matrix G^{!=n}_[2] and all of X_[n] (prod_{m!=n} I_m rows, at most 2^24) */
} trals_method;

/* Problem description (Algorithm 2 inputs: X, target ranks; J per update; seed). */
typedef struct {
  int32_t order;           /* N, 2 <= N <= 16 */
  const int64_t* dims;     /* host array I[0..N-1], each in [1, 2^21] */
  const int32_t* ranks;    /* host array R[0..N-1], each in [1, 32]; core n is R[n-1] x I[n] x R[n] */
  int64_t samples;         /* J in [max_n R[n-1]*R[n], 2^24] (fewer rows cannot give a full-rank
                              system); ignored by TRALS_EXACT */
  uint64_t seed;           /* Philox4x64-10 key word 0 */
  uint64_t stream_id;      /* Philox4x64-10 key word 1 (independent problems use distinct ids) */
  int32_t precision;       /* TRALS_F64, TRALS_F32, TRALS_BF16 or TRALS_BF16_CHAINS */
  const void* init_cores;  /* optional device pointer to all N cores (layout above), element type
                              init_dtype; NULL draws every entry iid N(0,1) (Section 3) from the seed */
  int32_t init_dtype;      /* TRALS_F64 or TRALS_F32 */
  int32_t method;          /* trals_method; 0 (TRALS_LEVERAGE) is the paper's proposal */
  int32_t normalize;       /* 0: the algorithms as stated.  1: after each update, core n is
                              replaced by Q and core n+1 by R G_{n+1} (mode-1 product), where
                              G_n = Q R is the QR factorisation of its (R[n-1] I[n]) x R[n]
                              unfolding with R's diagonal positive (a normalisation step, which
                              Section 2.1 allows).  TR(G) and every sampling distribution are
                              unchanged in exact arithmetic; the core scales cannot drift apart,
                              which keeps the sampled systems well conditioned on long runs.  A
                              rank-deficient core then fails with TRALS_ESINGULAR after its update. */
} trals_desc;

/* Generated data source (serving): the tensor is X = TR(G*) + sigma Z with given "true" cores
 * G* and iid N(0,1) noise Z, and is never materialised; every update computes only its J
 * sampled fibers (Algorithm 2, "sample X") from G* and the noise generator.  Z at C-order linear
 * index e is the Box-Muller transform of the Philox4x64-10 block with key (noise_seed,
 * noise_stream) and counter (e, ~0, ~0, 0): z = sqrt(-2 ln u1) cos(2 pi u2), u1 =
 * (w0 >> 11 + 1) 2^-53, u2 = (w1 >> 11) 2^-53.  sigma = noise_rel ||TR(G*)||_F / sqrt(prod I),
 * the norm taken by transfer matrices. */
typedef struct {
  const void* true_cores;   /* device: the N cores of G*, layout as trals_desc.init_cores */
  int32_t true_dtype;       /* TRALS_F64 or TRALS_F32 */
  const int32_t* true_ranks;/* host array of N ranks of G*; NULL = the decomposition's ranks */
  double noise_rel;         /* >= 0 */
  uint64_t noise_seed, noise_stream;
} trals_source;

/* Bytes of device workspace trals_create needs for this description (TRALS_EXACT holds the full
 * design matrix of the largest update: (max_n prod_{m!=n} I_m) x max_n R[n-1]R[n] entries).
 * Pure host computation.  Returns TRALS_EINVAL for an invalid description. */
int trals_workspace_bytes(const trals_desc* desc, size_t* bytes);

/* Build a handle: validates desc, copies X into per-mode data panels inside the
 * workspace (X may be freed afterwards), loads or draws the initial cores and
 * computes the sampling tables of cores 1..N-1 (Algorithm 2, first two steps).
 * X_dev: device pointer to prod(I) elements of type x_dtype (TRALS_F64 or TRALS_F32).
 * stream: a hipStream_t (NULL = default stream), borrowed for the handle's lifetime.
 * Fails with TRALS_EINVAL on NaN/Inf in X or a workspace smaller than
 * trals_workspace_bytes(desc). */
int trals_create(const trals_desc* desc, const void* X_dev, int32_t x_dtype, void* ws_dev,
                 size_t ws_bytes, void* stream, trals_handle* out);

/* As trals_workspace_bytes / trals_create, for a generated data source (no X, no panels).
 * trals_create_generated returns once its work is enqueued (it does not synchronise the
 * stream): an unusable source (||TR(G*)||_F zero or not finite) or a failed initial table is
 * reported as TRALS_ESINGULAR by the next call that synchronises or by trals_query.
 * trals_fit_error of such a handle returns ||TR(G) - TR(G*)||_F / ||TR(G*)||_F (the error
 * against the noise-free tensor, by transfer matrices).  The sizing call reads only the ranks,
 * dtype and noise level of src (true_cores may be NULL there); trals_create_generated needs
 * the device pointer. */
int trals_workspace_bytes_generated(const trals_desc* desc, const trals_source* src, size_t* bytes);
int trals_create_generated(const trals_desc* desc, const trals_source* src, void* ws_dev, size_t ws_bytes,
                           void* stream, trals_handle* out);

/* Run n_sweeps outer iterations of Algorithm 2 (each updates cores 0..N-1 in
 * order), continuing from the handle's update counter. */
int trals_sweep(trals_handle h, int32_t n_sweeps);

/* Sample count of the following updates (Section 3.2, Adaptive Sample Size: J may change between updates at no
 * cost).  Sampled methods only; samples in [max_n R[n-1]*R[n], the J given at creation] (the
 * workspace was sized for that J).  trals_samples returns the current J (-1 for NULL). */
int trals_set_samples(trals_handle h, int64_t samples);
int64_t trals_samples(trals_handle h);

/* ||TR(G)||_F of the current cores by transfer matrices (trace of prod_n sum_i G_n(:,i,:) (x)
 * G_n(:,i,:), O(sum_n I_n R^4) work, no pass over X).  Synchronises the stream. */
int trals_tr_norm(trals_handle h, double* norm);

/* Termination by the change of ||TR(G)||_F (Section 3.1, Termination Criteria): run whole sweeps until
 * |n_k - n_{k-1}| / n_k < rel_tol after sweep k, or max_sweeps sweeps.  Reports the sweeps run
 * and the last relative change (-1 if none).  Synchronises once per sweep. */
int trals_sweep_until(trals_handle h, int32_t max_sweeps, double rel_tol, int32_t* sweeps_done,
                      double* last_change);

/* Estimate of the relative error ||TR(G) - X||_F / ||X||_F from sampled entries (Section 3.1,
 * Termination Criteria: the exact error needs every entry of X).  `samples` entries are drawn
 * uniformly with replacement (entry s: word 0 r of the Philox4x64-10 block with key (seed,
 * stream_id) and counter (s, tag, 0, 1), C-order linear index floor(r E / 2^64), E = prod I), and
 * *rel_err = sqrt((E / samples) sum_s (TR(G)(i_s) - X(i_s))^2 / ||X||_F^2); E/samples times the
 * sum is an unbiased estimate of ||TR(G) - X||_F^2.  O(samples N R^3) work.  Handles with a
 * dense X only (TRALS_EINVAL for a generated source); samples in [1, 2^40].  Synchronises. */
int trals_fit_estimate(trals_handle h, int64_t samples, uint64_t tag, double* rel_err);

/* Termination by the change of the sampled error estimate (Section 3.1): run whole sweeps until
 * |e_k - e_{k-1}| / e_k < rel_tol, e_k = trals_fit_estimate(h, samples, 0) after sweep k (the same
 * sampled entries every time), or max_sweeps sweeps.  Reports the sweeps run, the last estimate
 * and the last relative change (-1 if none).  Synchronises once per sweep. */
int trals_sweep_until_estimate(trals_handle h, int32_t max_sweeps, double rel_tol, int64_t samples,
                               int32_t* sweeps_done, double* last_estimate, double* last_change);

/* Enqueue n_sweeps like trals_sweep and return without synchronising the stream (several
 * handles on different streams then overlap on the device).  flags: 0 or TRALS_ASYNC_FIT, which
 * also enqueues the relative error (trals_fit_error's value: the clean-ring fit of a generated
 * source, a full pass over X otherwise) after the sweeps.  The status word and that error are
 * copied into pinned host memory (a slot of a block the library allocates once per process)
 * before the completion event, so that trals_query never waits: it returns TRALS_PENDING while
 * the stream still runs the enqueued work, TRALS_OK once it finished, TRALS_ESINGULAR if a solve
 * failed; on TRALS_OK *fit (if fit is not NULL) receives the error when TRALS_ASYNC_FIT was given,
 * NaN otherwise.  trals_destroy waits for pending work before it returns. */
#define TRALS_ASYNC_FIT 1
int trals_sweep_async(trals_handle h, int32_t n_sweeps, int32_t flags);
int trals_query(trals_handle h, double* fit);

/* Run n_updates single core updates (inner iterations of Algorithm 2),
 * continuing from the update counter; core n = counter mod N is updated next. */
int trals_step(trals_handle h, int32_t n_updates);

/* Relative error ||TR(G) - X||_F / ||X||_F (Section 4.1) over every entry of X,
 * with FP64 accumulation.  Synchronises the stream. */
int trals_fit_error(trals_handle h, double* rel_err);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the relative error ||TR(G) - X||_F / ||X||_F of the
 * cores G against the dense tensor X, as trals_fit_error computes it for a handle, without a
 * handle or workspace.  It allocates nothing: its scratch (slice-major FP64 copies of the cores
 * and the partial sums) is a fixed array of TRALS_NOALLOC_SCRATCH_BYTES per GPU inside the
 * library, held until the process ends.
 *   order, dims, ranks: as in trals_desc (host arrays, read during the call).
 *   cores_dev: device, the N cores one after the other, core n in C order (R[n-1], I[n], R[n]),
 *     element type cores_dtype (TRALS_F64 or TRALS_F32).
 *   X_dev: device, prod(I) elements in C order, type x_dtype (TRALS_F64 or TRALS_F32).
 *   rel_err_dev: device, one double that receives the error.
 *   stream: hipStream_t the work is enqueued on (NULL = default stream); nothing is synchronised.
 * The sizes need sum_n I[n] R[n-1] R[n] + ceil(prod_{n<N-1} I[n] / 8) + 1026 doubles of scratch;
 * a larger problem returns TRALS_ERANGE before any work is enqueued.  Every call on one GPU uses
 * that GPU's one scratch array: calls that overlap on a GPU (two streams, two host threads) race
 * and must be serialised by the caller.  A non-finite entry of X gives a NaN error. */
#define TRALS_NOALLOC_SCRATCH_BYTES (16u << 20)
int trals_fit_error_noalloc(int32_t order, const int64_t* dims, const int32_t* ranks, const void* cores_dev,
                            int32_t cores_dtype, const void* X_dev, int32_t x_dtype, double* rel_err_dev,
                            void* stream);

/* Release the handle (not the workspace).  NULL is a no-op. */
int trals_destroy(trals_handle h);

/* Copy all cores out to / in from dst_dev / src_dev (layout above, element type
 * dtype = TRALS_F64 or TRALS_F32).  trals_set_cores recomputes every sampling
 * table and clears a failed state; it does not change the update counter. */
int trals_get_cores(trals_handle h, void* dst_dev, int32_t dtype);
int trals_set_cores(trals_handle h, const void* src_dev, int32_t dtype);

/* Samples of the most recent update (host arrays): idx_host[j*(N-1)+k] is the
 * index drawn in mode (n+1+k) mod N for sample j, w_host[j] the Definition 5
 * rescaling 1/sqrt(J q_j), J the current sample count.  Either pointer may be
 * NULL.  TRALS_ESTATE before the first update (or after trals_set_samples);
 * TRALS_EINVAL for TRALS_EXACT. */
int trals_get_last_samples(trals_handle h, int32_t* idx_host, double* w_host);

/* Number of core updates run so far (sweeps * N + position in the sweep). */
int64_t trals_update_counter(trals_handle h);

/* Set the update counter (used to resume a run from saved cores); the next
 * update is core counter mod N and draws from that counter's Philox stream. */
int trals_set_update_counter(trals_handle h, int64_t counter);

/* Kernel timing with HIP events, recorded on the handle's stream around each
 * launch of the kernel groups below (for measurement; off by default).
 * trals_profile_read synchronises the stream and returns the summed duration
 * and launch count of one group since profiling was enabled, then keeps
 * accumulating. */
typedef enum {
  TRALS_K_DRAW = 0,      /* Algorithm 3 sampler fused with the Algorithm 4 sketched rows */
  TRALS_K_CONTRACT = 1,  /* fused fiber gather + [A^T A | A^T X~] partials (matrix cores) */
  TRALS_K_REDUCE = 2,    /* fixed-order reduction of the split-K partials of H and B */
  TRALS_K_FACTOR = 3,    /* Cholesky factor of H and its inverse */
  TRALS_K_SOLVE = 4,     /* solve rows: the new core */
  TRALS_K_TABLE = 5,     /* a core's leverage table (eq. (3)): Gram, factor, leverage rows, scan */
  TRALS_K_COUNT = 6
} trals_kernel;
int trals_profile(trals_handle h, int32_t enable);
int trals_profile_read(trals_handle h, int32_t kernel, double* total_ms, int64_t* launches);

/* Static description of a status code. */
const char* trals_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* TRALS_H */
