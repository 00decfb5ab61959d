// Host runtime behind the C ABI declared in include/trals.h: argument validation, workspace
// carving, and the per-update launch sequence of Algorithm 2:
//   draw (sample + sketch) -> normal equations -> fixed-order reduction -> Cholesky and
//   inverse factor of H -> solve rows (new core) -> new core's table (Gram, Cholesky and
//   inverse factor, leverage rows + scan).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/trals.h"
#include "kernels.h"

using namespace trals;

namespace {

constexpr size_t kAlign = 256;
// FP32 path contraction: FP32 operands widened on the FP64 matrix cores, or (when some update
// has more than kThreeSliceMinP unknowns) three 8-bit slices on the BF16 matrix cores (exact
// slice products, FP64 block sums), which keeps two waves per SIMD only up to 80-row tiles
// and so wins where the FP64 kernel would need several row tiles anyway
constexpr int kThreeSliceMinP = 128;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t panel[kMaxOrder];
  size_t core[kMaxOrder];
  size_t cdf[kMaxOrder];
  size_t fitx;
  // generated source: true cores (FP64 slice-major), their subchain rows, the sampled fibers,
  // and the transfer-matrix work area
  size_t tcore[kMaxOrder];
  size_t Tm, Xg, inner, inner_res;
  size_t idx, w, A, S3, E3, D3, ED3, Hpart, Bpart, Bred, M, M2, F, F2, gauge, qr, qalt, ysol, partial, scal, total;
  int64_t partial_count;
};

struct Problem {
  int N;
  int64_t dims[kMaxOrder];
  int32_t ranks[kMaxOrder];
  int64_t J;     // samples per update (sampled methods); rows of the largest design (exact)
  int64_t Jcap;  // J at creation: the workspace holds up to this many samples
  int method;    // TRALS_LEVERAGE, TRALS_UNIFORM or TRALS_EXACT
  bool normalize;  // orthonormalise each updated core along its bond to the next core
  uint64_t seed, stream_id;
  int prec;
  int sk_dt, panel_dt, ne_dt;  // cores are FP64 in every precision
  bool bf16_chains;            // BF16 form: subchain products on BF16 matrix cores
  size_t sk_sz, panel_sz;
  int64_t E;     // prod dims
  int Pmax;
  int64_t Imax;
  // the tables of the N-1 modes one update draws from fit in the draw kernel's LDS for every
  // n: device tables then hold the weights Q, summed in LDS by each draw; otherwise the
  // inclusive sums C, scanned on the device after every table computation
  bool tables_as_weights;
  // generated source (X = TR(G*) + sigma Z, sampled fibers computed per update)
  bool generated;
  int32_t tranks[kMaxOrder];
  int Ptmax;
  double noise_rel;
  uint64_t noise_seed, noise_stream;
};

Ring ring_of(const Problem& p, const int32_t* ranks) {
  Ring g;
  memset(&g, 0, sizeof(g));
  g.N = p.N;
  for (int n = 0; n < p.N; ++n) {
    g.dims[n] = (int)p.dims[n];
    g.ranks[n] = ranks[n];
  }
  return g;
}

int P_of(const Problem& p, int n) { return p.ranks[(n + p.N - 1) % p.N] * p.ranks[n]; }

// rows of update n's least-squares problem: J samples, or every index tuple of the other modes
int64_t J_of(const Problem& p, int n) { return p.method == TRALS_EXACT ? p.E / p.dims[n] : p.J; }

int validate(const trals_desc* d, Problem* p, const trals_source* src = nullptr) {
  if (!d || !d->dims || !d->ranks) return TRALS_EINVAL;
  if (d->order < 2 || d->order > kMaxOrder) return TRALS_EINVAL;
  if (d->precision != TRALS_F64 && d->precision != TRALS_F32 && d->precision != TRALS_BF16 &&
      d->precision != TRALS_BF16_CHAINS)
    return TRALS_EINVAL;
  memset(p, 0, sizeof(*p));
  p->N = d->order;
  p->E = 1;
  for (int n = 0; n < p->N; ++n) {
    if (d->dims[n] < 1 || d->dims[n] > (int64_t)1 << 21) return TRALS_EINVAL;  // grid-y limit of the contraction
    if (d->ranks[n] < 1 || d->ranks[n] > kMaxRank) return TRALS_EINVAL;
    p->dims[n] = d->dims[n];
    p->ranks[n] = d->ranks[n];
    // a materialised tensor is limited to 2^40 entries; a generated one to int64 linear indices
    if (p->E > ((int64_t)1 << (src ? 62 : 40)) / d->dims[n]) return TRALS_EINVAL;
    p->E *= d->dims[n];
  }
  p->method = d->method;
  if (d->normalize != 0 && d->normalize != 1) return TRALS_EINVAL;
  p->normalize = d->normalize == 1;
  if (p->method != TRALS_LEVERAGE && p->method != TRALS_UNIFORM && p->method != TRALS_EXACT) return TRALS_EINVAL;
  p->Pmax = 0;
  p->Imax = 0;
  for (int n = 0; n < p->N; ++n) {
    p->Pmax = P_of(*p, n) > p->Pmax ? P_of(*p, n) : p->Pmax;
    p->Imax = p->dims[n] > p->Imax ? p->dims[n] : p->Imax;
  }
  if (p->method == TRALS_EXACT) {
    // Algorithm 1: the full design matrix of update n has prod_{m != n} I_m rows
    if (src) return TRALS_EINVAL;  // needs the data panels
    p->J = 0;
    for (int n = 0; n < p->N; ++n) {
      const int64_t rows = p->E / p->dims[n];
      if (rows < P_of(*p, n) || rows > ((int64_t)1 << 24)) return TRALS_EINVAL;
      p->J = rows > p->J ? rows : p->J;
    }
  } else {
    p->J = d->samples;
    // grid-z limit of the split-K partials; fewer than Pmax rows cannot give a full-rank system
    if (p->J < p->Pmax || p->J > ((int64_t)1 << 24)) return TRALS_EINVAL;
  }
  p->Jcap = p->J;
  {
    int64_t tot = 0, mn = p->dims[0];
    for (int n = 0; n < p->N; ++n) {
      tot += p->dims[n];
      mn = p->dims[n] < mn ? p->dims[n] : mn;
    }
    p->tables_as_weights = (tot - mn) * 8 <= (int64_t)kDrawTableBytes;
  }
  p->seed = d->seed;
  p->stream_id = d->stream_id;
  p->bf16_chains = d->precision == TRALS_BF16_CHAINS;
  p->prec = p->bf16_chains ? TRALS_BF16 : d->precision;
  // storage of the sketch (FP64 or FP32) and of the data panels (FP64, FP32 or BF16), and the
  // arithmetic of the normal-equation products; the cores (tiny) are FP64 throughout
  // sketch: FP64 rows, FP32 rows, or (BF16 form) two transposed BF16 copies of the same size as
  // the FP32 rows
  p->sk_dt = p->prec == TRALS_F64 ? 0 : p->prec == TRALS_F32 ? 1 : 2;
  p->sk_sz = p->sk_dt == 0 ? 8 : 4;
  p->panel_dt = p->prec == TRALS_F64 ? 0 : p->prec == TRALS_F32 ? 1 : 2;
  p->panel_sz = p->panel_dt == 0 ? 8 : p->panel_dt == 1 ? 4 : 2;
  // FP32: FP32 sketch and fibers widened exactly on the FP64 matrix cores (ne_dt 1), or the
  // three-slice form on the BF16 matrix cores (ne_dt 3) for large P (Pmax is set below)
  p->ne_dt = p->panel_dt;
  if (p->prec == TRALS_F32 && p->Pmax > kThreeSliceMinP) p->ne_dt = 3;
  if (d->init_cores && d->init_dtype != TRALS_F64 && d->init_dtype != TRALS_F32) return TRALS_EINVAL;
  if (src) {
    if (src->true_dtype != TRALS_F64 && src->true_dtype != TRALS_F32) return TRALS_EINVAL;
    if (!(src->noise_rel >= 0.0) || !isfinite(src->noise_rel)) return TRALS_EINVAL;
    p->generated = true;
    p->Ptmax = 0;
    for (int n = 0; n < p->N; ++n) {
      const int32_t r = src->true_ranks ? src->true_ranks[n] : d->ranks[n];
      if (r < 1 || r > kMaxRank) return TRALS_EINVAL;
      p->tranks[n] = r;
    }
    for (int n = 0; n < p->N; ++n) {
      const int Pt = p->tranks[(n + p->N - 1) % p->N] * p->tranks[n];
      p->Ptmax = Pt > p->Ptmax ? Pt : p->Ptmax;
    }
    p->noise_rel = src->noise_rel;
    p->noise_seed = src->noise_seed;
    p->noise_stream = src->noise_stream;
  }
  return TRALS_OK;
}


void plan(const Problem& p, Layout* L) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  if (!p.generated) {
    for (int n = 0; n < p.N; ++n) L->panel[n] = take((size_t)p.E * p.panel_sz);
    // the fit error reads X in C order: the last panel, or an FP32 copy in the BF16 form
    L->fitx = p.panel_dt == 2 ? take((size_t)p.E * 4) : L->panel[p.N - 1];
  } else {
    for (int n = 0; n < p.N; ++n) {
      const int Pt = p.tranks[(n + p.N - 1) % p.N] * p.tranks[n];
      L->tcore[n] = take((size_t)p.dims[n] * Pt * 8);
    }
    L->Tm = take((size_t)p.J * p.Ptmax * 8);
    L->Xg = take((size_t)p.J * p.Imax * p.panel_sz);
  }
  {
    // transfer-matrix inner products: <G, G> (norm of the ring), and <G, G*>, <G*, G*> for a
    // generated source
    const Ring rr = ring_of(p, p.ranks);
    size_t w = ring_inner_doubles(rr, rr);
    if (p.generated) {
      const Ring rt = ring_of(p, p.tranks);
      w = ring_inner_doubles(rr, rt) > w ? ring_inner_doubles(rr, rt) : w;
      w = ring_inner_doubles(rt, rt) > w ? ring_inner_doubles(rt, rt) : w;
    }
    // work area, then the result doubles: [0] <G,G>, [1] <G,G*>, [2] <G*,G*>, [3] sigma, [4] fit
    L->inner = take((w + 8) * 8);
    L->inner_res = L->inner + w * 8;
  }
  for (int n = 0; n < p.N; ++n) L->core[n] = take((size_t)p.dims[n] * P_of(p, n) * 8);
  for (int n = 0; n < p.N; ++n) L->cdf[n] = take((size_t)p.dims[n] * 8);
  size_t hpart = 0, bpart = 0;
  for (int n = 0; n < p.N; ++n) {
    const int P = P_of(p, n);
    const NormalEqPlan pl = plan_normal_eq(P, (int)p.dims[n], J_of(p, n), p.ne_dt, kPlanCUs);
    const size_t h = (size_t)pl.splits * P * P, b = (size_t)pl.splits * P * p.dims[n];
    hpart = h > hpart ? h : hpart;
    bpart = b > bpart ? b : bpart;
  }
  L->idx = take((size_t)p.J * (p.N - 1) * 4);
  L->w = take((size_t)p.J * 8);
  L->A = take((size_t)(p.J + kSketchPadRows) * p.Pmax * p.sk_sz);
  {
    // three-slice sketch (BF16) and its block exponents
    const size_t ld = (size_t)(p.J + kSplitBlock - 1) / kSplitBlock * kSplitBlock;
    // (the BF16 form: its two transposed sketches, rounded from the draw's FP32 rows)
    L->S3 = take((p.ne_dt == 3 ? 3 : p.ne_dt == 2 && !p.bf16_chains ? 2 : 0) * (size_t)p.Pmax * ld * 2);
    L->E3 = take(p.ne_dt == 3 ? (size_t)p.Pmax * (ld / kSplitBlock) * 4 : 0);
    // the weighted fibers in the same form (the contraction's column operand); for the BF16
    // form the gathered raw BF16 fibers, one slice
    L->D3 = take((p.ne_dt == 3 ? 3 : p.ne_dt == 2 ? 1 : 0) * (size_t)p.Imax * ld * 2);
    L->ED3 = take(p.ne_dt == 3 ? (size_t)p.Imax * (ld / kSplitBlock) * 4 : 0);
  }
  L->Hpart = take(hpart * 8);  // FP64 split-K partials
  L->Bpart = take(bpart * 8);
  L->Bred = take((size_t)p.Pmax * p.Imax * 8);
  L->M = take((size_t)p.Pmax * p.Pmax * 8);   // H
  L->M2 = take((size_t)p.Pmax * p.Pmax * 8);  // Gram of a core for its leverage
  L->F = take(chol_work_doubles(p.Pmax) * 8);
  L->F2 = take(chol_work_doubles(p.Pmax) * 8);
  L->gauge = take(gauge_work_doubles() * 8);
  {
    // pivoted-QR work copy of the largest core unfolding (rank-revealing table path)
    size_t qr = 0;
    if (p.method == TRALS_LEVERAGE)
      for (int n = 0; n < p.N; ++n) {
        const size_t c = (size_t)p.dims[n] * P_of(p, n);
        qr = c > qr ? c : qr;
      }
    L->qr = take(qr * 8);
  }
  // a table formed beside the next update (taken if its factorisation breaks down)
  L->qalt = take(p.method == TRALS_LEVERAGE ? (size_t)p.Imax * 8 : 0);
  // the first half of a solve spread over several workgroups per row group (P > 128)
  L->ysol = take(p.Pmax > 128 ? solve_split_doubles((int)p.Imax, p.Pmax) * 8 : 0);
  const int64_t fit_rows = p.generated ? 0 : p.E / p.dims[p.N - 1];
  const int64_t fit_blocks = (fit_rows + kFitRows - 1) / kFitRows;
  L->partial_count = fit_blocks > kScanBlocks ? fit_blocks : kScanBlocks;
  L->partial = take((size_t)L->partial_count * 8);
  L->scal = take(64);  // [0] double result, [8] u64 nonfinite, [16] int status, [20] int table
                       // breakdown, [24] int completion counter of the solve, [28] int guard
                       // word of the repeated draws after a table breakdown
  L->total = off;
}

}  // namespace

struct Prof {
  bool on = false;
  std::vector<hipEvent_t> ev[TRALS_K_COUNT];
  size_t used[TRALS_K_COUNT] = {};
  double ms[TRALS_K_COUNT] = {};
  int64_t count[TRALS_K_COUNT] = {};
};

struct trals_ctx {
  Prof prof;
  Problem p;
  Layout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  int64_t upd = 0;
  bool failed = false;
  bool table_valid[kMaxOrder] = {};
  bool have_last = false;
  hipEvent_t done = nullptr;  // end of the last asynchronous sweep
  bool pending = false;
  struct HostResult {         // pinned host copy of the status word and fit, written by the stream
    int status;
    int fit_valid;
    double fit;
  };
  HostResult* host_res = nullptr;
  bool async_fit = false;
  double xnorm2 = 0.0;   // ||X||_F^2, or ||TR(G*)||_F^2 for a generated source
  hipError_t last_hip = hipSuccess;
  // a wide core's table checked beside the next update (table_ahead): the second stream, its
  // fork and join events, and the mode whose check is outstanding (-1: none)
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int ahead_mode = -1;

  template <typename T>
  T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
  int* status() { return reinterpret_cast<int*>(ws + L.scal + 16); }
  int* table_fail() { return reinterpret_cast<int*>(ws + L.scal + 20); }
  int* solve_counter() { return reinterpret_cast<int*>(ws + L.scal + 24); }
  int* redo_word() { return reinterpret_cast<int*>(ws + L.scal + 28); }
  double* scal_d() { return reinterpret_cast<double*>(ws + L.scal); }
  unsigned long long* nonfinite() { return reinterpret_cast<unsigned long long*>(ws + L.scal + 8); }
};

#define HIPTRY(expr)                      \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) {               \
      h->last_hip = e_;                   \
      return TRALS_EHIP;                  \
    }                                     \
  } while (0)

namespace {

hipError_t prof_mark(trals_ctx* h, int k, int which, hipStream_t s = nullptr) {
  if (!h->prof.on) return hipSuccess;
  Prof& pr = h->prof;
  const size_t slot = 2 * pr.used[k] + which;
  while (pr.ev[k].size() <= slot) {
    hipEvent_t e;
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    pr.ev[k].push_back(e);
  }
  const hipError_t r = hipEventRecord(pr.ev[k][slot], s ? s : h->stream);
  if (which == 1) pr.used[k] += 1;
  return r;
}

// an event pair of group k for a launch that stamps them itself (kernel start / end)
hipError_t prof_pair(trals_ctx* h, int k, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (!h->prof.on) return hipSuccess;
  Prof& pr = h->prof;
  const size_t slot = 2 * pr.used[k];
  while (pr.ev[k].size() <= slot + 1) {
    hipEvent_t e;
    const hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    pr.ev[k].push_back(e);
  }
  *e0 = pr.ev[k][slot];
  *e1 = pr.ev[k][slot + 1];
  pr.used[k] += 1;
  return hipSuccess;
}

#define PROF_BEGIN(k) HIPTRY(prof_mark(h, (k), 0))
#define PROF_END(k) HIPTRY(prof_mark(h, (k), 1))

Ring make_ring(const Problem& p) { return ring_of(p, p.ranks); }

LevWideArgs wide_table_args(trals_ctx* h, int m, const double* G) {
  LevWideArgs la;
  memset(&la, 0, sizeof(la));
  la.G = G;
  la.I = (int)h->p.dims[m];
  la.P = P_of(h->p, m);
  la.K = h->at<double>(h->L.M2);
  la.F = h->at<double>(h->L.F2);
  la.qr_work = h->at<double>(h->L.qr);
  la.Q = h->at<uint64_t>(h->L.cdf[m]);
  la.status = h->status();
  la.fail = h->table_fail();
  la.rel_tol = kTableRelTol;
  return la;
}

// Sampling table of mode m (eq. (3), Definition 4) from the rows of G (I_m x P, row i the
// lateral slice i: the core unfolding G_(2), or a matrix with the same column space), launched
// on stream s and scanned in place when the draws take inclusive sums.  The numerical rank
// decides the reading:
//  * tall (I > P): the column Gram K = G^T G factored with the table tolerance; if it factors,
//    G has full column rank and l_i = ||W g_i||^2 (W = L^{-1}); otherwise the leverage rows'
//    launch takes the table from the pivoted QR of G (rank-revealing);
//  * wide (I <= P): the row Gram G G^T factored likewise; if it factors, G has full row rank
//    and p_i = 1/I exactly; otherwise the pivoted-QR table.
int table_launches(trals_ctx* h, int m, const double* G, hipStream_t s) {
  const Problem& p = h->p;
  const int P = P_of(p, m);
  const int I = (int)p.dims[m];
  uint64_t* Q = h->at<uint64_t>(h->L.cdf[m]);
  HIPTRY(prof_mark(h, TRALS_K_TABLE, 0, s));
  double* M2 = h->at<double>(h->L.M2);
  double* F2 = h->at<double>(h->L.F2);
  if (p.method == TRALS_LEVERAGE && I > P) {
    // a blocked factorisation (P > 144, a multiple of 16) takes the Gram block-packed
    const bool prepack = chol_prepack_ok(P);
    HIPTRY(launch_syrk(G, I, P, prepack ? chol_packed_input(F2, P) : M2, h->status(), s, /*trans=*/false,
                       h->table_fail(), prepack));
    CholArgs ca;
    memset(&ca, 0, sizeof(ca));
    ca.P = P;
    ca.H = M2;
    ca.W = F2;
    ca.prepacked = prepack ? 1 : 0;
    ca.status = h->status();
    ca.fail = h->table_fail();
    ca.rel_tol = kTableRelTol;
    HIPTRY(launch_chol(ca, s));
    TriArgs ta;
    memset(&ta, 0, sizeof(ta));
    ta.P = P;
    ta.In_lev = I;
    ta.Wlev = F2;
    ta.Blev = G;
    ta.Q = Q;
    ta.status = h->status();
    ta.lev_fail = h->table_fail();
    ta.qr_work = h->at<double>(h->L.qr);
    HIPTRY(launch_trisolve(ta, s));
  } else if (p.method == TRALS_LEVERAGE) {
    HIPTRY(launch_lev_wide(wide_table_args(h, m, G), s));
  } else {
    HIPTRY(launch_lev_uniform(I, Q, h->status(), s));
  }
  if (!p.tables_as_weights) HIPTRY(launch_scan_u64(Q, I, h->status(), s));
  HIPTRY(prof_mark(h, TRALS_K_TABLE, 1, s));
  h->table_valid[m] = true;
  return TRALS_OK;
}

// table of core m from the core itself (initial cores, or after the sample count changed)
int compute_table(trals_ctx* h, int m) {
  if (h->p.method == TRALS_EXACT) {  // no sampling
    h->table_valid[m] = true;
    return TRALS_OK;
  }
  return table_launches(h, m, h->at<const double>(h->L.core[m]), h->stream);
}

// The table of a wide core (I <= P) with more rows than one workgroup factors.  Its numerical
// rank takes a blocked factorisation of the row Gram (several launches, a few workgroups each),
// but the table is exactly uniform whenever that factors.  The uniform table is written at once
// on the handle's stream, where the next update draws from it, and the factorisation (with the
// pivoted-QR table into qalt) runs on a second stream beside the next update's draws and
// contraction.  The next update joins it before its own factorisation: after a breakdown the
// QR table replaces the uniform one and the draws and contraction are repeated (launches
// guarded by a device word), so every result is that of the serial order.
bool table_ahead_applies(const trals_ctx* h, int m) {
  const Problem& p = h->p;
  const int I = (int)p.dims[m];
  return p.method == TRALS_LEVERAGE && !p.generated && I <= P_of(p, m) && !chol_single_workgroup(I);
}

// the handle's second stream (default priority) and its fork / join events, made on first use
hipError_t aux_stream(trals_ctx* h) {
  if (h->aux) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming);
  return e;
}

int table_ahead(trals_ctx* h, int m) {
  const Problem& p = h->p;
  const int I = (int)p.dims[m];
  HIPTRY(aux_stream(h));
  uint64_t* Q = h->at<uint64_t>(h->L.cdf[m]);
  uint64_t* Qalt = h->at<uint64_t>(h->L.qalt);
  HIPTRY(hipEventRecord(h->ev_fork, h->stream));
  HIPTRY(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
  LevWideArgs la = wide_table_args(h, m, h->at<const double>(h->L.core[m]));
  la.Q = Qalt;
  HIPTRY(launch_lev_wide(la, h->aux));
  if (!p.tables_as_weights) HIPTRY(launch_scan_u64(Qalt, I, h->status(), h->aux));
  HIPTRY(hipEventRecord(h->ev_join, h->aux));
  HIPTRY(prof_mark(h, TRALS_K_TABLE, 0));
  HIPTRY(launch_lev_uniform(I, Q, h->status(), h->stream));
  if (!p.tables_as_weights) HIPTRY(launch_scan_u64(Q, I, h->status(), h->stream));
  HIPTRY(prof_mark(h, TRALS_K_TABLE, 1));
  h->table_valid[m] = true;
  h->ahead_mode = m;
  return TRALS_OK;
}

// join an outstanding table check into the handle's stream; the guard word then says whether
// the launches it guards repeat their work
int table_settle(trals_ctx* h) {
  if (h->ahead_mode < 0) return TRALS_OK;
  const int m = h->ahead_mode;
  h->ahead_mode = -1;
  HIPTRY(hipStreamWaitEvent(h->stream, h->ev_join, 0));
  HIPTRY(launch_table_settle(h->table_fail(), h->status(), h->at<const uint64_t>(h->L.qalt),
                             h->at<uint64_t>(h->L.cdf[m]), (int)h->p.dims[m], h->redo_word(), h->stream));
  return TRALS_OK;
}

int run_update(trals_ctx* h) {
  const Problem& p = h->p;
  const int N = p.N;
  const int n = (int)(h->upd % N);
  for (int m = 0; m < N; ++m)
    if (m != n && !h->table_valid[m]) {
      const int rc = compute_table(h, m);
      if (rc) return rc;
    }
  const int P = P_of(p, n);
  const int In = (int)p.dims[n];
  const int64_t Jn = J_of(p, n);
  const bool exact = p.method == TRALS_EXACT;
  // panel rows are the other modes in C order: stride of mode m = prod_{m' > m, m' != n} I_m'
  int64_t pstride[kMaxOrder];
  for (int k = 0; k < N - 1; ++k) {
    const int m = (n + 1 + k) % N;
    int64_t st = 1;
    for (int m2 = m + 1; m2 < N; ++m2)
      if (m2 != n) st *= p.dims[m2];
    pstride[k] = st;
  }

  DrawArgs da;
  memset(&da, 0, sizeof(da));
  da.ring = make_ring(p);
  da.n = n;
  da.J = Jn;
  da.seed = p.seed;
  da.stream_id = p.stream_id;
  da.u = (uint64_t)h->upd;
  for (int m = 0; m < N; ++m) {
    da.cdf.p[m] = h->at<const uint64_t>(h->L.cdf[m]);
    da.cores.p[m] = h->at<const double>(h->L.core[m]);
  }
  da.idx = h->at<int32_t>(h->L.idx);
  da.w = h->at<double>(h->L.w);
  da.A = h->at<void>(h->L.A);
  // the BF16 form's draw writes FP32 rows (rounded and transposed by the gather pass); with the
  // chain products on BF16 matrix cores it writes the two transposed BF16 sketches itself
  const bool rows32 = p.sk_dt == 2 && !p.bf16_chains;
  const int draw_dt = rows32 ? 1 : p.sk_dt;
  if (p.sk_dt == 2 && !rows32) {
    da.ldt = (Jn + 63) / 64 * 64;
    da.A2 = h->at<char>(h->L.A) + (size_t)P * da.ldt * 2;
  }
  da.status = h->status();
  da.mfma_chain = p.bf16_chains ? 1 : 0;
  da.weights = p.tables_as_weights ? 1 : 0;
  da.draw = exact ? 0 : 1;
  da.enumerate = exact ? 1 : 0;
  for (int k = 0; k < N - 1; ++k) da.en_stride[k] = pstride[k];
  PROF_BEGIN(TRALS_K_DRAW);
  HIPTRY(launch_draw(da, draw_dt, h->stream));
  if (p.generated) {
    // the sampled fibers of X = TR(G*) + sigma Z: true-core subchain rows for the same
    // indices, then the fibers themselves
    DrawArgs dt = da;
    dt.ring = ring_of(p, p.tranks);
    for (int m = 0; m < N; ++m) dt.cores.p[m] = h->at<const double>(h->L.tcore[m]);
    dt.draw = 0;
    dt.A = h->at<void>(h->L.Tm);
    HIPTRY(launch_draw(dt, 0, h->stream));
    FiberArgs fa;
    memset(&fa, 0, sizeof(fa));
    fa.J = p.J;
    fa.P = p.tranks[(n + N - 1) % N] * p.tranks[n];
    fa.In = In;
    fa.K = N - 1;
    fa.T = h->at<const double>(h->L.Tm);
    fa.idx = da.idx;
    auto cstride = [&](int m) {
      int64_t st = 1;
      for (int m2 = m + 1; m2 < N; ++m2) st *= p.dims[m2];
      return st;
    };
    for (int k = 0; k < N - 1; ++k) fa.lin_stride[k] = cstride((n + 1 + k) % N);
    fa.lin_stride_n = cstride(n);
    fa.true_core = h->at<const double>(h->L.tcore[n]);
    fa.sigma = h->at<const double>(h->L.inner_res) + 3;
    fa.noise_seed = p.noise_seed;
    fa.noise_stream = p.noise_stream;
    fa.out = h->at<void>(h->L.Xg);
    fa.status = h->status();
    HIPTRY(launch_fibers(fa, p.panel_dt, h->stream));
  }
  PROF_END(TRALS_K_DRAW);

  const NormalEqPlan pl = plan_normal_eq(P, In, Jn, p.ne_dt, kPlanCUs);
  NormalEqArgs na;
  memset(&na, 0, sizeof(na));
  na.A = da.A;
  na.A2 = da.A2;
  na.ld = da.ldt;
  if (p.ne_dt == 3) {
    na.S3 = h->at<__bf16>(h->L.S3);
    na.E = h->at<int>(h->L.E3);
    na.ld = (Jn + kSplitBlock - 1) / kSplitBlock * kSplitBlock;
    na.D3 = h->at<void>(h->L.D3);
    na.ED = h->at<int>(h->L.ED3);
  }
  if (p.ne_dt == 2) {
    na.D3 = h->at<void>(h->L.D3);
    na.ld = (Jn + 63) / 64 * 64;
    if (rows32) {
      na.S3 = h->at<__bf16>(h->L.S3);
      na.x1_rows = 1;
    }
  }
  na.panel = p.generated ? h->at<const void>(h->L.Xg) : h->at<const void>(h->L.panel[n]);
  // generated fibers are stored in sample order, and the enumerated rows of Algorithm 1 are the
  // panel's rows: row r of the sketch pairs with fiber row r
  na.direct = (p.generated || exact) ? 1 : 0;
  na.idx = da.idx;
  na.w = da.w;
  for (int k = 0; k < N - 1; ++k) na.stride[k] = pstride[k];
  na.K = N - 1;
  na.J = Jn;
  na.chunk = pl.chunk;
  na.P = P;
  na.In = In;
  na.gram_tiles = pl.gram_tiles;
  na.Hpart = h->at<double>(h->L.Hpart);
  na.Bpart = h->at<double>(h->L.Bpart);
  na.status = h->status();
  {
    // the contraction is timed by its own start/end stamps (an event record between two
    // kernels would add idle time to the span)
    hipEvent_t e0, e1;
    HIPTRY(prof_pair(h, TRALS_K_CONTRACT, &e0, &e1));
    HIPTRY(launch_normal_eq(na, pl, p.ne_dt, h->stream, e0, e1));
  }

  double* M = h->at<double>(h->L.M);
  double* F = h->at<double>(h->L.F);
  double* Bred = h->at<double>(h->L.Bred);  // I_n x P: row i = b_i
  // large P (a multiple of 16): H is reduced straight into the blocked factorisation's packed
  // work matrix, which then needs no packing launch
  const bool prepack = chol_prepack_ok(P);
  const int64_t packed = (int64_t)((P + 15) / 16) * ((P + 15) / 16 + 1) / 2 * kPackBlk;
  const ReduceJob jobH = prepack ? ReduceJob{na.Hpart, packed, 3, chol_packed_input(F, P)}
                                 : ReduceJob{na.Hpart, (int64_t)P * P, 1, M};
  const ReduceJob jobB{na.Bpart, (int64_t)P * In, 2, Bred};
  // eq. (3): the new core's leverage table.  Its unfolding is G_(2) = B^T H^{-1} (rows z_i =
  // H^{-1} b_i) with H nonsingular, so G_(2) and B^T have the same column space, hence the same
  // rank and the same leverage scores (Definition 4).  When both factorisations fit one
  // workgroup each, the table is taken from B^T beside the factorisation of H (same launches)
  // instead of after the solve.  B = H G_(2)^T carries the conditioning of H: if the Gram of
  // B^T does not factor within the table tolerance, the table is instead taken from the pivoted
  // QR of the new core once it is solved (by the solve's last workgroup).  Larger
  // problems take the table from the new core after the solve.
  const bool pair = p.method == TRALS_LEVERAGE && chol_single_workgroup(P);
  const bool wide = In <= P;
  // without a table beside it, a single-workgroup factorisation reduces B with extra workgroups
  const bool b_beside = !pair && chol_single_workgroup(P);
  CholArgs ca;
  memset(&ca, 0, sizeof(ca));
  ca.P = P;
  ca.H = M;
  ca.W = F;
  ca.prepacked = prepack ? 1 : 0;
  ca.status = h->status();
  TriArgs ta;
  memset(&ta, 0, sizeof(ta));
  ta.P = P;
  ta.In_sol = In;
  ta.Wsol = F;
  ta.Bsol = Bred;
  ta.core = h->at<double>(h->L.core[n]);
  ta.status = h->status();
  if (P > 128) ta.split_work = h->at<double>(h->L.ysol);
  uint64_t* Qn = h->at<uint64_t>(h->L.cdf[n]);
  PROF_BEGIN(TRALS_K_REDUCE);
  HIPTRY(launch_reduce_parts(jobH, b_beside ? ReduceJob{nullptr, 0, 2, nullptr} : jobB, pl.splits, P, h->status(),
                             h->stream));
  PROF_END(TRALS_K_REDUCE);
  if (h->ahead_mode >= 0) {
    // the previous core's table was checked beside these draws (table_ahead): join it, then
    // repeat the draws, the contraction and its reduction, launches that skip unless that
    // check broke down and replaced the uniform table they drew from
    const int rc = table_settle(h);
    if (rc) return rc;
    int* g = h->redo_word();
    DrawArgs dr = da;
    dr.status = g;
    HIPTRY(launch_draw(dr, draw_dt, h->stream));
    NormalEqArgs nr = na;
    nr.status = g;
    HIPTRY(launch_normal_eq(nr, pl, p.ne_dt, h->stream, nullptr, nullptr));
    HIPTRY(launch_reduce_parts(jobH, b_beside ? ReduceJob{nullptr, 0, 2, nullptr} : jobB, pl.splits, P, g, h->stream));
  }
  // a wide core of at most 144 rows whose update factors H in blocks (P > 144): its row rank
  // (full: the uniform table) from the rows b_i of B^T (the same rank), checked on the second
  // stream beside the factorisation of H; a breakdown leaves the table to the new core after
  // the solve
  const bool wide_beside = p.method == TRALS_LEVERAGE && !p.generated && !pair && In <= P &&
                           chol_single_workgroup(In) && !chol_single_workgroup(P);
  if (wide_beside) {
    HIPTRY(aux_stream(h));
    HIPTRY(hipEventRecord(h->ev_fork, h->stream));
    HIPTRY(hipStreamWaitEvent(h->aux, h->ev_fork, 0));
    LevWideArgs lb = wide_table_args(h, n, Bred);
    lb.qr_work = nullptr;  // the breakdown word only
    HIPTRY(launch_lev_wide(lb, h->aux));
    HIPTRY(hipEventRecord(h->ev_join, h->aux));
  }
  if (pair) {
    CholArgs ck;
    memset(&ck, 0, sizeof(ck));
    LevWideArgs lw = wide_table_args(h, n, Bred);
    lw.qr_work = nullptr;  // a breakdown is left to the QR of the new core below
    if (!wide) {
      // K = B B^T, factored beside H with the table tolerance; the leverage rows of B^T then
      // run in the solve's launch
      PROF_BEGIN(TRALS_K_TABLE);
      HIPTRY(launch_syrk(Bred, In, P, h->at<double>(h->L.M2), h->status(), h->stream, /*trans=*/false,
                         h->table_fail()));
      PROF_END(TRALS_K_TABLE);
      ck.P = P;
      ck.H = h->at<double>(h->L.M2);
      ck.W = h->at<double>(h->L.F2);
      ck.status = h->status();
      ck.fail = h->table_fail();
      ck.rel_tol = kTableRelTol;
      ta.In_lev = In;
      ta.Wlev = ck.W;
      ta.Blev = Bred;
      ta.Q = Qn;
      ta.lev_fail = h->table_fail();
    }
    // the table from the pivoted QR of the new core, if that Gram breaks down: by the solve's
    // last workgroup
    ta.Q = Qn;
    ta.last_counter = h->solve_counter();
    ta.core_fail = h->table_fail();
    ta.fallback_work = h->at<double>(h->L.qr);
    PROF_BEGIN(TRALS_K_FACTOR);
    HIPTRY(launch_chol_pair(ca, wide ? nullptr : &ck, wide ? &lw : nullptr, h->stream, h->solve_counter()));
    PROF_END(TRALS_K_FACTOR);
  } else {
    PROF_BEGIN(TRALS_K_FACTOR);
    HIPTRY(launch_chol(ca, h->stream, b_beside ? &jobB : nullptr, pl.splits));
    PROF_END(TRALS_K_FACTOR);
  }
  PROF_BEGIN(TRALS_K_SOLVE);
  HIPTRY(launch_trisolve(ta, h->stream));
  PROF_END(TRALS_K_SOLVE);
  if (wide_beside) {
    PROF_BEGIN(TRALS_K_TABLE);
    HIPTRY(hipStreamWaitEvent(h->stream, h->ev_join, 0));
    LevWideArgs lf = wide_table_args(h, n, h->at<const double>(h->L.core[n]));
    lf.run_if = h->table_fail();  // only after a breakdown of the check from B^T
    HIPTRY(launch_lev_wide(lf, h->stream));
    if (!p.tables_as_weights) HIPTRY(launch_scan_u64(Qn, In, h->status(), h->stream));
    PROF_END(TRALS_K_TABLE);
  }
  if (pair && !p.tables_as_weights) {
    PROF_BEGIN(TRALS_K_TABLE);
    HIPTRY(launch_scan_u64(Qn, In, h->status(), h->stream));
    PROF_END(TRALS_K_TABLE);
  }
  if (p.normalize) {
    const int nx = (n + 1) % N;
    PROF_BEGIN(TRALS_K_SOLVE);
    HIPTRY(launch_gauge(h->at<double>(h->L.core[n]), In, p.ranks[(n + N - 1) % N], p.ranks[n],
                        h->at<double>(h->L.core[nx]), p.dims[nx], p.ranks[nx], h->at<double>(h->L.M2),
                        h->at<double>(h->L.gauge), h->status(), h->stream));
    PROF_END(TRALS_K_SOLVE);
  }
  if (pair || wide_beside) {
    h->table_valid[n] = true;
  } else if (table_ahead_applies(h, n)) {
    const int rc = table_ahead(h, n);  // checked beside the next update
    if (rc) return rc;
  } else {
    const int rc = compute_table(h, n);  // from the new core; uniform tables; none when exact
    if (rc) return rc;
  }
  h->upd += 1;
  h->have_last = !exact;
  return TRALS_OK;
}

// <TR(G), TR(G)> by transfer matrices into inner_res[0] (enqueued on the handle's stream)
int ring_norm_enqueue(trals_ctx* h) {
  const Problem& p = h->p;
  const Ring rr = make_ring(p);
  PerMode<const double> G;
  for (int n = 0; n < p.N; ++n) G.p[n] = h->at<const double>(h->L.core[n]);
  HIPTRY(launch_ring_inner(rr, G, rr, G, h->at<double>(h->L.inner), h->at<double>(h->L.inner_res), h->stream));
  return TRALS_OK;
}

int sync_status(trals_ctx* h) {
  int st = 0;
  HIPTRY(hipMemcpyAsync(&st, h->status(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPTRY(hipStreamSynchronize(h->stream));
  if (st != kDevOk) {
    h->failed = true;
    return TRALS_ESINGULAR;
  }
  return TRALS_OK;
}

int load_cores(trals_ctx* h, const void* src, int dtype);

// initial cores (given, or N(0,1) from the seed) and the sampling tables of cores 1..N-1
int init_cores_and_tables(trals_ctx* h, const trals_desc* desc, bool wait = true) {
  const Problem& p = h->p;
  if (desc->init_cores) {
    const int r2 = load_cores(h, desc->init_cores, desc->init_dtype);
    if (r2) return r2;
  } else {
    for (int n = 0; n < p.N; ++n) {
      const int64_t cnt = (int64_t)p.dims[n] * P_of(p, n);
      HIPTRY(launch_core_normal(h->at<void>(h->L.core[n]), 0, cnt, p.seed, p.stream_id, n, h->stream));
    }
  }
  for (int m = 1; m < p.N; ++m) {
    const int r3 = compute_table(h, m);
    if (r3) return r3;
  }
  return wait ? sync_status(h) : TRALS_OK;
}

int load_cores(trals_ctx* h, const void* src, int dtype) {
  const Problem& p = h->p;
  const size_t esz = dtype == TRALS_F64 ? 8 : 4;
  size_t off = 0;
  for (int n = 0; n < p.N; ++n) {
    const int Rp = p.ranks[(n + p.N - 1) % p.N], Rn = p.ranks[n];
    const int I = (int)p.dims[n];
    HIPTRY(launch_core_import((const char*)src + off, dtype == TRALS_F64 ? 0 : 1, h->at<void>(h->L.core[n]), 0,
                              Rp, I, Rn, h->stream));
    off += (size_t)Rp * I * Rn * esz;
  }
  return TRALS_OK;
}

// Pinned host slots for the results of asynchronous sweeps: one block allocated on first use
// and kept for the life of the process, handed out one slot per handle.
struct PinnedPool {
  std::mutex mu;
  char* base = nullptr;
  bool tried = false;
  std::vector<int> free_slots;
};
PinnedPool& pinned_pool() {
  static PinnedPool pool;
  return pool;
}
constexpr int kPinnedSlots = 4096;
constexpr size_t kPinnedSlotBytes = 64;

void* pinned_get() {
  PinnedPool& pool = pinned_pool();
  std::lock_guard<std::mutex> lock(pool.mu);
  if (!pool.tried) {
    pool.tried = true;
    void* b = nullptr;
    if (hipHostMalloc(&b, (size_t)kPinnedSlots * kPinnedSlotBytes, hipHostMallocDefault) == hipSuccess) {
      pool.base = (char*)b;
      for (int i = kPinnedSlots - 1; i >= 0; --i) pool.free_slots.push_back(i);
    }
  }
  if (pool.free_slots.empty()) return nullptr;
  const int i = pool.free_slots.back();
  pool.free_slots.pop_back();
  return pool.base + (size_t)i * kPinnedSlotBytes;
}

void pinned_put(void* ptr) {
  if (!ptr) return;
  PinnedPool& pool = pinned_pool();
  std::lock_guard<std::mutex> lock(pool.mu);
  pool.free_slots.push_back((int)(((char*)ptr - pool.base) / kPinnedSlotBytes));
}

// the clean-ring fit of a generated source into inner_res[4] (enqueued)
int enqueue_clean_fit(trals_ctx* h) {
  const Problem& p = h->p;
  const Ring rr = make_ring(p), rt = ring_of(p, p.tranks);
  PerMode<const double> G, T;
  for (int n = 0; n < p.N; ++n) {
    G.p[n] = h->at<const double>(h->L.core[n]);
    T.p[n] = h->at<const double>(h->L.tcore[n]);
  }
  double* work = h->at<double>(h->L.inner);
  double* res = h->at<double>(h->L.inner_res);
  HIPTRY(launch_ring_inner(rr, G, rr, G, work, res, h->stream));
  HIPTRY(launch_ring_inner(rr, G, rt, T, work, res + 1, h->stream));
  HIPTRY(launch_clean_fit(res, res + 4, h->stream));
  return TRALS_OK;
}

// the fit of a dense tensor (one pass over X) into inner_res[4] (enqueued)
int enqueue_dense_fit(trals_ctx* h) {
  const Problem& p = h->p;
  FitArgs fa;
  memset(&fa, 0, sizeof(fa));
  fa.ring = make_ring(p);
  for (int m = 0; m < p.N; ++m) fa.cores.p[m] = h->at<const void>(h->L.core[m]);
  fa.X = h->at<const void>(h->L.fitx);
  fa.rows = p.E / p.dims[p.N - 1];
  fa.partial = h->at<double>(h->L.partial);
  int nb = 0;
  HIPTRY(launch_fit(fa, 0, p.panel_dt == 2 ? 1 : p.panel_dt, &nb, h->stream));
  HIPTRY(launch_sum_partials(fa.partial, nb, h->scal_d(), h->stream));
  HIPTRY(launch_dense_fit(h->scal_d(), h->xnorm2, h->at<double>(h->L.inner_res) + 4, h->stream));
  return TRALS_OK;
}

}  // namespace

extern "C" {

const char* trals_strerror(int code) {
  switch (code) {
    case TRALS_OK: return "ok";
    case TRALS_EINVAL: return "invalid argument";
    case TRALS_ENOMEM: return "out of host memory";
    case TRALS_ESINGULAR: return "sampled normal equations not positive definite, or a zero core";
    case TRALS_EHIP: return "HIP runtime error";
    case TRALS_ESTATE: return "handle in a failed or incomplete state";
    case TRALS_PENDING: return "work still running";
    case TRALS_ERANGE: return "problem exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

int trals_workspace_bytes(const trals_desc* desc, size_t* bytes) {
  if (!bytes) return TRALS_EINVAL;
  Problem p;
  const int rc = validate(desc, &p);
  if (rc) return rc;
  Layout L;
  plan(p, &L);
  *bytes = L.total;
  return TRALS_OK;
}

int trals_create(const trals_desc* desc, const void* X_dev, int32_t x_dtype, void* ws_dev, size_t ws_bytes,
                 void* stream, trals_handle* out) {
  if (!out) return TRALS_EINVAL;
  *out = nullptr;
  Problem p;
  int rc = validate(desc, &p);
  if (rc) return rc;
  if (!X_dev || !ws_dev || (x_dtype != TRALS_F64 && x_dtype != TRALS_F32)) return TRALS_EINVAL;
  if (((uintptr_t)ws_dev) % kAlign) return TRALS_EINVAL;
  Layout L;
  plan(p, &L);
  if (ws_bytes < L.total) return TRALS_EINVAL;
  trals_ctx* h = new (std::nothrow) trals_ctx();
  if (!h) return TRALS_ENOMEM;
  h->p = p;
  h->L = L;
  h->ws = (char*)ws_dev;
  h->stream = (hipStream_t)stream;
  rc = [&]() -> int {
    HIPTRY(hipMemsetAsync(h->ws + L.scal, 0, 64, h->stream));
    // sketch rows are read past row J (finite values needed there)
    HIPTRY(hipMemsetAsync(h->ws + L.A, 0, (size_t)(p.J + kSketchPadRows) * p.Pmax * p.sk_sz, h->stream));
    // norm and finiteness of X
    HIPTRY(launch_scan_x(X_dev, x_dtype, p.E, h->at<double>(L.partial), kScanBlocks, h->nonfinite(), h->stream));
    HIPTRY(launch_sum_partials(h->at<double>(L.partial), kScanBlocks, h->scal_d(), h->stream));
    double x2 = 0.0;
    unsigned long long bad = 0;
    HIPTRY(hipMemcpyAsync(&x2, h->scal_d(), 8, hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipMemcpyAsync(&bad, h->nonfinite(), 8, hipMemcpyDeviceToHost, h->stream));
    HIPTRY(hipStreamSynchronize(h->stream));
    if (bad) return TRALS_EINVAL;
    if (!(x2 > 0.0)) return TRALS_EINVAL;
    h->xnorm2 = x2;
    // per-mode panels (mode n contiguous)
    for (int n = 0; n < p.N; ++n) {
      int64_t A = 1, B = 1;
      for (int k = 0; k < n; ++k) A *= p.dims[k];
      for (int k = n + 1; k < p.N; ++k) B *= p.dims[k];
      HIPTRY(launch_panel(X_dev, x_dtype, h->at<void>(L.panel[n]), p.panel_dt, A, p.dims[n], B, h->stream));
    }
    if (p.panel_dt == 2)
      HIPTRY(launch_panel(X_dev, x_dtype, h->at<void>(L.fitx), 1, p.E / p.dims[p.N - 1], p.dims[p.N - 1], 1,
                          h->stream));
    return init_cores_and_tables(h, desc);
  }();
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return TRALS_OK;
}

int trals_workspace_bytes_generated(const trals_desc* desc, const trals_source* src, size_t* bytes) {
  if (!bytes || !src) return TRALS_EINVAL;
  Problem p;
  const int rc = validate(desc, &p, src);
  if (rc) return rc;
  Layout L;
  plan(p, &L);
  *bytes = L.total;
  return TRALS_OK;
}

int trals_create_generated(const trals_desc* desc, const trals_source* src, void* ws_dev, size_t ws_bytes,
                           void* stream, trals_handle* out) {
  if (!out || !src || !src->true_cores) return TRALS_EINVAL;
  *out = nullptr;
  Problem p;
  int rc = validate(desc, &p, src);
  if (rc) return rc;
  if (!ws_dev || ((uintptr_t)ws_dev) % kAlign) return TRALS_EINVAL;
  Layout L;
  plan(p, &L);
  if (ws_bytes < L.total) return TRALS_EINVAL;
  trals_ctx* h = new (std::nothrow) trals_ctx();
  if (!h) return TRALS_ENOMEM;
  h->p = p;
  h->L = L;
  h->ws = (char*)ws_dev;
  h->stream = (hipStream_t)stream;
  rc = [&]() -> int {
    HIPTRY(hipMemsetAsync(h->ws + L.scal, 0, 64, h->stream));
    HIPTRY(hipMemsetAsync(h->ws + L.A, 0, (size_t)(p.J + kSketchPadRows) * p.Pmax * p.sk_sz, h->stream));
    // true cores into slice-major FP64
    const size_t esz = src->true_dtype == TRALS_F64 ? 8 : 4;
    size_t off = 0;
    for (int n = 0; n < p.N; ++n) {
      const int Rp = p.tranks[(n + p.N - 1) % p.N], Rn = p.tranks[n];
      const int I = (int)p.dims[n];
      HIPTRY(launch_core_import((const char*)src->true_cores + off, src->true_dtype == TRALS_F64 ? 0 : 1,
                                h->at<void>(L.tcore[n]), 0, Rp, I, Rn, h->stream));
      off += (size_t)Rp * I * Rn * esz;
    }
    // ||TR(G*)||_F^2 by transfer matrices; noise sigma = noise_rel ||TR(G*)||_F / sqrt(prod I)
    const Ring rt = ring_of(p, p.tranks);
    PerMode<const double> T;
    for (int n = 0; n < p.N; ++n) T.p[n] = h->at<const double>(L.tcore[n]);
    // kept on the device (no host round trip): <G*, G*> in inner_res[2], sigma in inner_res[3]
    double* res = h->at<double>(L.inner_res);
    HIPTRY(launch_ring_inner(rt, T, rt, T, h->at<double>(L.inner), res + 2, h->stream));
    double entries = 1.0;
    for (int n = 0; n < p.N; ++n) entries *= (double)p.dims[n];
    HIPTRY(launch_source_scale(res + 2, p.noise_rel, entries, res + 3, h->status(), h->stream));
    return init_cores_and_tables(h, desc, /*wait=*/false);
  }();
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return TRALS_OK;
}

static int run_updates(trals_ctx* h, int64_t count) {
  if (!h) return TRALS_EINVAL;
  if (h->failed) return TRALS_ESTATE;
  if (count < 0) return TRALS_EINVAL;
  for (int64_t u = 0; u < count; ++u) {
    const int rc = run_update(h);
    if (rc) {
      h->failed = true;
      return rc;
    }
  }
  const int rc = table_settle(h);
  if (rc) {
    h->failed = true;
    return rc;
  }
  return sync_status(h);
}

int trals_sweep(trals_handle h, int32_t n_sweeps) {
  if (!h) return TRALS_EINVAL;
  return run_updates(h, (int64_t)n_sweeps * h->p.N);
}

int trals_sweep_async(trals_handle h, int32_t n_sweeps, int32_t flags) {
  if (!h || n_sweeps < 0 || (flags & ~TRALS_ASYNC_FIT)) return TRALS_EINVAL;
  if (h->failed) return TRALS_ESTATE;
  const int64_t count = (int64_t)n_sweeps * h->p.N;
  for (int64_t u = 0; u < count; ++u) {
    const int rc = run_update(h);
    if (rc) {
      h->failed = true;
      return rc;
    }
  }
  {
    const int rc = table_settle(h);
    if (rc) {
      h->failed = true;
      return rc;
    }
  }
  const bool fit = (flags & TRALS_ASYNC_FIT) != 0;
  if (fit) {
    const int rc = h->p.generated ? enqueue_clean_fit(h) : enqueue_dense_fit(h);
    if (rc) return rc;
  }
  if (!h->host_res) h->host_res = (trals_ctx::HostResult*)pinned_get();
  if (h->host_res) {
    // status and fit to pinned host memory, in stream order before the completion event
    h->host_res->fit_valid = fit ? 1 : 0;
    HIPTRY(hipMemcpyAsync(&h->host_res->status, h->status(), sizeof(int), hipMemcpyDeviceToHost, h->stream));
    if (fit)
      HIPTRY(hipMemcpyAsync(&h->host_res->fit, h->at<double>(h->L.inner_res) + 4, sizeof(double),
                            hipMemcpyDeviceToHost, h->stream));
  }
  if (!h->done) HIPTRY(hipEventCreateWithFlags(&h->done, hipEventDisableTiming));
  HIPTRY(hipEventRecord(h->done, h->stream));
  h->pending = true;
  h->async_fit = fit;
  return TRALS_OK;
}

int trals_query(trals_handle h, double* fit) {
  if (!h) return TRALS_EINVAL;
  if (fit) *fit = NAN;
  if (h->failed) return TRALS_ESTATE;
  if (!h->pending) return TRALS_OK;
  const hipError_t q = hipEventQuery(h->done);
  if (q == hipErrorNotReady) return TRALS_PENDING;
  HIPTRY(q);
  h->pending = false;
  if (h->host_res) {
    if (h->host_res->status != kDevOk) {
      h->failed = true;
      return TRALS_ESINGULAR;
    }
    if (fit && h->host_res->fit_valid) *fit = h->host_res->fit;
    return TRALS_OK;
  }
  // no pinned slot: the stream is idle, so this copies the status word and returns at once
  const int rc = sync_status(h);
  if (rc == TRALS_OK && fit && h->async_fit) {
    HIPTRY(hipMemcpy(fit, h->at<double>(h->L.inner_res) + 4, sizeof(double), hipMemcpyDeviceToHost));
  }
  return rc;
}

int trals_step(trals_handle h, int32_t n_updates) { return run_updates(h, n_updates); }

int trals_fit_error(trals_handle h, double* rel_err) {
  if (!h || !rel_err) return TRALS_EINVAL;
  if (h->failed) return TRALS_ESTATE;
  const Problem& p = h->p;
  if (p.generated) {
    // ||TR(G) - TR(G*)||^2 = <G,G> - 2 <G,G*> + <G*,G*> by transfer matrices (noise excluded)
    const Ring rr = make_ring(p), rt = ring_of(p, p.tranks);
    PerMode<const double> G, T;
    for (int n = 0; n < p.N; ++n) {
      G.p[n] = h->at<const double>(h->L.core[n]);
      T.p[n] = h->at<const double>(h->L.tcore[n]);
    }
    double* work = h->at<double>(h->L.inner);
    double* res = h->at<double>(h->L.inner_res);
    HIPTRY(launch_ring_inner(rr, G, rr, G, work, res, h->stream));
    HIPTRY(launch_ring_inner(rr, G, rt, T, work, res + 1, h->stream));
    double r[3] = {0.0, 0.0, 0.0};
    HIPTRY(hipMemcpyAsync(r, res, 24, hipMemcpyDeviceToHost, h->stream));
    const int st = sync_status(h);
    if (st) return st;
    const double d2 = r[0] - 2.0 * r[1] + r[2];
    *rel_err = sqrt((d2 > 0.0 ? d2 : 0.0) / r[2]);
    return TRALS_OK;
  }
  FitArgs fa;
  memset(&fa, 0, sizeof(fa));
  fa.ring = make_ring(p);
  for (int m = 0; m < p.N; ++m) fa.cores.p[m] = h->at<const void>(h->L.core[m]);
  fa.X = h->at<const void>(h->L.fitx);
  fa.rows = p.E / p.dims[p.N - 1];
  fa.partial = h->at<double>(h->L.partial);
  int nb = 0;
  HIPTRY(launch_fit(fa, 0, p.panel_dt == 2 ? 1 : p.panel_dt, &nb, h->stream));
  HIPTRY(launch_sum_partials(fa.partial, nb, h->scal_d(), h->stream));
  double r2 = 0.0;
  HIPTRY(hipMemcpyAsync(&r2, h->scal_d(), 8, hipMemcpyDeviceToHost, h->stream));
  HIPTRY(hipStreamSynchronize(h->stream));
  *rel_err = sqrt(r2 / h->xnorm2);
  return TRALS_OK;
}

int trals_destroy(trals_handle h) {
  if (!h) return TRALS_OK;
  if (h->pending) (void)hipStreamSynchronize(h->stream);  // work may still use the workspace
  if (h->aux) {
    (void)hipStreamSynchronize(h->aux);  // a table check left behind by a failed update
    (void)hipStreamDestroy(h->aux);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->done) (void)hipEventDestroy(h->done);
  pinned_put(h->host_res);
  for (auto& v : h->prof.ev)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
  delete h;
  return TRALS_OK;
}

int trals_profile(trals_handle h, int32_t enable) {
  if (!h) return TRALS_EINVAL;
  HIPTRY(hipStreamSynchronize(h->stream));
  h->prof.on = enable != 0;
  for (int k = 0; k < TRALS_K_COUNT; ++k) {
    h->prof.used[k] = 0;
    h->prof.ms[k] = 0.0;
    h->prof.count[k] = 0;
  }
  return TRALS_OK;
}

int trals_profile_read(trals_handle h, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!h || kernel < 0 || kernel >= TRALS_K_COUNT) return TRALS_EINVAL;
  HIPTRY(hipStreamSynchronize(h->stream));
  for (int k = 0; k < TRALS_K_COUNT; ++k) {
    Prof& pr = h->prof;
    for (size_t i = 0; i < pr.used[k]; ++i) {
      float ms = 0.f;
      HIPTRY(hipEventElapsedTime(&ms, pr.ev[k][2 * i], pr.ev[k][2 * i + 1]));
      pr.ms[k] += ms;
      pr.count[k] += 1;
    }
    pr.used[k] = 0;
  }
  if (total_ms) *total_ms = h->prof.ms[kernel];
  if (launches) *launches = h->prof.count[kernel];
  return TRALS_OK;
}

int trals_get_cores(trals_handle h, void* dst_dev, int32_t dtype) {
  if (!h || !dst_dev || (dtype != TRALS_F64 && dtype != TRALS_F32)) return TRALS_EINVAL;
  const Problem& p = h->p;
  const size_t esz = dtype == TRALS_F64 ? 8 : 4;
  size_t off = 0;
  for (int n = 0; n < p.N; ++n) {
    const int Rp = p.ranks[(n + p.N - 1) % p.N], Rn = p.ranks[n];
    const int I = (int)p.dims[n];
    HIPTRY(launch_core_export(h->at<const void>(h->L.core[n]), 0, (char*)dst_dev + off,
                              dtype == TRALS_F64 ? 0 : 1, Rp, I, Rn, h->stream));
    off += (size_t)Rp * I * Rn * esz;
  }
  HIPTRY(hipStreamSynchronize(h->stream));
  return TRALS_OK;
}

int trals_set_cores(trals_handle h, const void* src_dev, int32_t dtype) {
  if (!h || !src_dev || (dtype != TRALS_F64 && dtype != TRALS_F32)) return TRALS_EINVAL;
  HIPTRY(hipMemsetAsync(h->ws + h->L.scal + 16, 0, sizeof(int), h->stream));
  h->failed = false;
  int rc = load_cores(h, src_dev, dtype);
  if (rc) return rc;
  for (int m = 0; m < h->p.N; ++m) h->table_valid[m] = false;
  const int nxt = (int)(h->upd % h->p.N);
  for (int m = 0; m < h->p.N; ++m)
    if (m != nxt) {
      rc = compute_table(h, m);
      if (rc) return rc;
    }
  return sync_status(h);
}

int trals_get_last_samples(trals_handle h, int32_t* idx_host, double* w_host) {
  if (!h || h->p.method == TRALS_EXACT) return TRALS_EINVAL;
  if (!h->have_last) return TRALS_ESTATE;
  const Problem& p = h->p;
  if (idx_host)
    HIPTRY(hipMemcpyAsync(idx_host, h->at<void>(h->L.idx), (size_t)p.J * (p.N - 1) * 4, hipMemcpyDeviceToHost,
                          h->stream));
  if (w_host)
    HIPTRY(hipMemcpyAsync(w_host, h->at<void>(h->L.w), (size_t)p.J * 8, hipMemcpyDeviceToHost, h->stream));
  HIPTRY(hipStreamSynchronize(h->stream));
  return TRALS_OK;
}

int64_t trals_update_counter(trals_handle h) { return h ? h->upd : -1; }

int trals_set_samples(trals_handle h, int64_t samples) {
  if (!h || h->p.method == TRALS_EXACT) return TRALS_EINVAL;
  if (samples < h->p.Pmax || samples > h->p.Jcap) return TRALS_EINVAL;
  h->p.J = samples;
  h->have_last = false;
  return TRALS_OK;
}

int64_t trals_samples(trals_handle h) { return h ? h->p.J : -1; }

int trals_fit_estimate(trals_handle h, int64_t samples, uint64_t tag, double* rel_err) {
  if (!h || !rel_err || samples < 1 || samples > ((int64_t)1 << 40)) return TRALS_EINVAL;
  if (h->p.generated) return TRALS_EINVAL;  // the estimate reads entries of a dense X
  if (h->failed) return TRALS_ESTATE;
  const Problem& p = h->p;
  FitSampleArgs fa;
  memset(&fa, 0, sizeof(fa));
  fa.ring = make_ring(p);
  for (int m = 0; m < p.N; ++m) fa.cores.p[m] = h->at<const void>(h->L.core[m]);
  fa.X = h->at<const void>(h->L.fitx);
  fa.E = p.E;
  fa.S = samples;
  fa.seed = p.seed;
  fa.stream_id = p.stream_id;
  fa.tag = tag;
  fa.partial = h->at<double>(h->L.partial);
  int nb = 0;
  HIPTRY(launch_fit_sample(fa, p.panel_dt == 2 ? 1 : p.panel_dt, &nb, h->stream));
  HIPTRY(launch_sum_partials(fa.partial, nb, h->scal_d(), h->stream));
  double r2 = 0.0;
  HIPTRY(hipMemcpyAsync(&r2, h->scal_d(), 8, hipMemcpyDeviceToHost, h->stream));
  const int st = sync_status(h);
  if (st) return st;
  *rel_err = sqrt(((double)p.E / (double)samples) * r2 / h->xnorm2);
  return TRALS_OK;
}

int trals_sweep_until_estimate(trals_handle h, int32_t max_sweeps, double rel_tol, int64_t samples,
                               int32_t* sweeps_done, double* last_estimate, double* last_change) {
  if (!h || max_sweeps < 1 || !(rel_tol >= 0.0)) return TRALS_EINVAL;
  if (h->failed) return TRALS_ESTATE;
  double prev = 0.0, change = -1.0;
  int rc = trals_fit_estimate(h, samples, 0, &prev);
  if (rc) return rc;
  double cur = prev;
  int32_t done = 0;
  while (done < max_sweeps) {
    rc = run_updates(h, h->p.N);
    if (rc) break;
    ++done;
    rc = trals_fit_estimate(h, samples, 0, &cur);
    if (rc) break;
    change = cur > 0.0 ? fabs(cur - prev) / cur : 0.0;
    prev = cur;
    if (change < rel_tol) break;
  }
  if (sweeps_done) *sweeps_done = done;
  if (last_estimate) *last_estimate = cur;
  if (last_change) *last_change = change;
  return rc;
}

int trals_tr_norm(trals_handle h, double* norm) {
  if (!h || !norm) return TRALS_EINVAL;
  if (h->failed) return TRALS_ESTATE;
  const int rc = ring_norm_enqueue(h);
  if (rc) return rc;
  double g2 = 0.0;
  HIPTRY(hipMemcpyAsync(&g2, h->at<double>(h->L.inner_res), 8, hipMemcpyDeviceToHost, h->stream));
  HIPTRY(hipStreamSynchronize(h->stream));
  *norm = sqrt(g2 > 0.0 ? g2 : 0.0);
  return TRALS_OK;
}

int trals_sweep_until(trals_handle h, int32_t max_sweeps, double rel_tol, int32_t* sweeps_done,
                      double* last_change) {
  if (!h || max_sweeps < 1 || !(rel_tol >= 0.0)) return TRALS_EINVAL;
  if (h->failed) return TRALS_ESTATE;
  double prev = 0.0, change = -1.0;
  int rc = trals_tr_norm(h, &prev);
  if (rc) return rc;
  int32_t done = 0;
  while (done < max_sweeps) {
    rc = run_updates(h, h->p.N);
    if (rc) break;
    ++done;
    double cur = 0.0;
    rc = trals_tr_norm(h, &cur);
    if (rc) break;
    change = cur > 0.0 ? fabs(cur - prev) / cur : 0.0;
    prev = cur;
    if (change < rel_tol) break;
  }
  if (sweeps_done) *sweeps_done = done;
  if (last_change) *last_change = change;
  return rc;
}

int trals_set_update_counter(trals_handle h, int64_t counter) {
  if (!h || counter < 0) return TRALS_EINVAL;
  h->upd = counter;
  h->have_last = false;
  return TRALS_OK;
}

}  // extern "C"
