// Host-side internals of libtt: the index object, its workspace and the
// kernel launchers implemented in the .hip translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/tt.h"

namespace tt {

// Work partition constants.  The streaming chunk size, the Gram task size,
// the light/heavy Gram threshold and the heavy-task workgroup width are
// per-index tuning parameters (tt_index_tune); these are their defaults and
// the supported streaming chunk sizes.
constexpr int kChunkDefault = 1024;
constexpr int kGramPieceDefault = 4096;
constexpr int kGramLightDefault = 512;
constexpr int kGramWavesDefault = 4;
constexpr int kSolveWgsDefault = 0;
constexpr int kPcgWgsDefault = -1;
constexpr int kCcdXcdDefault = -1;
constexpr int kCcdLdsDefault = -1;
// Largest record set a CCD++ pass copies into LDS (tuning ccd_lds).
constexpr int64_t kCcdLdsBytes = 48 * 1024;
constexpr int kReduceMin = 4;      // rows with more tasks are pre-reduced
constexpr int kSegSlots = 16;      // carry slots summed per first-level block
constexpr int64_t kGramBatchBytes = 256ll << 20;  // Gram workspace per batch

// Elements of one Gram task's matrix in the lower-tile layout (the
// NB (NB + 1) / 2 lower 16 x 16 tiles of the RP x RP matrix, NB = RP / 16).
__host__ __device__ constexpr int gram_task_elems(int RP) { return 128 * (RP / 16) * (RP / 16 + 1); }

// CCD++ layout of one mode's stream (index.hip, built on first use): the
// nonzeros of each row grouped by the bucket of their index in the mode
// with the most rows among the others (kCcdBuckets row ranges of balanced
// nonzero count), tasks cut at bucket boundaries and at gram_piece
// nonzeros, and a schedule that gives bucket b's tasks to workgroups b,
// b + kCcdBuckets, ...: workgroups are dispatched to the XCDs in turn, so
// each XCD's L2 sees the column records of one bucket's rows only.
constexpr int kCcdBuckets = 8;
struct CcdLayout {
  bool built = false;
  int big = -1;                          // the bucketed mode (-1: no layout)
  int32_t bnd[kCcdBuckets + 1] = {};     // bucket row boundaries in mode `big`
  int32_t *d_key = nullptr;              // new order: row of each nonzero
  int32_t *d_oidx[TT_MAX_ORDER] = {};    // new order: the other modes' indices
  int32_t *d_inv = nullptr;              // sorted position -> new position
  int64_t ntask = 0;
  int64_t *d_task = nullptr;             // ntask + 1 boundaries in the new order
  int32_t *d_row_task = nullptr;         // I + 1: tasks of row i
  int64_t nsched = 0;                    // workgroups of a pass (4 tasks each)
  int32_t *d_sched = nullptr;            // nsched * 4 task ids, -1 = none
};

struct ModeIndex {
  int64_t I = 0;
  std::vector<int64_t> h_ptr;   // host copy of the row pointers (partitions)
  std::vector<void *> part;     // device arrays of the current partitions
  int64_t nrows = 0;            // rows holding >= 1 nonzero
  int64_t *d_ptr = nullptr;     // I + 1 offsets into the sorted stream
  int32_t *d_perm = nullptr;    // sorted position -> COO position
  int32_t *d_key = nullptr;     // sorted mode index
  int32_t *d_oidx[TT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr};
  void *d_t = nullptr;          // observed values in this mode's order
  int32_t *d_rows = nullptr;    // nonzero rows
  // streaming partition: chunks of whole light rows (<= chunk nnz) and
  // single pieces of heavy rows (> chunk nnz)
  int64_t nchunk = 0;
  int64_t *d_chunk = nullptr;       // nchunk + 1 boundaries
  int32_t *d_chunk_slot = nullptr;  // -1: light chunk; else carry slot
  int64_t nslot = 0;
  int64_t nheavy = 0;
  int32_t *d_heavy_row = nullptr;   // nheavy
  int32_t *d_heavy_slot = nullptr;  // nheavy + 1
  int64_t nseg = 0;                 // carry segments (<= kSegSlots slots each)
  int32_t *d_seg = nullptr;         // nseg + 1 slot boundaries
  int32_t *d_heavy_seg = nullptr;   // nheavy + 1 segment ranges
  // Gram tasks: pieces of <= gram_piece nnz of one row
  int64_t ntask = 0;
  int64_t *d_task = nullptr;        // ntask + 1 boundaries
  int32_t *d_row_task = nullptr;    // I + 1: tasks of row i
  std::vector<int32_t> h_row_task;  // host copy, for batching
  std::vector<int64_t> h_task;      // host copy of task boundaries
  std::vector<int64_t> h_heavy_nnz; // prefix sums of heavy-task sizes
  int32_t max_task_per_row = 0;
  int32_t *d_heavy_task = nullptr;  // tasks with > gram_light nonzeros of rows with
  std::vector<int32_t> h_heavy_task;  // several tasks
  int32_t *d_multi_row = nullptr;   // rows with > kReduceMin tasks
  std::vector<int32_t> h_multi_row;
  // rows whose only Gram task is light: their Gram is formed inside the
  // solve kernel (no workspace); the other rows; the light tasks of rows
  // with several tasks (all ascending)
  int32_t *d_solo_row = nullptr;
  std::vector<int32_t> h_solo_row;
  std::vector<int64_t> h_solo_nnz;  // prefix sums of the solo rows' nonzeros
  int32_t *d_rest_row = nullptr;
  std::vector<int32_t> h_rest_row;
  // rows whose only Gram task is heavy (ascending)
  int32_t *d_hsolo_row = nullptr;
  std::vector<int32_t> h_hsolo_row;
  std::vector<int64_t> h_hsolo_nnz;  // prefix sums of the heavy solo rows' nonzeros
  // the same partition without the heavy solo class (for ranks whose heavy
  // solo rows are not fused with their solve): every heavy task, and every
  // row that is not solo
  int32_t *d_heavy_task_all = nullptr;
  std::vector<int32_t> h_heavy_task_all;
  std::vector<int64_t> h_heavy_nnz_all;
  int32_t *d_rest_row_all = nullptr;
  std::vector<int32_t> h_rest_row_all;
  int32_t *d_light_task = nullptr;
  std::vector<int32_t> h_light_task;
  double mean_row = 0.0;            // m / nrows
  CcdLayout ccd;                    // arrays in `part` (rebuilt with the partitions)
};

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace tt

struct tt_index {
  int N = 0;
  int64_t dims[TT_MAX_ORDER] = {0, 0, 0, 0};
  int64_t m = 0;
  tt_dtype vdt = TT_F32;
  bool has_t = false;
  tt::ModeIndex mode[TT_MAX_ORDER];
  std::vector<void *> owned;                 // device allocations to free
  std::map<std::string, tt::Buf> ws;         // named workspace buffers
  int64_t max_I = 0, sum_I = 0, max_nchunk = 0, max_nslot = 0, max_nseg = 0;
  tt_tuning tune = {tt::kChunkDefault, tt::kGramPieceDefault, tt::kGramLightDefault,
                    tt::kGramWavesDefault, tt::kSolveWgsDefault, tt::kPcgWgsDefault,
                    tt::kCcdXcdDefault, tt::kCcdLdsDefault};
  int cu_count = 0;  // compute units of the device the index was built on
  // Gauss-Newton position map (built on first use, N x m): slot n != zmode
  // maps mode-n sorted positions to mode-zmode sorted positions
  int32_t *d_zmap = nullptr;
};

namespace tt {

// ----- index partitions (index.hip) ------------------------------------------
tt_status build_partitions(tt_index *ix, int n, hipStream_t s);
// Mode whose factor rows are the costliest to gather (the most rows): the
// Gauss-Newton matvec evaluates its per-nonzero scalars in that mode's order.
int gn_zmode(const tt_index *ix);
// The index's Gauss-Newton position map, built (allocated, filled on stream s
// and synchronized) on first use; fails while s is capturing a graph.
tt_status zmap_get(tt_index *ix, hipStream_t s, const int32_t **out);
// The CCD++ layout of mode n (built on first use: allocates and
// synchronizes s), or *out = NULL when the tuning (ccd_xcd) or the shape
// does not call for one; vsz = bytes of one dense value.
tt_status ccd_layout_get(tt_index *ix, int n, size_t vsz, hipStream_t s,
                         const CcdLayout **out);

// ----- error handling ------------------------------------------------------
void set_error(const char *fmt, ...);
tt_status hip_fail(hipError_t e, const char *what);
#define TT_HIP(call)                                           \
  do {                                                         \
    hipError_t _e = (call);                                    \
    if (_e != hipSuccess) return ::tt::hip_fail(_e, #call);    \
  } while (0)
#define TT_CHECK(cond, ...)                                    \
  do {                                                         \
    if (!(cond)) {                                             \
      ::tt::set_error(__VA_ARGS__);                            \
      return TT_ERR_INVALID_ARG;                               \
    }                                                          \
  } while (0)

// Workspace buffer `name` of at least `bytes`, grown (never shrunk) on demand;
// growth fails with TT_ERR_INVALID_ARG while an instantiated graph is alive.
tt_status ws_get(tt_index *ix, const char *name, size_t bytes, void **out);
// Number of instantiated graphs not yet destroyed (process-wide).
int live_graphs();

inline size_t dtype_size(tt_dtype d) { return d == TT_F64 ? 8 : (d == TT_F32 ? 4 : 2); }
inline size_t value_size(tt_dtype fdt) { return fdt == TT_F64 ? 8 : 4; }

// ----- kernel profiler ------------------------------------------------------
// While enabled, ProfScope brackets a launch with HIP events on its stream
// and tags it with algorithmic bytes and flops (process-global state).
struct ProfScope {
  ProfScope(const char *name, hipStream_t s, double bytes, double flops);
  ~ProfScope();
  int slot = -1;
  hipStream_t stream = nullptr;
};
bool prof_on();

// ----- launchers (return hipError_t of the last launch) ----------------------
// index.hip
tt_status build_index_impl(int N, const int64_t *dims, int64_t m,
                           const int32_t *const *d_idx, const void *d_t,
                           tt_dtype vdt, hipStream_t s, tt_index *ix);

// stream.hip: per-nonzero and segmented kernels over one mode's sorted stream.
struct StreamCall {
  const tt_index *ix;
  int mode;                 // stream (sorted) order processed
  int R;
  int64_t ldA;
  tt_dtype fdt;
  const void *A[TT_MAX_ORDER];   // factors (NULL entries allowed for TTTP)
  const void *X[TT_MAX_ORDER];   // GN direction blocks
  const void *s;            // per-nonzero values in this mode's order or NULL
  const int32_t *s_perm;    // if non-NULL, s is in COO order: s[perm[e]]
  double w_const;
  int epi, loss;
  double lam_own;           // GRAD/GN: added lam_own * own row (done by prefill)
  void *out;                // dense (I x R) or per-nonzero output
  const int32_t *out_perm;  // TTTP: scatter to out[perm[e]] when non-NULL
  int accumulate;
  double *sum_parts;        // TTTP: per-chunk FP64 partial sums (or NULL)
  double *carry;            // segmented: carry workspace
  double *carry_partial;    // heavy-row partials (NULL: after the index-wide carry slots)
  const double *skip;       // optional device flag: launches become no-ops
  void *zout;               // when non-NULL, also store per nonzero (value dtype, this
                            // mode's sorted order): GN w_e * z_e, gradient phi''(t_e, m_e)
  const char *prof_name;    // profiler tag (NULL: named after the operation)
};
enum StreamOp { OP_TTTP = 0, OP_MTTKRP = 1, OP_GRAD = 2, OP_GN = 3, OP_NEWTON = 4 };
hipError_t launch_stream(StreamOp op, const StreamCall &c, hipStream_t s);
int stream_group_width(tt_dtype fdt, int R);
int stream_rp(tt_dtype fdt, int R);

// The conjugate-gradient loop of tt_gn_step as one persistent kernel
// (pcg_loop_impl.h), for R <= kPcgMaxRank.  pass[0] is the OP_GN pass of
// the Gauss-Newton product and pass[1], pass[2] its OP_MTTKRP passes, set
// up as gn_matvec sets them up (their carry and skip fields are replaced).
constexpr int kPcgMaxRank = 16;
// PCG scalar slot that the persistent loop sets to 1 when a barrier wait
// gave up (the step is then not applied), 0 otherwise
constexpr int kPcgAbortSlot = 11;
struct PcgLoopCall {
  StreamCall pass[3];
  double *carry;            // pcg_loop_carry_doubles(ix) doubles
  const void *L[TT_MAX_ORDER];   // preconditioner factors per mode
  void *x, *r, *z, *p, *q;  // PCG vectors, dense dtype, modes' blocks in order
  double lambda2;
  double *parts;            // 3 x dot_parts_needed(sum_n I_n R) doubles
  double *sc;               // PCG scalar slots after stage 0
  double tol;
  int kmax;
  unsigned *bar;            // pcg_loop_bar_words() barrier words
  int wgs_per_cu;
};
int64_t pcg_loop_carry_doubles(const tt_index *ix);
int pcg_loop_bar_words();
// Largest iteration count one launch can take with wgs_per_cu workgroups
// per compute unit (its barrier counter must not wrap).
int64_t pcg_loop_max_iters(const tt_index *ix, int wgs_per_cu);
hipError_t launch_pcg_loop(const PcgLoopCall &c, hipStream_t s);
// Automatic choice (pcg_wgs = -1): the persistent loop when every streaming
// phase fits in one round of a grid of two resident workgroups per compute
// unit, i.e. the launch-bound sizes where it pays.
bool pcg_loop_fits(const PcgLoopCall &c);

// MTTKRP after argument checks (api.cpp).  `carry` = NULL takes the carry
// slots from the index workspace; otherwise `carry` holds this mode's slots
// (nslot x stream_rp) followed by its heavy-row partials (nseg x stream_rp).
tt_status mttkrp_checked(tt_index *ix, const void *d_s, int s_order, const void *const *d_A,
                         int R, int64_t ldA, tt_dtype fdt, int mode, void *d_out,
                         int accumulate, hipStream_t stream, double *carry);

// solve.hip: Gram on matrix cores + batched FP64 Cholesky.
struct SolveCall {
  const tt_index *ix;
  int mode, R;
  int64_t ldA;
  tt_dtype fdt;
  const void *A[TT_MAX_ORDER];
  const void *w;            // weights in this mode's order, or NULL
  const int32_t *w_perm;    // COO-order weights gathered through perm
  double w_scale;           // weights are multiplied by this (1 normally)
  double lambda;
  const void *rhs;          // I x R dense dtype (ignored when fused_rhs)
  int fused_rhs;            // 1: rhs = MTTKRP of the observed values, formed in the
                            // Gram pass (FP32 and BF16 forms)
  void *X;                  // I x R in fdt, leading dim ldA (may alias A)
  int32_t *info;            // optional
  void *Lstore;             // when non-NULL: keep the Cholesky factors (I x RP(RP+1)/2),
                            // FP64 for the FP64 form, FP32 otherwise
  int factor_only;          // 1: factor and store, no solve
  // Newton form of alternating minimization (FP32 and BF16 forms; needs
  // fused_rhs, w NULL, w_scale 1): one pass forms G = sum phi''(t, m) h h^T
  // and M = sum phi'(t, m) h with m the model value from A[mode], and the
  // rows solve (G + lambda I) x = -(M + own_coef A[mode][i])
  int newton;
  int loss;
  double own_coef;
  const double *skip;       // optional device flag: every launch becomes a no-op
  // FP32 / BF16 least-squares form with fused_rhs: also write the model value
  // <A[mode][i], h_e> of every nonzero (factors before the update) to model[e]
  // in this mode's sorted order (value dtype), from the Gram pass's gathers
  void *model;
};
tt_status run_solve_factor(tt_index *ix, const SolveCall &c, hipStream_t s);
// The Gram (and fused right-hand-side) workspaces of one row batch of
// Solve Factor on `mode`; acquiring them first lets a call fail before it
// enqueues anything.
tt_status solve_workspace(tt_index *ix, int mode, int R, tt_dtype fdt, bool fused_rhs,
                          void **G, double **M);
// Apply stored factors: X = (L L^T)^{-1} rhs, X dense dtype (not fdt).
hipError_t launch_apply_factor(const tt_index *ix, int mode, int R, tt_dtype fdt,
                               const void *Lstore, const void *rhs, void *X,
                               const double *skip, hipStream_t s);

// vec.hip: dense helpers (dense dtype = double for TT_F64 else float).
hipError_t launch_fill(void *p, int64_t n, tt_dtype dense, double v, hipStream_t s);
// y[i*R + r] = a * x[i*ldx + r] (+ b * y) over I rows; x in dtype xdt.
hipError_t launch_scale_rows(void *y, const void *x, tt_dtype xdt, int64_t ldx,
                             int64_t I, int R, double a, tt_dtype ydt, hipStream_t s);
hipError_t launch_sum_doubles(const double *parts, int64_t n, double *out,
                              int accumulate, hipStream_t s, const double *skip = nullptr);
hipError_t launch_sumsq_rows(const void *A, tt_dtype fdt, int64_t ldA, int64_t I,
                             int R, double scale, double *parts, int64_t *nparts,
                             hipStream_t s, const double *skip = nullptr);
int64_t sumsq_parts_needed(int64_t I, int R);

// PCG vector kernels (blocks concatenated into one contiguous dense array).
hipError_t launch_dot_parts(const void *x, const void *y, int64_t n, tt_dtype dense,
                            double *parts, int64_t *nparts, hipStream_t s);
int64_t dot_parts_needed(int64_t n);
hipError_t launch_axpy2(void *x, const void *p, void *r, const void *q, int64_t n,
                        tt_dtype dense, const double *sc, int ia, hipStream_t s);
hipError_t launch_xpby(void *p, const void *z, int64_t n, tt_dtype dense,
                       const double *sc, int ib, hipStream_t s);
hipError_t launch_pcg_scalar(double *sc, int stage, double tol, hipStream_t s);
// stats[0..3] = iterations, final relative residual, initial residual norm, *f0
hipError_t launch_pcg_stats(const double *sc, const double *f0, double *stats, hipStream_t s);
hipError_t launch_add_to_factor(void *A, tt_dtype fdt, int64_t ldA, int64_t I, int R,
                                const void *dx, hipStream_t s, const double *skip = nullptr);
// A += D, both I x R in the factor dtype fdt with leading dimensions ldA, ldD.
hipError_t launch_add_rows(void *A, int64_t ldA, const void *D, int64_t ldD, tt_dtype fdt,
                           int64_t I, int R, hipStream_t s, const double *skip = nullptr);
// One CCD++ column update (ccd.hip): every mode's column r in turn; rho[n]
// = residual in mode n's order, recs[n] = I_n records (column r - 1 old,
// new; column r old, current; dense dtype, aligned to 4 values), carried
// from column to column: mode n's pass of column r > 0 first moves its
// residual copy from column r - 1's old to its new rank-1 term.  lay[n]:
// mode n's CCD++ layout or NULL (lay may be NULL).  part = 2 x max tasks
// doubles.
hipError_t launch_ccd_column(const tt_index *ix, int r, void *const *d_A, int64_t ldA,
                             tt_dtype fdt, double lambda, void *const *rho, void *const *recs,
                             const CcdLayout *const *lay, double *part, int32_t *d_info,
                             hipStream_t s);
// Alternating-minimization Newton bookkeeping on the device (see vec.hip).
hipError_t launch_gam_flag(double *sc, double tol, int count, int check, hipStream_t s);

}  // namespace tt
