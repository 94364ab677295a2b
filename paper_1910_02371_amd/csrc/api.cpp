// C ABI of libtt: argument checking, dispatch onto the kernels, and the two
// completion drivers built from the primitives (ALS sweep, Section 2.2;
// preconditioned Gauss-Newton step, Section 2.5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

namespace tt {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

tt_status hip_fail(hipError_t e, const char *what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return TT_ERR_HIP;
}

// Instantiated graphs alive in the process (tt_graph_end .. tt_graph_destroy).
// A graph replays its kernels on the device addresses recorded at capture,
// so while any is alive no workspace may be reallocated and no partition
// rebuilt.
static std::atomic<int> g_live_graphs{0};

int live_graphs() { return g_live_graphs.load(); }

tt_status ws_get(tt_index *ix, const char *name, size_t bytes, void **out) {
  Buf &b = ix->ws[name];
  if (b.bytes < bytes) {
    if (b.p && live_graphs() > 0) {
      set_error("workspace '%s' would grow from %zu to %zu bytes while %d instantiated "
                "graph(s) replay kernels on it: destroy the graphs first, or reserve the "
                "workspaces (tt_index_reserve) for the largest call before capturing",
                name, b.bytes, bytes, live_graphs());
      return TT_ERR_INVALID_ARG;
    }
    if (b.p) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "workspace resize");
      hipFree(b.p);
      b.p = nullptr;
      b.bytes = 0;
    }
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
      set_error("workspace '%s' of %zu bytes: %s", name, want, hipGetErrorString(e));
      return TT_ERR_OOM;
    }
    b.bytes = want;
  }
  *out = b.p;
  return TT_OK;
}

#define TT_ST(x)                          \
  do {                                    \
    tt_status _s = (x);                   \
    if (_s != TT_OK) return _s;           \
  } while (0)
#define TT_LAUNCH(x, what)                               \
  do {                                                   \
    hipError_t _e = (x);                                 \
    if (_e != hipSuccess) return hip_fail(_e, what);     \
  } while (0)

static tt_dtype dense_of(tt_dtype fdt) { return fdt == TT_F64 ? TT_F64 : TT_F32; }

static tt_status check_common(const tt_index *ix, int R, int64_t ldA, tt_dtype fdt) {
  TT_CHECK(ix != nullptr, "index is NULL");
  TT_CHECK(fdt == TT_F64 || fdt == TT_F32 || fdt == TT_BF16, "bad factor dtype %d", (int)fdt);
  TT_CHECK(R >= 1 && R <= TT_MAX_RANK, "rank %d outside [1, %d]", R, TT_MAX_RANK);
  TT_CHECK(ldA >= R, "ldA %lld < R %d", (long long)ldA, R);
  // kernels address factor and dense blocks with 32-bit byte offsets
  if ((double)ix->max_I * (double)ldA * 8.0 >= 4294967296.0) {
    set_error("factor matrices of %lld x %lld elements exceed the 4 GiB addressing limit",
              (long long)ix->max_I, (long long)ldA);
    return TT_ERR_UNSUPPORTED;
  }
  if (ix->N != 3) {
    set_error("order %d: the GPU kernels implement order-3 tensors", ix->N);
    return TT_ERR_UNSUPPORTED;
  }
  return TT_OK;
}

// Per-nonzero array in the order of `mode`: returns (pointer, perm) where
// perm != NULL means "gather through perm" (COO order input).
static tt_status resolve_values(const tt_index *ix, const void *v, int order, int mode,
                                tt_dtype fdt, const void **out, const int32_t **perm,
                                const char *what) {
  *perm = nullptr;
  *out = nullptr;
  if (v == nullptr) return TT_OK;
  if (v == TT_INDEX_T) {
    TT_CHECK(ix->has_t, "%s: the index holds no observed values", what);
    TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64),
             "%s: value dtype of the index does not match the factor dtype", what);
    *out = ix->mode[mode].d_t;
    return TT_OK;
  }
  if (order == TT_ORDER_PER_MODE) {
    const void *const *arr = reinterpret_cast<const void *const *>(v);
    TT_CHECK(arr[mode] != nullptr, "%s: per-mode array %d is NULL", what, mode);
    *out = arr[mode];
    return TT_OK;
  }
  if (order == TT_ORDER_COO) {
    *out = v;
    *perm = ix->mode[mode].d_perm;
    return TT_OK;
  }
  TT_CHECK(order >= 0 && order < ix->N, "%s: bad order %d", what, order);
  if (order != mode) {
    set_error("%s: values in mode-%d order cannot feed a mode-%d pass", what, order, mode);
    return TT_ERR_UNSUPPORTED;
  }
  *out = v;
  return TT_OK;
}

static tt_status carry_ws(tt_index *ix, double **carry) {
  void *p = nullptr;
  // carry slots, then first-level partials of the heavy-row reduction
  TT_ST(ws_get(ix, "carry",
               (size_t)(std::max<int64_t>(ix->max_nslot, 1) + std::max<int64_t>(ix->max_nseg, 1)) *
                   64 * 8,
               &p));
  *carry = (double *)p;
  return TT_OK;
}

static StreamCall base_call(const tt_index *ix, int mode, int R, int64_t ldA, tt_dtype fdt) {
  StreamCall c;
  memset(&c, 0, sizeof(c));
  c.ix = ix;
  c.mode = mode;
  c.R = R;
  c.ldA = ldA;
  c.fdt = fdt;
  c.w_const = 1.0;
  return c;
}

// Process TTTP in `mode` order; internal (no argument checks).
static tt_status tttp_mode(tt_index *ix, int mode, const void *s, const int32_t *s_perm,
                           const void *const *d_A, int R, int64_t ldA, tt_dtype fdt, int epi,
                           int loss, void *out, const int32_t *out_perm, double *d_sum,
                           const double *skip, hipStream_t st) {
  StreamCall c = base_call(ix, mode, R, ldA, fdt);
  for (int p = 0; p < ix->N; ++p) c.A[p] = d_A[p];
  c.s = s;
  c.s_perm = s_perm;
  c.epi = epi;
  c.loss = loss;
  c.out = out;
  c.out_perm = out_perm;
  c.skip = skip;
  if (d_sum) {
    void *p = nullptr;
    TT_ST(ws_get(ix, "tsum", (size_t)std::max<int64_t>(ix->max_nchunk, 1) * 8, &p));
    c.sum_parts = (double *)p;
  }
  TT_LAUNCH(launch_stream(OP_TTTP, c, st), "tttp kernel");
  if (d_sum) {
    if (ix->mode[mode].nchunk > 0)
      TT_LAUNCH(launch_sum_doubles(c.sum_parts, ix->mode[mode].nchunk, d_sum, 0, st), "sum");
    else
      TT_LAUNCH(launch_fill(d_sum, 1, TT_F64, 0.0, st), "sum");
  }
  return TT_OK;
}

static int best_mode(const tt_index *ix) {
  int b = 0;
  for (int n = 1; n < ix->N; ++n)
    if (ix->mode[n].mean_row > ix->mode[b].mean_row) b = n;
  return b;
}

static tt_status mttkrp_impl(tt_index *ix, const void *s, const int32_t *s_perm, double w_const,
                             const void *const *d_A, int R, int64_t ldA, tt_dtype fdt, int mode,
                             void *out, int accumulate, hipStream_t st,
                             double *carry = nullptr) {
  const ModeIndex &md = ix->mode[mode];
  StreamCall c = base_call(ix, mode, R, ldA, fdt);
  if (carry) {
    c.carry = carry;
    c.carry_partial = carry + md.nslot * (int64_t)stream_rp(fdt, R);
  } else {
    TT_ST(carry_ws(ix, &c.carry));
  }
  if (!accumulate && md.nrows < md.I)
    TT_LAUNCH(launch_fill(out, md.I * R, dense_of(fdt), 0.0, st), "fill");
  for (int p = 0; p < ix->N; ++p) c.A[p] = d_A[p];
  c.s = s;
  c.s_perm = s_perm;
  c.w_const = w_const;
  c.out = out;
  c.accumulate = accumulate;
  TT_LAUNCH(launch_stream(OP_MTTKRP, c, st), "mttkrp kernel");
  return TT_OK;
}

// Gauss-Newton matvec (Section 2.5): Y_d = lambda2 X_d + J_d^T diag(w) J X for
// every mode d.  The per-nonzero scalar w_e z_e (z = J X, the TTTP-shaped
// Jacobian-vector product) is the same for every block, so it is formed once,
// in the sorted order of the mode with the most rows (whose factor rows miss
// the caches when gathered): that pass also accumulates its own block and
// stores w_e z_e; the other blocks are MTTKRPs of those scalars, read through
// the index's position map, which gather no direction rows at all.
// The streaming passes of one Gauss-Newton product Y += J^T diag(w) J X:
// c[0] the OP_GN pass in zmode's order (it also stores w_e z_e per nonzero
// in zbuf), c[1..N-1] OP_MTTKRP passes of the other modes reading those
// scalars through the position map.
static void gn_passes(tt_index *ix, const void *const *w, double w_const,
                      const int32_t *const *w_perm, const void *const *d_A,
                      const void *const *d_X, int R, int64_t ldA, tt_dtype fdt,
                      void *const *d_Y, double *carry, int zm, const int32_t *zmap, void *zbuf,
                      StreamCall *c) {
  c[0] = base_call(ix, zm, R, ldA, fdt);
  for (int p = 0; p < ix->N; ++p) {
    c[0].A[p] = d_A[p];
    c[0].X[p] = d_X[p];
  }
  c[0].s = w ? w[zm] : nullptr;
  c[0].s_perm = w_perm ? w_perm[zm] : nullptr;
  c[0].w_const = w_const;
  c[0].out = d_Y[zm];
  c[0].accumulate = 1;
  c[0].carry = carry;
  c[0].zout = zbuf;
  int i = 1;
  for (int d = 0; d < ix->N; ++d) {
    if (d == zm) continue;
    c[i] = base_call(ix, d, R, ldA, fdt);
    for (int p = 0; p < ix->N; ++p) c[i].A[p] = d_A[p];
    c[i].s = zbuf;
    c[i].s_perm = zmap + (int64_t)d * ix->m;
    c[i].out = d_Y[d];
    c[i].accumulate = 1;
    c[i].carry = carry;
    c[i].prof_name = "gn_mttkrp";
    ++i;
  }
}

static tt_status gn_matvec_impl(tt_index *ix, const void *const *w, double w_const,
                                const int32_t *const *w_perm, const void *const *d_A,
                                const void *const *d_X, int R, int64_t ldA, tt_dtype fdt,
                                double lambda2, void *const *d_Y, const double *skip,
                                hipStream_t st) {
  double *carry = nullptr;
  TT_ST(carry_ws(ix, &carry));
  const int zm = gn_zmode(ix);
  const int32_t *zmap = nullptr;
  TT_ST(zmap_get(ix, st, &zmap));
  void *zbuf = nullptr;
  TT_ST(ws_get(ix, "gn_z", (size_t)std::max<int64_t>(ix->m, 1) * value_size(fdt), &zbuf));
  for (int d = 0; d < ix->N; ++d) {
    const ModeIndex &md = ix->mode[d];
    TT_LAUNCH(launch_scale_rows(d_Y[d], d_X[d], dense_of(fdt), R, md.I, R, lambda2,
                                dense_of(fdt), st),
              "gn prefill");
  }
  StreamCall c[TT_MAX_ORDER];
  gn_passes(ix, w, w_const, w_perm, d_A, d_X, R, ldA, fdt, d_Y, carry, zm, zmap, zbuf, c);
  for (int i = 0; i < ix->N; ++i) {
    c[i].skip = skip;
    TT_LAUNCH(launch_stream(i == 0 ? OP_GN : OP_MTTKRP, c[i], st),
              i == 0 ? "gn kernel" : "gn mttkrp kernel");
  }
  return TT_OK;
}

static tt_status gradient_impl(tt_index *ix, const void *const *d_A, int R, int64_t ldA,
                               tt_dtype fdt, int loss, double lambda, void *const *d_G,
                               hipStream_t st) {
  double *carry = nullptr;
  TT_ST(carry_ws(ix, &carry));
  for (int d = 0; d < ix->N; ++d) {
    const ModeIndex &md = ix->mode[d];
    TT_LAUNCH(launch_scale_rows(d_G[d], d_A[d], fdt, ldA, md.I, R, 2.0 * lambda,
                                dense_of(fdt), st),
              "gradient prefill");
    StreamCall c = base_call(ix, d, R, ldA, fdt);
    for (int p = 0; p < ix->N; ++p) c.A[p] = d_A[p];
    c.s = md.d_t;
    c.loss = loss;
    c.out = d_G[d];
    c.accumulate = 1;
    c.carry = carry;
    TT_LAUNCH(launch_stream(OP_GRAD, c, st), "gradient kernel");
  }
  return TT_OK;
}

static tt_status objective_impl(tt_index *ix, const void *const *d_A, int R, int64_t ldA,
                                tt_dtype fdt, int loss, double lambda, double *d_f,
                                hipStream_t st) {
  const int mode = best_mode(ix);
  TT_ST(tttp_mode(ix, mode, ix->mode[mode].d_t, nullptr, d_A, R, ldA, fdt, TT_EPI_PHI, loss,
                  nullptr, nullptr, d_f, nullptr, st));
  if (lambda != 0.0) {
    int64_t need = 0;
    for (int n = 0; n < ix->N; ++n) need = std::max(need, sumsq_parts_needed(ix->mode[n].I, R));
    void *p = nullptr;
    TT_ST(ws_get(ix, "sumsq", (size_t)need * 8, &p));
    for (int n = 0; n < ix->N; ++n) {
      int64_t np = 0;
      TT_LAUNCH(launch_sumsq_rows(d_A[n], fdt, ldA, ix->mode[n].I, R, lambda, (double *)p, &np,
                                  st),
                "sumsq");
      TT_LAUNCH(launch_sum_doubles((double *)p, np, d_f, 1, st), "sum");
    }
  }
  return TT_OK;
}

}  // namespace tt

using namespace tt;

extern "C" {

const char *tt_last_error(void) { return g_err.c_str(); }

const char *tt_version(void) { return "libtt 0.1 (gfx950)"; }

tt_status tt_build_index(int order, const int64_t *dims, int64_t nnz,
                         const int32_t *const *d_idx, const void *d_t, tt_dtype vdt,
                         uint32_t flags, hipStream_t stream, tt_index **out) {
  g_err.clear();
  TT_CHECK(out != nullptr, "out is NULL");
  *out = nullptr;
  TT_CHECK(order >= 2 && order <= TT_MAX_ORDER, "order %d outside [2, %d]", order,
           TT_MAX_ORDER);
  TT_CHECK(dims != nullptr && d_idx != nullptr, "dims/d_idx NULL");
  TT_CHECK(nnz >= 0 && nnz < ((int64_t)1 << 31), "nnz %lld outside [0, 2^31)", (long long)nnz);
  TT_CHECK(vdt == TT_F64 || vdt == TT_F32, "value dtype must be TT_F64 or TT_F32");
  TT_CHECK(flags == 0, "flags must be 0");
  for (int n = 0; n < order; ++n) {
    TT_CHECK(dims[n] >= 1 && dims[n] < ((int64_t)1 << 31), "dims[%d] = %lld", n,
             (long long)dims[n]);
    TT_CHECK(nnz == 0 || d_idx[n] != nullptr, "d_idx[%d] is NULL", n);
  }
  if (order != 3) {
    set_error("order %d: the GPU kernels implement order-3 tensors", order);
    return TT_ERR_UNSUPPORTED;
  }
  tt_index *ix = new (std::nothrow) tt_index();
  if (!ix) {
    set_error("host allocation failed");
    return TT_ERR_OOM;
  }
  tt_status st = build_index_impl(order, dims, nnz, d_idx, d_t, vdt, stream, ix);
  if (st != TT_OK) {
    std::string keep = g_err;
    tt_index_destroy(ix);
    g_err = keep;
    return st;
  }
  *out = ix;
  return TT_OK;
}

tt_status tt_index_destroy(tt_index *ix) {
  if (!ix) return TT_OK;
  hipDeviceSynchronize();
  for (void *p : ix->owned) hipFree(p);
  for (int n = 0; n < ix->N; ++n)
    for (void *p : ix->mode[n].part) hipFree(p);
  for (auto &kv : ix->ws)
    if (kv.second.p) hipFree(kv.second.p);
  delete ix;
  return TT_OK;
}

}  // extern "C"

// Workspace of tt_gn_step: PCG vectors (dense dtype, all modes' blocks),
// FP64 scalars and dot-product partials, the preconditioner's row-packed
// Cholesky factors (dense dtype) and, for the Poisson loss, phi'' per mode.
struct GnWs {
  void *x, *r, *z, *p, *q, *sc, *parts, *w, *L;
  void *loop_carry, *loop_bar;  // persistent loop only (else NULL)
};

static tt_status gn_workspace(tt_index *ix, int R, tt_dtype fdt, tt_loss loss, GnWs *ws) {
  const int N = ix->N;
  const size_t dsz = value_size(fdt);
  const int RP = R <= 16 ? 16 : (R <= 32 ? 32 : 64);
  int64_t ntot = 0, Ltot = 0;
  for (int d = 0; d < N; ++d) {
    ntot += ix->mode[d].I * R;
    Ltot += ix->mode[d].I * (int64_t)RP * (RP + 1) / 2;
  }
  TT_ST(ws_get(ix, "pcg_x", ntot * dsz, &ws->x));
  TT_ST(ws_get(ix, "pcg_r", ntot * dsz, &ws->r));
  TT_ST(ws_get(ix, "pcg_z", ntot * dsz, &ws->z));
  TT_ST(ws_get(ix, "pcg_p", ntot * dsz, &ws->p));
  TT_ST(ws_get(ix, "pcg_q", ntot * dsz, &ws->q));
  TT_ST(ws_get(ix, "pcg_sc", 32 * 8, &ws->sc));
  // three sets of dot-product partials (the persistent loop alternates them)
  TT_ST(ws_get(ix, "pcg_parts", (size_t)dot_parts_needed(ntot) * 3 * 8, &ws->parts));
  TT_ST(ws_get(ix, "pcg_L", (size_t)Ltot * (fdt == TT_F64 ? 8 : 4), &ws->L));
  ws->w = nullptr;
  if (loss == TT_LOSS_POISSON_LOG) TT_ST(ws_get(ix, "pcg_w", (size_t)N * ix->m * dsz, &ws->w));
  ws->loop_carry = ws->loop_bar = nullptr;
  if (ix->tune.pcg_wgs != 0 && R <= kPcgMaxRank) {
    TT_ST(ws_get(ix, "pcg_loop_carry", (size_t)pcg_loop_carry_doubles(ix) * 8, &ws->loop_carry));
    TT_ST(ws_get(ix, "pcg_loop_bar", (size_t)pcg_loop_bar_words() * 4, &ws->loop_bar));
  }
  return TT_OK;
}

extern "C" {

tt_status tt_index_reserve(tt_index *ix, int R, tt_dtype fdt, uint32_t flags) {
  g_err.clear();
  TT_ST(check_common(ix, R, R, fdt));
  TT_CHECK((flags & ~(TT_RESERVE_GN | TT_RESERVE_GN_POISSON)) == 0, "bad flags 0x%x", flags);
  double *c = nullptr;
  TT_ST(carry_ws(ix, &c));
  void *p = nullptr;
  TT_ST(ws_get(ix, "tsum", (size_t)std::max<int64_t>(ix->max_nchunk, 1) * 8, &p));
  TT_ST(ws_get(ix, "rhs", (size_t)ix->max_I * R * value_size(fdt), &p));
  const int RP = R <= 16 ? 16 : (R <= 32 ? 32 : 64);
  const int64_t task_bytes = (int64_t)gram_task_elems(RP) * (fdt == TT_F64 ? 8 : 4);
  int64_t wt = 1;
  for (int n = 0; n < ix->N; ++n) {
    const ModeIndex &md = ix->mode[n];
    int64_t w = std::max<int64_t>(kGramBatchBytes / task_bytes, md.max_task_per_row);
    w = std::min<int64_t>(w, std::max<int64_t>(md.ntask, 1));
    wt = std::max(wt, w);
  }
  TT_ST(ws_get(ix, "gram", (size_t)(wt * task_bytes), &p));
  if (fdt != TT_F64) TT_ST(ws_get(ix, "gram_rhs", (size_t)(wt * RP * 8), &p));  // fused ALS rhs
  int64_t need = 0;
  for (int n = 0; n < ix->N; ++n) need = std::max(need, sumsq_parts_needed(ix->mode[n].I, R));
  TT_ST(ws_get(ix, "sumsq", (size_t)need * 8, &p));
  if (flags) {
    GnWs ws;
    TT_ST(gn_workspace(ix, R, fdt,
                       (flags & TT_RESERVE_GN_POISSON) ? TT_LOSS_POISSON_LOG : TT_LOSS_LS, &ws));
    TT_ST(ws_get(ix, "gn_z", (size_t)std::max<int64_t>(ix->m, 1) * value_size(fdt), &p));
    const int32_t *zmap = nullptr;
    TT_ST(zmap_get(ix, nullptr, &zmap));
  }
  return TT_OK;
}

tt_status tt_index_tune(tt_index *ix, const tt_tuning *t, hipStream_t stream) {
  g_err.clear();
  TT_CHECK(ix != nullptr && t != nullptr, "NULL argument");
  TT_CHECK(t->chunk == 512 || t->chunk == 1024 || t->chunk == 2048,
           "chunk %d is not 512, 1024 or 2048", t->chunk);
  TT_CHECK(t->gram_piece >= 1024 && t->gram_piece <= 65536, "gram_piece %d outside [1024, 65536]",
           t->gram_piece);
  TT_CHECK(t->gram_light >= 0 && t->gram_light <= t->gram_piece,
           "gram_light %d outside [0, gram_piece]", t->gram_light);
  TT_CHECK(t->gram_waves == 2 || t->gram_waves == 4 || t->gram_waves == 8,
           "gram_waves %d is not 2, 4 or 8", t->gram_waves);
  TT_CHECK(t->solve_wgs >= 0 && t->solve_wgs <= 64, "solve_wgs %d outside [0, 64]",
           t->solve_wgs);
  TT_CHECK(t->pcg_wgs >= -1 && t->pcg_wgs <= 16, "pcg_wgs %d outside [-1, 16]", t->pcg_wgs);
  TT_CHECK(t->ccd_xcd >= -1 && t->ccd_xcd <= 1, "ccd_xcd %d outside [-1, 1]", t->ccd_xcd);
  TT_CHECK(t->ccd_lds == -1 || t->ccd_lds == 0, "ccd_lds %d is not -1 or 0", t->ccd_lds);
  TT_CHECK(live_graphs() == 0,
           "%d instantiated graph(s) are alive: retuning rebuilds the work partitions "
           "their kernels read; destroy the graphs first", live_graphs());
  ix->tune = *t;
  for (int n = 0; n < ix->N; ++n) TT_ST(build_partitions(ix, n, stream));
  return TT_OK;
}

tt_status tt_index_get_tuning(const tt_index *ix, tt_tuning *out) {
  g_err.clear();
  TT_CHECK(ix != nullptr && out != nullptr, "NULL argument");
  *out = ix->tune;
  return TT_OK;
}

tt_status tt_index_view(const tt_index *ix, int mode, const int64_t **d_ptr,
                        const int32_t **d_perm, const int32_t **d_key,
                        const int32_t **d_rows, int64_t *nrows) {
  TT_CHECK(ix != nullptr, "index is NULL");
  TT_CHECK(mode >= 0 && mode < ix->N, "bad mode %d", mode);
  const ModeIndex &md = ix->mode[mode];
  if (d_ptr) *d_ptr = md.d_ptr;
  if (d_perm) *d_perm = md.d_perm;
  if (d_key) *d_key = md.d_key;
  if (d_rows) *d_rows = md.d_rows;
  if (nrows) *nrows = md.nrows;
  return TT_OK;
}

tt_status tt_index_other(const tt_index *ix, int mode, int other,
                         const int32_t **d_sorted_idx) {
  TT_CHECK(ix != nullptr, "index is NULL");
  TT_CHECK(mode >= 0 && mode < ix->N && other >= 0 && other < ix->N && other != mode,
           "bad modes %d/%d", mode, other);
  TT_CHECK(d_sorted_idx != nullptr, "output NULL");
  *d_sorted_idx = ix->mode[mode].d_oidx[other];
  return TT_OK;
}

tt_status tttp(const tt_index *cix, const void *d_s, int s_order, const void *const *d_A, int R,
               int64_t ldA, tt_dtype fdt, tt_epilogue epi, tt_loss loss, void *d_out,
               int out_order, double *d_sum, hipStream_t stream) {
  g_err.clear();
  tt_index *ix = const_cast<tt_index *>(cix);
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(d_A != nullptr, "d_A is NULL");
  TT_CHECK(epi >= TT_EPI_NONE && epi <= TT_EPI_D2PHI, "bad epilogue %d", (int)epi);
  TT_CHECK(loss == TT_LOSS_LS || loss == TT_LOSS_POISSON_LOG, "bad loss %d", (int)loss);
  TT_CHECK(s_order >= TT_ORDER_COO && s_order < ix->N, "bad s_order %d", s_order);
  TT_CHECK(out_order >= TT_ORDER_COO && out_order < ix->N, "bad out_order %d", out_order);
  int given = 0;
  for (int p = 0; p < ix->N; ++p) given += d_A[p] != nullptr;
  TT_CHECK(given >= 1, "tttp needs at least one factor");
  if (epi != TT_EPI_NONE) {
    TT_CHECK(d_s != nullptr, "loss epilogues need the observed values");
    TT_CHECK(given == ix->N, "loss epilogues need every factor");
  }
  TT_CHECK(d_out != nullptr || d_sum != nullptr || ix->m == 0, "no output");
  // processing order
  int mode;
  if (out_order >= 0) {
    mode = out_order;
  } else if (d_s != nullptr && d_s != TT_INDEX_T && s_order >= 0) {
    mode = s_order;
  } else {
    mode = best_mode(ix);
  }
  const void *s = nullptr;
  const int32_t *s_perm = nullptr;
  TT_ST(resolve_values(ix, d_s, s_order, mode, fdt, &s, &s_perm, "tttp values"));
  const int32_t *out_perm = out_order == TT_ORDER_COO ? ix->mode[mode].d_perm : nullptr;
  if (ix->m == 0) {
    if (d_sum) TT_LAUNCH(launch_fill(d_sum, 1, TT_F64, 0.0, stream), "fill");
    return TT_OK;
  }
  return tttp_mode(ix, mode, s, s_perm, d_A, R, ldA, fdt, epi, loss, d_out, out_perm, d_sum,
                   nullptr, stream);
}

tt_status mttkrp(const tt_index *cix, const void *d_s, int s_order, const void *const *d_A,
                 int R, int64_t ldA, tt_dtype fdt, int mode, void *d_out, int accumulate,
                 hipStream_t stream) {
  g_err.clear();
  return mttkrp_checked(const_cast<tt_index *>(cix), d_s, s_order, d_A, R, ldA, fdt, mode,
                        d_out, accumulate, stream, nullptr);
}

}  // extern "C"

namespace tt {

tt_status mttkrp_checked(tt_index *ix, const void *d_s, int s_order, const void *const *d_A,
                         int R, int64_t ldA, tt_dtype fdt, int mode, void *d_out,
                         int accumulate, hipStream_t stream, double *carry) {
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(mode >= 0 && mode < ix->N, "bad mode %d", mode);
  TT_CHECK(d_A != nullptr && d_out != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p)
    TT_CHECK(p == mode || d_A[p] != nullptr, "factor %d is NULL", p);
  const void *s = nullptr;
  const int32_t *s_perm = nullptr;
  TT_ST(resolve_values(ix, d_s, s_order, mode, fdt, &s, &s_perm, "mttkrp values"));
  return mttkrp_impl(ix, s, s_perm, 1.0, d_A, R, ldA, fdt, mode, d_out, accumulate, stream,
                     carry);
}

}  // namespace tt

extern "C" {

}  // extern "C"

// The ALS right-hand side MTTKRP_n(t) for a Solve Factor call: fused into the
// Gram pass for the FP32 and BF16 forms (one pass over the mode's nonzeros
// computes both), a separate MTTKRP into the index workspace for FP64.
static tt_status als_rhs(tt_index *ix, const void *const *A, int R, int64_t ldA, tt_dtype fdt,
                         int mode, SolveCall *c, hipStream_t stream) {
  if (fdt != TT_F64) {
    c->fused_rhs = 1;
    c->rhs = nullptr;
    return TT_OK;
  }
  void *M = nullptr;
  TT_ST(ws_get(ix, "rhs", (size_t)ix->max_I * R * value_size(fdt), &M));
  TT_ST(solve_workspace(ix, mode, R, fdt, false, nullptr, nullptr));
  TT_ST(mttkrp_impl(ix, ix->mode[mode].d_t, nullptr, 1.0, A, R, ldA, fdt, mode, M, 0, stream));
  c->rhs = M;
  return TT_OK;
}

extern "C" {

tt_status solve_factor(const tt_index *cix, const void *d_w, int w_order, const void *const *d_A,
                       int R, int64_t ldA, tt_dtype fdt, int mode, const void *d_rhs,
                       double lambda, void *d_X, int32_t *d_info, uint32_t flags,
                       hipStream_t stream) {
  g_err.clear();
  tt_index *ix = const_cast<tt_index *>(cix);
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(mode >= 0 && mode < ix->N, "bad mode %d", mode);
  TT_CHECK(d_A != nullptr && d_rhs != nullptr && d_X != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p)
    TT_CHECK(p == mode || d_A[p] != nullptr, "factor %d is NULL", p);
  TT_CHECK((flags & ~TT_SYNC) == 0, "bad flags");
  TT_CHECK(!(flags & TT_SYNC) || d_info != nullptr, "TT_SYNC needs d_info");
  SolveCall c;
  memset(&c, 0, sizeof(c));
  c.ix = ix;
  c.mode = mode;
  c.R = R;
  c.ldA = ldA;
  c.fdt = fdt;
  for (int p = 0; p < ix->N; ++p) c.A[p] = d_A[p];
  TT_ST(resolve_values(ix, d_w, w_order, mode, fdt, &c.w, &c.w_perm, "solve_factor weights"));
  c.w_scale = 1.0;
  c.lambda = lambda;
  c.rhs = d_rhs;
  if (d_rhs == TT_RHS_MTTKRP) {
    // right-hand side = MTTKRP of the observed values with the other factors
    TT_CHECK(ix->has_t, "TT_RHS_MTTKRP needs observed values in the index");
    TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64), "value dtype does not match factor dtype");
    TT_CHECK(d_w == nullptr, "TT_RHS_MTTKRP is defined for unweighted Grams (d_w NULL)");
    TT_ST(als_rhs(ix, c.A, R, ldA, fdt, mode, &c, stream));
  }
  c.X = d_X;
  c.info = d_info;
  TT_ST(run_solve_factor(ix, c, stream));
  if (flags & TT_SYNC) {
    const int64_t I = ix->mode[mode].I;
    std::vector<int32_t> h(I);
    TT_HIP(hipMemcpyAsync(h.data(), d_info, I * 4, hipMemcpyDeviceToHost, stream));
    TT_HIP(hipStreamSynchronize(stream));
    for (int64_t i = 0; i < I; ++i)
      if (h[i] != 0) {
        set_error("row %lld: leading minor of order %d is not positive", (long long)i, h[i]);
        return TT_ERR_NOT_SPD;
      }
  }
  return TT_OK;
}

tt_status solve_factor_model(tt_index *ix, const void *const *d_A, int R, int64_t ldA,
                             tt_dtype fdt, int mode, double lambda, void *d_X, int32_t *d_info,
                             void *d_model, hipStream_t stream) {
  g_err.clear();
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(mode >= 0 && mode < ix->N, "bad mode %d", mode);
  TT_CHECK(d_A != nullptr && d_X != nullptr && d_model != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p) TT_CHECK(d_A[p] != nullptr, "factor %d is NULL", p);
  TT_CHECK(ix->has_t, "the index holds no observed values");
  TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64), "value dtype does not match factor dtype");
  SolveCall c;
  memset(&c, 0, sizeof(c));
  c.ix = ix;
  c.mode = mode;
  c.R = R;
  c.ldA = ldA;
  c.fdt = fdt;
  for (int p = 0; p < ix->N; ++p) c.A[p] = d_A[p];
  c.w_scale = 1.0;
  c.lambda = lambda;
  c.rhs = TT_RHS_MTTKRP;
  if (fdt == TT_F64) {
    // the FP64 form forms its right-hand side by a separate MTTKRP pass, so
    // the model values come from a TTTP pass of their own
    TT_ST(tttp_mode(ix, mode, nullptr, nullptr, d_A, R, ldA, fdt, TT_EPI_NONE, TT_LOSS_LS,
                    d_model, nullptr, nullptr, nullptr, stream));
  } else {
    c.model = d_model;
  }
  TT_ST(als_rhs(ix, c.A, R, ldA, fdt, mode, &c, stream));
  c.X = d_X;
  c.info = d_info;
  return run_solve_factor(ix, c, stream);
}

tt_status gn_matvec(const tt_index *cix, const void *d_w, int w_order, double w_const,
                    const void *const *d_A, const void *const *d_X, int R, int64_t ldA,
                    tt_dtype fdt, double lambda2, void *const *d_Y, hipStream_t stream) {
  g_err.clear();
  tt_index *ix = const_cast<tt_index *>(cix);
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(d_A != nullptr && d_X != nullptr && d_Y != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p)
    TT_CHECK(d_A[p] && d_X[p] && d_Y[p], "block %d is NULL", p);
  const void *w[TT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr};
  const int32_t *wp[TT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr};
  if (d_w != nullptr) {
    TT_CHECK(w_order == TT_ORDER_PER_MODE || w_order == TT_ORDER_COO || d_w == TT_INDEX_T,
             "gn_matvec weights must be per-mode, COO or the index values");
    for (int d = 0; d < ix->N; ++d)
      TT_ST(resolve_values(ix, d_w, w_order, d, fdt, &w[d], &wp[d], "gn_matvec weights"));
  }
  return gn_matvec_impl(ix, d_w ? w : nullptr, w_const, d_w ? wp : nullptr, d_A, d_X, R, ldA,
                        fdt, lambda2, d_Y, nullptr, stream);
}

tt_status newton_matvec(const tt_index *cix, const void *d_w, int w_order, double w_const,
                        const void *d_g, int g_order, const void *const *d_A,
                        const void *const *d_X, int R, int64_t ldA, tt_dtype fdt,
                        double lambda2, void *const *d_Y, hipStream_t stream) {
  g_err.clear();
  tt_index *ix = const_cast<tt_index *>(cix);
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(d_A != nullptr && d_X != nullptr && d_Y != nullptr && d_g != nullptr,
           "NULL argument");
  for (int p = 0; p < ix->N; ++p)
    TT_CHECK(d_A[p] && d_X[p] && d_Y[p], "block %d is NULL", p);
  TT_CHECK(d_g != TT_INDEX_T, "newton_matvec: phi' cannot be the index values");
  TT_CHECK(g_order == TT_ORDER_PER_MODE || g_order == TT_ORDER_COO,
           "newton_matvec phi' must be per-mode or COO");
  const void *w[TT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr};
  const int32_t *wp[TT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr};
  const void *g[TT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr};
  const int32_t *gp[TT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr};
  if (d_w != nullptr) {
    TT_CHECK(w_order == TT_ORDER_PER_MODE || w_order == TT_ORDER_COO || d_w == TT_INDEX_T,
             "newton_matvec weights must be per-mode, COO or the index values");
    for (int d = 0; d < ix->N; ++d)
      TT_ST(resolve_values(ix, d_w, w_order, d, fdt, &w[d], &wp[d], "newton_matvec weights"));
  }
  for (int d = 0; d < ix->N; ++d)
    TT_ST(resolve_values(ix, d_g, g_order, d, fdt, &g[d], &gp[d], "newton_matvec phi'"));
  // the Gauss-Newton part (phi'' terms and lambda2 X) ...
  TT_ST(gn_matvec_impl(ix, d_w ? w : nullptr, w_const, d_w ? wp : nullptr, d_A, d_X, R, ldA,
                       fdt, lambda2, d_Y, nullptr, stream));
  // ... plus, per block, the phi' terms of the off-diagonal Hessian blocks
  double *carry = nullptr;
  TT_ST(carry_ws(ix, &carry));
  for (int d = 0; d < ix->N; ++d) {
    StreamCall c = base_call(ix, d, R, ldA, fdt);
    for (int p = 0; p < ix->N; ++p) {
      c.A[p] = d_A[p];
      c.X[p] = d_X[p];
    }
    c.s = g[d];
    c.s_perm = gp[d];
    c.out = d_Y[d];
    c.accumulate = 1;
    c.carry = carry;
    TT_LAUNCH(launch_stream(OP_NEWTON, c, stream), "newton kernel");
  }
  return TT_OK;
}

tt_status tt_gradient(const tt_index *cix, const void *const *d_A, int R, int64_t ldA,
                      tt_dtype fdt, tt_loss loss, double lambda, void *const *d_G,
                      hipStream_t stream) {
  g_err.clear();
  tt_index *ix = const_cast<tt_index *>(cix);
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(ix->has_t, "the index holds no observed values");
  TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64), "value dtype does not match factor dtype");
  TT_CHECK(loss == TT_LOSS_LS || loss == TT_LOSS_POISSON_LOG, "bad loss %d", (int)loss);
  TT_CHECK(d_A != nullptr && d_G != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p) TT_CHECK(d_A[p] && d_G[p], "block %d is NULL", p);
  return gradient_impl(ix, d_A, R, ldA, fdt, loss, lambda, d_G, stream);
}

tt_status tt_objective(const tt_index *cix, const void *const *d_A, int R, int64_t ldA,
                       tt_dtype fdt, tt_loss loss, double lambda, double *d_f,
                       hipStream_t stream) {
  g_err.clear();
  tt_index *ix = const_cast<tt_index *>(cix);
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(ix->has_t, "the index holds no observed values");
  TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64), "value dtype does not match factor dtype");
  TT_CHECK(loss == TT_LOSS_LS || loss == TT_LOSS_POISSON_LOG, "bad loss %d", (int)loss);
  TT_CHECK(d_A != nullptr && d_f != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p) TT_CHECK(d_A[p], "factor %d is NULL", p);
  return objective_impl(ix, d_A, R, ldA, fdt, loss, lambda, d_f, stream);
}

tt_status tt_als_sweep(tt_index *ix, void *const *d_A, int R, int64_t ldA, tt_dtype fdt,
                       double lambda, int32_t *d_info, hipStream_t stream) {
  g_err.clear();
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(ix->has_t, "the index holds no observed values");
  TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64), "value dtype does not match factor dtype");
  TT_CHECK(d_A != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p) TT_CHECK(d_A[p], "factor %d is NULL", p);
  const void *A[TT_MAX_ORDER] = {d_A[0], d_A[1], d_A[2], nullptr};
  int64_t off = 0;
  for (int n = 0; n < ix->N; ++n) {
    SolveCall c;
    memset(&c, 0, sizeof(c));
    c.ix = ix;
    c.mode = n;
    c.R = R;
    c.ldA = ldA;
    c.fdt = fdt;
    for (int p = 0; p < ix->N; ++p) c.A[p] = A[p];
    c.w_scale = 1.0;
    c.lambda = lambda;
    TT_ST(als_rhs(ix, A, R, ldA, fdt, n, &c, stream));
    c.X = d_A[n];
    c.info = d_info ? d_info + off : nullptr;
    TT_ST(run_solve_factor(ix, c, stream));
    off += ix->mode[n].I;
  }
  return TT_OK;
}

tt_status tt_gn_step(tt_index *ix, void *const *d_A, int R, int64_t ldA, tt_dtype fdt,
                     tt_loss loss, double lambda, double tol, int kmax, double *d_stats,
                     hipStream_t st) {
  g_err.clear();
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(ix->has_t, "the index holds no observed values");
  TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64), "value dtype does not match factor dtype");
  TT_CHECK(loss == TT_LOSS_LS || loss == TT_LOSS_POISSON_LOG, "bad loss %d", (int)loss);
  TT_CHECK(kmax >= 0, "kmax < 0");
  TT_CHECK(d_A != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p) TT_CHECK(d_A[p], "factor %d is NULL", p);
  const int N = ix->N;
  const tt_dtype dn = dense_of(fdt);
  const size_t dsz = value_size(fdt);
  const int RP = R <= 16 ? 16 : (R <= 32 ? 32 : 64);
  int64_t off[TT_MAX_ORDER + 1] = {0};
  for (int d = 0; d < N; ++d) off[d + 1] = off[d] + ix->mode[d].I * R;
  const int64_t ntot = off[N];
  // workspace
  GnWs ws;
  TT_ST(gn_workspace(ix, R, fdt, loss, &ws));
  void *vx = ws.x, *vr = ws.r, *vz = ws.z, *vp = ws.p, *vq = ws.q, *vsc = ws.sc,
       *vparts = ws.parts, *vw = ws.w, *vL = ws.L;
  const size_t lsz = fdt == TT_F64 ? 8 : 4;  // preconditioner factors: dense dtype
  char *X = (char *)vx, *Rv = (char *)vr, *Z = (char *)vz, *P = (char *)vp, *Q = (char *)vq;
  double *sc = (double *)vsc, *parts = (double *)vparts;
  char *L = (char *)vL;
  const void *A[TT_MAX_ORDER] = {d_A[0], d_A[1], d_A[2], nullptr};
  auto blk = [&](char *base, int d) -> void * { return base + off[d] * dsz; };
  void *Lb[TT_MAX_ORDER];
  {
    int64_t lo = 0;
    for (int d = 0; d < N; ++d) {
      Lb[d] = L + lo * lsz;
      lo += ix->mode[d].I * (int64_t)RP * (RP + 1) / 2;
    }
  }
  // objective before the step (slot 10)
  TT_ST(objective_impl(ix, A, R, ldA, fdt, loss, lambda, sc + 10, st));
  // weights phi'' in each mode's order
  const void *w[TT_MAX_ORDER] = {nullptr, nullptr, nullptr, nullptr};
  double w_const = 2.0;
  if (loss == TT_LOSS_POISSON_LOG) {
    for (int d = 0; d < N; ++d) {
      w[d] = (char *)vw + (size_t)d * ix->m * dsz;
      TT_ST(tttp_mode(ix, d, ix->mode[d].d_t, nullptr, A, R, ldA, fdt, TT_EPI_D2PHI, loss,
                      (void *)w[d], nullptr, nullptr, nullptr, st));
    }
  }
  // b = -grad f ; x = 0 ; r = b
  void *G[TT_MAX_ORDER];
  for (int d = 0; d < N; ++d) G[d] = blk(Q, d);
  TT_ST(gradient_impl(ix, A, R, ldA, fdt, loss, lambda, G, st));
  TT_LAUNCH(launch_scale_rows(Rv, Q, dn, R, ntot / R, R, -1.0, dn, st), "negate");
  TT_LAUNCH(launch_fill(X, ntot, dn, 0.0, st), "fill");
  // block-diagonal preconditioner: factor (G_phi'' + 2 lambda I) per mode
  for (int d = 0; d < N; ++d) {
    SolveCall c;
    memset(&c, 0, sizeof(c));
    c.ix = ix;
    c.mode = d;
    c.R = R;
    c.ldA = ldA;
    c.fdt = fdt;
    for (int p = 0; p < N; ++p) c.A[p] = A[p];
    c.w = w[d];
    c.w_scale = w[d] ? 1.0 : w_const;
    c.lambda = 2.0 * lambda;
    c.Lstore = Lb[d];
    c.factor_only = 1;
    TT_ST(run_solve_factor(ix, c, st));
  }
  auto precond = [&](const double *skip) -> tt_status {
    for (int d = 0; d < N; ++d)
      TT_LAUNCH(launch_apply_factor(ix, d, R, fdt, Lb[d], blk(Rv, d), blk(Z, d), skip, st),
                "precond");
    return TT_OK;
  };
  auto dot = [&](const void *a, const void *b, int slot) -> tt_status {
    int64_t np = 0;
    TT_LAUNCH(launch_dot_parts(a, b, ntot, dn, parts, &np, st), "dot");
    TT_LAUNCH(launch_sum_doubles(parts, np, sc + slot, 0, st), "dot sum");
    return TT_OK;
  };
  const double *done = sc + 5;
  TT_ST(precond(nullptr));
  TT_ST(dot(Rv, Z, 0));
  TT_ST(dot(Rv, Rv, 2));
  TT_LAUNCH(launch_pcg_scalar(sc, 0, tol, st), "pcg");
  TT_LAUNCH(launch_scale_rows(P, Z, dn, R, ntot / R, R, 1.0, dn, st), "copy");
  void *Pb[TT_MAX_ORDER], *Qb[TT_MAX_ORDER];
  const void *Pc[TT_MAX_ORDER];
  for (int d = 0; d < N; ++d) {
    Pb[d] = blk(P, d);
    Pc[d] = Pb[d];
    Qb[d] = blk(Q, d);
  }
  // all iterations in one persistent kernel (same arithmetic), if chosen
  bool persist = ws.loop_bar != nullptr && kmax > 0 &&
                 kmax <= pcg_loop_max_iters(ix, ix->tune.pcg_wgs);
  PcgLoopCall pc;
  memset(&pc, 0, sizeof(pc));
  if (persist) {
    const int32_t *zmap = nullptr;
    TT_ST(zmap_get(ix, st, &zmap));
    void *zbuf = nullptr;
    TT_ST(ws_get(ix, "gn_z", (size_t)std::max<int64_t>(ix->m, 1) * value_size(fdt), &zbuf));
    gn_passes(ix, loss == TT_LOSS_POISSON_LOG ? w : nullptr, w_const, nullptr, A, Pc, R, ldA,
              fdt, Qb, nullptr, gn_zmode(ix), zmap, zbuf, pc.pass);
    pc.wgs_per_cu = ix->tune.pcg_wgs > 0 ? ix->tune.pcg_wgs : 2;
    if (ix->tune.pcg_wgs < 0) persist = pcg_loop_fits(pc);
  }
  if (persist) {
    pc.carry = (double *)ws.loop_carry;
    for (int d = 0; d < N; ++d) pc.L[d] = Lb[d];
    pc.x = X;
    pc.r = Rv;
    pc.z = Z;
    pc.p = P;
    pc.q = Q;
    pc.lambda2 = 2.0 * lambda;
    pc.parts = parts;
    pc.sc = sc;
    pc.tol = tol;
    pc.kmax = kmax;
    pc.bar = (unsigned *)ws.loop_bar;
    TT_LAUNCH(launch_pcg_loop(pc, st), "pcg loop");
  }
  for (int k = 0; k < (persist ? 0 : kmax); ++k) {
    TT_ST(gn_matvec_impl(ix, loss == TT_LOSS_POISSON_LOG ? w : nullptr, w_const, nullptr, A, Pc,
                         R, ldA, fdt, 2.0 * lambda, Qb, done, st));
    TT_ST(dot(P, Q, 1));
    TT_LAUNCH(launch_pcg_scalar(sc, 1, tol, st), "pcg");
    TT_LAUNCH(launch_axpy2(X, P, Rv, Q, ntot, dn, sc, 0, st), "axpy");
    TT_ST(dot(Rv, Rv, 2));
    TT_LAUNCH(launch_pcg_scalar(sc, 2, tol, st), "pcg");
    TT_ST(precond(done));
    TT_ST(dot(Rv, Z, 4));
    TT_LAUNCH(launch_pcg_scalar(sc, 3, tol, st), "pcg");
    TT_LAUNCH(launch_xpby(P, Z, ntot, dn, sc, 0, st), "xpby");
  }
  for (int d = 0; d < N; ++d)
    TT_LAUNCH(launch_add_to_factor(d_A[d], fdt, ldA, ix->mode[d].I, R, blk(X, d), st,
                                   persist ? sc + kPcgAbortSlot : nullptr),
              "step");
  if (d_stats) TT_LAUNCH(launch_pcg_stats(sc, sc + 10, d_stats, st), "stats");
  return TT_OK;
}

tt_status tt_ccd_sweep(tt_index *ix, void *const *d_A, int R, int64_t ldA, tt_dtype fdt,
                       double lambda, int32_t *d_info, hipStream_t st) {
  g_err.clear();
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(ix->has_t, "the index holds no observed values");
  TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64), "value dtype does not match factor dtype");
  TT_CHECK(d_A != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p) TT_CHECK(d_A[p], "factor %d is NULL", p);
  const int N = ix->N;
  const size_t vsz = value_size(fdt);
  const void *A[TT_MAX_ORDER] = {d_A[0], d_A[1], d_A[2], nullptr};
  // workspace: the residual rho = t - model in every mode's sorted order,
  // one record per factor row (columns r - 1 and r, dense dtype), and the
  // per-task partial sums of a mode pass
  void *rho[TT_MAX_ORDER] = {}, *recs[TT_MAX_ORDER] = {};
  void *vrho = nullptr, *vrec = nullptr, *vpart = nullptr;
  const int64_t m1 = std::max<int64_t>(ix->m, 1);
  // each mode's stream layout (regrouped per XCD bucket, or the sorted one)
  const CcdLayout *lay[TT_MAX_ORDER] = {};
  for (int n = 0; n < N; ++n) TT_ST(ccd_layout_get(ix, n, vsz, st, &lay[n]));
  int64_t max_task = 1;
  for (int n = 0; n < N; ++n)
    max_task = std::max(max_task, lay[n] ? lay[n]->ntask : ix->mode[n].ntask);
  TT_ST(ws_get(ix, "ccd_rho", (size_t)N * m1 * vsz, &vrho));
  TT_ST(ws_get(ix, "ccd_recs", (size_t)4 * (ix->sum_I + N) * vsz, &vrec));
  TT_ST(ws_get(ix, "ccd_part", (size_t)2 * max_task * 8, &vpart));
  {
    char *c = (char *)vrec;  // each mode's records, 4 vsz each
    for (int n = 0; n < N; ++n) {
      rho[n] = (char *)vrho + (size_t)n * m1 * vsz;
      recs[n] = c;
      c += (size_t)(ix->mode[n].I + 1) * 4 * vsz;
    }
  }
  for (int n = 0; n < N && ix->m > 0; ++n)
    TT_ST(tttp_mode(ix, n, ix->mode[n].d_t, nullptr, A, R, ldA, fdt, TT_EPI_RESID, TT_LOSS_LS,
                    rho[n], lay[n] ? lay[n]->d_inv : nullptr, nullptr, nullptr, st));
  for (int r = 0; r < R; ++r)
    TT_LAUNCH(launch_ccd_column(ix, r, d_A, ldA, fdt, lambda, rho, recs, lay, (double *)vpart,
                                d_info, st),
              "ccd column");
  return TT_OK;
}

tt_status tt_gam_sweep(tt_index *ix, void *const *d_A, int R, int64_t ldA, tt_dtype fdt,
                       tt_loss loss, double lambda, double tol, int max_inner,
                       int32_t *d_info, int32_t *h_iters, hipStream_t st) {
  g_err.clear();
  TT_ST(check_common(ix, R, ldA, fdt));
  TT_CHECK(ix->has_t, "the index holds no observed values");
  TT_CHECK((ix->vdt == TT_F64) == (fdt == TT_F64), "value dtype does not match factor dtype");
  TT_CHECK(loss == TT_LOSS_LS || loss == TT_LOSS_POISSON_LOG, "bad loss %d", (int)loss);
  TT_CHECK(max_inner >= 0, "max_inner < 0");
  TT_CHECK(d_A != nullptr, "NULL argument");
  for (int p = 0; p < ix->N; ++p) TT_CHECK(d_A[p], "factor %d is NULL", p);
  const int N = ix->N;
  const tt_dtype dn = dense_of(fdt);
  const void *A[TT_MAX_ORDER] = {d_A[0], d_A[1], d_A[2], nullptr};
  // workspace: -gradient rows (dense), the Newton step (factor dtype, ldA),
  // phi'' in one mode's order (Poisson), step and factor norms
  void *vg = nullptr, *vd = nullptr, *vw = nullptr, *vparts = nullptr, *vsc = nullptr;
  const size_t fsz = fdt == TT_F64 ? 8 : (fdt == TT_F32 ? 4 : 2);
  TT_ST(ws_get(ix, "gam_d", (size_t)ix->max_I * ldA * fsz, &vd));
  int64_t need = 0;
  for (int n = 0; n < N; ++n) need = std::max(need, sumsq_parts_needed(ix->mode[n].I, R));
  TT_ST(ws_get(ix, "sumsq", (size_t)need * 8, &vparts));
  TT_ST(ws_get(ix, "gam_sc", (3 + TT_MAX_ORDER) * 8, &vsc));
  double *carry = nullptr;
  if (fdt == TT_F64) {
    // the FP64 form's separate gradient pass: row gradients, phi'' per
    // nonzero (Poisson), carries of its segmented reduction
    TT_ST(ws_get(ix, "gam_g", (size_t)ix->max_I * R * value_size(fdt), &vg));
    if (loss == TT_LOSS_POISSON_LOG)
      TT_ST(ws_get(ix, "gam_w", (size_t)std::max<int64_t>(ix->m, 1) * value_size(fdt), &vw));
    TT_ST(carry_ws(ix, &carry));
  }
  double *sc = (double *)vsc, *parts = (double *)vparts;
  if (fdt != TT_F64) {
    // FP32 and BF16 forms: the Newton system of a mode is formed in one
    // pass per iteration -- the Gram pass evaluates the model value, phi'
    // and phi'' of each nonzero (no separate gradient pass) -- and the stop
    // rule is a device flag: once a mode has converged, its remaining
    // iterations' launches return at once.  sc: [||D||^2, ||A_n||^2, flag,
    // iterations of mode 0 .. N-1].
    for (int n = 0; n < N; ++n) TT_ST(solve_workspace(ix, n, R, fdt, true, nullptr, nullptr));
    TT_LAUNCH(launch_fill(sc, 3 + N, TT_F64, 0.0, st), "gam counters");
    int64_t off = 0;
    for (int n = 0; n < N; ++n) {
      const ModeIndex &md = ix->mode[n];
      TT_LAUNCH(launch_fill(sc + 2, 1, TT_F64, 0.0, st), "gam flag");
      for (int k = 0; k < max_inner; ++k) {
        SolveCall c;
        memset(&c, 0, sizeof(c));
        c.ix = ix;
        c.mode = n;
        c.R = R;
        c.ldA = ldA;
        c.fdt = fdt;
        for (int p = 0; p < N; ++p) c.A[p] = A[p];
        c.w_scale = 1.0;
        c.lambda = 2.0 * lambda;
        c.fused_rhs = 1;
        c.newton = 1;
        c.loss = loss;
        c.own_coef = 2.0 * lambda;
        c.X = vd;
        c.info = d_info ? d_info + off : nullptr;
        c.skip = sc + 2;
        TT_ST(run_solve_factor(ix, c, st));
        TT_LAUNCH(launch_add_rows(d_A[n], ldA, vd, ldA, fdt, md.I, R, st, sc + 2), "gam step");
        const bool check = tol > 0.0 && k + 1 < max_inner;
        if (check) {
          int64_t np = 0;
          TT_LAUNCH(launch_sumsq_rows(vd, fdt, ldA, md.I, R, 1.0, parts, &np, st, sc + 2),
                    "gam norm");
          TT_LAUNCH(launch_sum_doubles(parts, np, sc, 0, st, sc + 2), "gam norm");
          TT_LAUNCH(launch_sumsq_rows(d_A[n], fdt, ldA, md.I, R, 1.0, parts, &np, st, sc + 2),
                    "gam norm");
          TT_LAUNCH(launch_sum_doubles(parts, np, sc + 1, 0, st, sc + 2), "gam norm");
        }
        TT_LAUNCH(launch_gam_flag(sc, tol, 3 + n, check ? 1 : 0, st), "gam flag");
      }
      off += md.I;
    }
    if (h_iters) {
      double h[TT_MAX_ORDER] = {0, 0, 0, 0};
      TT_LAUNCH(hipMemcpyAsync(h, sc + 3, N * sizeof(double), hipMemcpyDeviceToHost, st),
                "gam iterations copy");
      TT_LAUNCH(hipStreamSynchronize(st), "gam iterations sync");
      for (int n = 0; n < N; ++n) h_iters[n] = (int32_t)h[n];
    }
    return TT_OK;
  }
  int64_t off = 0;
  for (int n = 0; n < N; ++n) {
    const ModeIndex &md = ix->mode[n];
    int k = 0;
    while (k < max_inner) {
      // -(MTTKRP_n(phi') + 2 lambda A_n): the row gradients (Table 1), negated;
      // the same pass stores phi'' in mode n's order (the constant 2 for LS)
      TT_LAUNCH(launch_scale_rows(vg, d_A[n], fdt, ldA, md.I, R, 2.0 * lambda, dn, st),
                "gam prefill");
      StreamCall c = base_call(ix, n, R, ldA, fdt);
      for (int p = 0; p < N; ++p) c.A[p] = A[p];
      c.s = md.d_t;
      c.loss = loss;
      c.out = vg;
      c.accumulate = 1;
      c.carry = carry;
      c.zout = vw;
      TT_LAUNCH(launch_stream(OP_GRAD, c, st), "gam gradient kernel");
      TT_LAUNCH(launch_scale_rows(vg, vg, dn, R, md.I, R, -1.0, dn, st), "gam negate");
      // per row: (G_phi'' + 2 lambda I) d_i = -g_i  (Solve Factor)
      SolveCall sc_call;
      memset(&sc_call, 0, sizeof(sc_call));
      sc_call.ix = ix;
      sc_call.mode = n;
      sc_call.R = R;
      sc_call.ldA = ldA;
      sc_call.fdt = fdt;
      for (int p = 0; p < N; ++p) sc_call.A[p] = A[p];
      sc_call.w = vw;
      sc_call.w_scale = vw ? 1.0 : 2.0;
      sc_call.lambda = 2.0 * lambda;
      sc_call.rhs = vg;
      sc_call.X = vd;
      sc_call.info = d_info ? d_info + off : nullptr;
      TT_ST(run_solve_factor(ix, sc_call, st));
      TT_LAUNCH(launch_add_rows(d_A[n], ldA, vd, ldA, fdt, md.I, R, st), "gam step");
      ++k;
      if (tol > 0.0 && k < max_inner) {
        int64_t np = 0;
        TT_LAUNCH(launch_sumsq_rows(vd, fdt, ldA, md.I, R, 1.0, parts, &np, st), "gam norm");
        TT_LAUNCH(launch_sum_doubles(parts, np, sc, 0, st), "gam norm");
        TT_LAUNCH(launch_sumsq_rows(d_A[n], fdt, ldA, md.I, R, 1.0, parts, &np, st),
                  "gam norm");
        TT_LAUNCH(launch_sum_doubles(parts, np, sc + 1, 0, st), "gam norm");
        double h[2] = {0.0, 0.0};
        TT_LAUNCH(hipMemcpyAsync(h, sc, sizeof(h), hipMemcpyDeviceToHost, st), "gam norm copy");
        TT_LAUNCH(hipStreamSynchronize(st), "gam norm sync");
        if (std::sqrt(h[0]) <= tol * std::sqrt(h[1])) break;
      }
    }
    if (h_iters) h_iters[n] = k;
    off += md.I;
  }
  return TT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Graph capture
// ---------------------------------------------------------------------------
struct tt_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

tt_status tt_graph_begin(hipStream_t stream) {
  g_err.clear();
  TT_CHECK(stream != nullptr, "graph capture needs a non-null stream");
  TT_CHECK(!tt::prof_on(), "turn the kernel profiler off before capturing");
  TT_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  return TT_OK;
}

tt_status tt_graph_end(hipStream_t stream, tt_graph **out) {
  g_err.clear();
  TT_CHECK(stream != nullptr && out != nullptr, "NULL argument");
  *out = nullptr;
  hipGraph_t g = nullptr;
  TT_HIP(hipStreamEndCapture(stream, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return hip_fail(e, "graph instantiate");
  }
  *out = new tt_graph{g, ex};
  g_live_graphs.fetch_add(1);
  return TT_OK;
}

tt_status tt_graph_launch(tt_graph *graph, hipStream_t stream) {
  g_err.clear();
  TT_CHECK(graph != nullptr, "graph is NULL");
  TT_HIP(hipGraphLaunch(graph->exec, stream));
  return TT_OK;
}

tt_status tt_graph_destroy(tt_graph *graph) {
  g_err.clear();
  if (!graph) return TT_OK;
  hipGraphExecDestroy(graph->exec);
  hipGraphDestroy(graph->graph);
  delete graph;
  g_live_graphs.fetch_sub(1);
  return TT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Kernel profiler
// ---------------------------------------------------------------------------
namespace tt {

struct ProfRec {
  const char *name;
  hipEvent_t a, b;
  double bytes, flops;
};

static struct {
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
} g_prof;

bool prof_on() { return g_prof.on; }

static hipEvent_t prof_event() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

ProfScope::ProfScope(const char *name, hipStream_t s, double bytes, double flops) {
  if (!g_prof.on) return;
  ProfRec r{name, prof_event(), prof_event(), bytes, flops};
  if (!r.a || !r.b) return;
  hipEventRecord(r.a, s);
  slot = (int)g_prof.recs.size();
  stream = s;
  g_prof.recs.push_back(r);
}

ProfScope::~ProfScope() {
  if (slot >= 0 && slot < (int)g_prof.recs.size()) hipEventRecord(g_prof.recs[slot].b, stream);
}

}  // namespace tt

extern "C" {

tt_status tt_profile_enable(int on) {
  g_err.clear();
  if (on) {
    hipDeviceSynchronize();
    for (auto &r : g_prof.recs) {
      g_prof.pool.push_back(r.a);
      g_prof.pool.push_back(r.b);
    }
    g_prof.recs.clear();
  }
  g_prof.on = on != 0;
  return TT_OK;
}

tt_status tt_profile_report(char *buf, int64_t cap, int64_t *needed) {
  g_err.clear();
  struct Agg {
    int64_t n = 0;
    double ms = 0, bytes = 0, flops = 0;
  };
  std::vector<std::pair<std::string, Agg>> agg;
  for (auto &r : g_prof.recs) {
    float ms = 0.f;
    TT_HIP(hipEventSynchronize(r.b));
    TT_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    auto it = std::find_if(agg.begin(), agg.end(),
                           [&](const std::pair<std::string, Agg> &x) { return x.first == r.name; });
    if (it == agg.end()) {
      agg.push_back({r.name, Agg()});
      it = agg.end() - 1;
    }
    it->second.n += 1;
    it->second.ms += ms;
    it->second.bytes += r.bytes;
    it->second.flops += r.flops;
  }
  std::string out = "{";
  char tmp[512];
  for (size_t i = 0; i < agg.size(); ++i) {
    snprintf(tmp, sizeof(tmp),
             "%s\"%s\": {\"launches\": %lld, \"ms\": %.6f, \"bytes\": %.6e, \"flops\": %.6e}",
             i ? ", " : "", agg[i].first.c_str(), (long long)agg[i].second.n, agg[i].second.ms,
             agg[i].second.bytes, agg[i].second.flops);
    out += tmp;
  }
  out += "}";
  if (needed) *needed = (int64_t)out.size() + 1;
  if (buf && cap > 0) {
    int64_t n = std::min<int64_t>(cap - 1, (int64_t)out.size());
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return TT_OK;
}

}  // extern "C"
