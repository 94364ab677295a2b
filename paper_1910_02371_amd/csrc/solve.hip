// Solve Factor (Section 3.4): per-row Gram matrices
//     G^(i) = sum_{e in row i} w_e h_e h_e^T,   h_e = Hadamard_{p != n} A_p[i_p(e)]
// built on matrix cores, then (G^(i) + lambda I) x_i = M_i solved per row by
// an FP64 Cholesky factorization and two triangular solves (the SPD solve of
// Section 3.4; the normal equations of Section 2.2).
//
// Gram: one wave per task (a piece of <= gram_piece nonzeros of one row).
// With H the task's rows h_e stacked, G = H^T diag(w) H is a K x R by K x R
// contraction over the nonzeros, mapped onto MFMA with the nonzero index as
// the reduction dimension: A-operand = h (R on the M index), B-operand = w h.
//   FP32/BF16 storage: v_mfma_f32_16x16x32_bf16 tiles over steps of 32
//                      nonzeros, each lane reading RP / 16 consecutive
//                      columns of a row (RP (RP / 16 + 1) / 32 tiles cover
//                      the upper triangle).  Each FP32 product h is split
//                      exactly into bf16 parts (three for FP32 factors; two
//                      for BF16 factors, whose products have 16 significant
//                      bits) and the parts' products accumulate in FP32.
//   FP64 storage: v_mfma_f64_16x16x4f64 tiles (lower triangle only).
// Each task writes its G to a batch workspace in the lower-tile layout: the
// NB (NB + 1) / 2 lower 16 x 16 tiles (NB = RP / 16), tile (I, J) at
// q = I (I + 1) / 2 + J, each row-major, which is the accumulator layout of
// v_mfma_f64_16x16x4f64 (lane l, register v: row 4 v + l / 16, column
// l % 16), so the solve kernel loads its tiles with coalesced reads.  Rows
// with several tasks are summed in FP64 in task order (deterministic).
//
// Solve: one wave per row.  S = G + lambda I stays in FP64 matrix-core
// accumulator tiles and a blocked right-looking Cholesky runs over panels
// of four columns: the panel is factored on the lanes (lane i = row i), and
// the trailing update S -= L_p L_p^T runs on v_mfma_f64_16x16x4f64.  The
// factor is collected row-packed in LDS for the triangular solves.
// Non-positive pivots follow LAPACK potrf: info = order of the failing
// leading minor, x = 0.
#include "solve_impl.h"

namespace tt {

template <class GT, class XT, class MT>
static hipError_t launch_solve_rp(int RP, SolveDev d, int64_t nrow, hipStream_t s) {
  if (nrow <= 0) return hipSuccess;
  d.nrow = nrow;
  dim3 g(solve_grid(d)), b(64);
  const bool pers = g.x < (unsigned)nrow;
  switch (RP) {
    case 16:
      if (pers) k_solve_rows<GT, XT, MT, 16, true><<<g, b, 0, s>>>(d);
      else k_solve_rows<GT, XT, MT, 16, false><<<g, b, 0, s>>>(d);
      break;
    case 32:
      if (pers) k_solve_rows<GT, XT, MT, 32, true><<<g, b, 0, s>>>(d);
      else k_solve_rows<GT, XT, MT, 32, false><<<g, b, 0, s>>>(d);
      break;
    default:
      if (pers) k_solve_rows<GT, XT, MT, 64, true><<<g, b, 0, s>>>(d);
      else k_solve_rows<GT, XT, MT, 64, false><<<g, b, 0, s>>>(d);
      break;
  }
  return hipGetLastError();
}

template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS>
static void launch_gram_heavy_rp(const GramDev &d, const int32_t *heavy, int64_t nheavy,
                                 double bytes, double flops, hipStream_t s) {
  if (nheavy <= 0) return;
  ProfScope ps("gram_heavy", s, bytes, flops);
  const dim3 g((unsigned)nheavy);
  auto launch = [&](auto mod) {
    constexpr bool MOD = decltype(mod)::value;
    switch (d.waves) {
      case 2: k_gram_f32_heavy<TR, RP, VEC, WEIGHTED, RHS, 2, MOD><<<g, dim3(128), 0, s>>>(d, heavy, nheavy); break;
      case 8: k_gram_f32_heavy<TR, RP, VEC, WEIGHTED, RHS, 8, MOD><<<g, dim3(512), 0, s>>>(d, heavy, nheavy); break;
      default: k_gram_f32_heavy<TR, RP, VEC, WEIGHTED, RHS, 4, MOD><<<g, dim3(256), 0, s>>>(d, heavy, nheavy); break;
    }
  };
  if constexpr (RHS && !WEIGHTED) {
    if (d.model != nullptr) {
      launch(std::true_type{});
      return;
    }
  }
  launch(std::false_type{});
}

template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS>
static void launch_gram_f32_rp(GramDev d, const GramLists &gl, hipStream_t s) {
  if (gl.nlight > 0) {
    ProfScope ps("gram_light", s, gl.light_bytes, gl.light_flops);
    const dim3 g((unsigned)((gl.nlight + 3) / 4));
    bool mod = false;
    if constexpr (RHS && !WEIGHTED) {
      mod = d.model != nullptr;
      if (mod) k_gram_f32<TR, RP, VEC, WEIGHTED, RHS, true><<<g, dim3(256), 0, s>>>(d, gl.light, gl.nlight);
    }
    if (!mod) k_gram_f32<TR, RP, VEC, WEIGHTED, RHS, false><<<g, dim3(256), 0, s>>>(d, gl.light, gl.nlight);
  }
  launch_gram_heavy_rp<TR, RP, VEC, WEIGHTED, RHS>(d, gl.heavy, gl.nheavy, gl.heavy_bytes,
                                                   gl.heavy_flops, s);
}

// The Gram kernels (workspace output) of one batch.
template <class TR, int RP>
static void launch_gram_f32_vec(const GramDev &d, const GramLists &gl, hipStream_t s) {
  gram_form<TR, RP>(d, [&](auto v, auto w, auto h) {
    launch_gram_f32_rp<TR, RP, decltype(v)::value, decltype(w)::value, decltype(h)::value>(
        d, gl, s);
  });
}

// Gram of one batch of tasks [task_base, task_end): light tasks one wave
// each, heavy tasks (the `heavy` slice) one workgroup each, then the
// pre-reduction of rows with many tasks (the `multi` slice).
struct GramWork {
  double light_nnz, heavy_nnz, light_tasks, reduce_tasks;
};

static hipError_t launch_gram(tt_dtype fdt, int RP, const GramDev &d, const GramLists &gl,
                              const int32_t *multi, int64_t nmulti,
                              const int32_t *row_task, const GramWork &wk, hipStream_t s) {
  const int64_t n = d.task_end - d.task_base;
  if (n <= 0) return hipSuccess;
  const int64_t nheavy = gl.nheavy;
  dim3 g((unsigned)((n + 3) / 4)), b(256);
  const double R = d.R, fb = fdt == TT_F64 ? 8 : (fdt == TT_F32 ? 4 : 2);
  const double gs = fdt == TT_F64 ? 8 : 4,
               pernz = 8 + (d.w ? gs : 0) + (d.M ? 4 : 0) + (d.model ? 4 : 0) + 2 * R * fb;
  const double tile = (double)gram_task_elems(RP) * gs;
  if (fdt == TT_F64) {
    ProfScope ps("gram_light", s, (wk.light_nnz + wk.heavy_nnz) * pernz + wk.light_tasks * tile,
                 (wk.light_nnz + wk.heavy_nnz) * R * (R + 1));
    switch (RP) {
      case 16: k_gram_f64<16><<<g, b, 0, s>>>(d); break;
      case 32: k_gram_f64<32><<<g, b, 0, s>>>(d); break;
      default: k_gram_f64<64><<<g, b, 0, s>>>(d); break;
    }
  } else {
    GramLists g2 = gl;
    g2.light_bytes = wk.light_nnz * pernz + wk.light_tasks * tile;
    g2.light_flops = wk.light_nnz * R * (R + 1);
    g2.heavy_bytes = wk.heavy_nnz * pernz + (double)nheavy * tile;
    g2.heavy_flops = wk.heavy_nnz * R * (R + 1);
    if (fdt == TT_F32) {
      switch (RP) {
        case 16: launch_gram_f32_vec<TrF32, 16>(d, g2, s); break;
        case 32: launch_gram_f32_vec<TrF32, 32>(d, g2, s); break;
        default: launch_gram_f32_vec<TrF32, 64>(d, g2, s); break;
      }
    } else {
      switch (RP) {
        case 16: launch_gram_f32_vec<TrBF16, 16>(d, g2, s); break;
        case 32: launch_gram_f32_vec<TrBF16, 32>(d, g2, s); break;
        default: launch_gram_f32_vec<TrBF16, 64>(d, g2, s); break;
      }
    }
  }
  if (nmulti > 0) {
    ProfScope ps("gram_reduce", s, wk.reduce_tasks * tile + (double)nmulti * tile,
                 wk.reduce_tasks * gram_task_elems(RP));
    dim3 gr((unsigned)nmulti, (unsigned)((gram_task_elems(RP) + 255) / 256));
    if (fdt == TT_F64) {
      switch (RP) {
        case 16: k_gram_reduce<double, 16><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (double *)d.G, d.skip); break;
        case 32: k_gram_reduce<double, 32><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (double *)d.G, d.skip); break;
        default: k_gram_reduce<double, 64><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (double *)d.G, d.skip); break;
      }
    } else {
      switch (RP) {
        case 16: k_gram_reduce<float, 16><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (float *)d.G, d.skip); break;
        case 32: k_gram_reduce<float, 32><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (float *)d.G, d.skip); break;
        default: k_gram_reduce<float, 64><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (float *)d.G, d.skip); break;
      }
      if (d.M) {
        switch (RP) {
          case 16: k_rhs_reduce<16><<<dim3((unsigned)nmulti), 256, 0, s>>>(multi, row_task, d.task_base, d.M, d.skip); break;
          case 32: k_rhs_reduce<32><<<dim3((unsigned)nmulti), 256, 0, s>>>(multi, row_task, d.task_base, d.M, d.skip); break;
          default: k_rhs_reduce<64><<<dim3((unsigned)nmulti), 256, 0, s>>>(multi, row_task, d.task_base, d.M, d.skip); break;
        }
      }
    }
  }
  return hipGetLastError();
}

// Fused Gram + Cholesky of the solo and heavy solo rows of one batch (FP32
// / BF16 forms; kernels instantiated in solve_fused_{f32,bf16}.hip).
static hipError_t launch_solo(tt_dtype fdt, int RP, const GramDev &d, const SolveDev &sd,
                              const GramLists &gl, hipStream_t s) {
  if (gl.nsolo <= 0 && gl.nhsolo <= 0) return hipSuccess;
  return fdt == TT_F32 ? launch_fused_rows_f32(RP, d, sd, gl, s)
                       : launch_fused_rows_bf16(RP, d, sd, gl, s);
}

// Gram tasks whose workspaces one row batch holds (at least a row's tasks).
static int64_t batch_tasks(const ModeIndex &md, int64_t task_bytes) {
  int64_t wtasks = std::max<int64_t>(kGramBatchBytes / task_bytes, md.max_task_per_row);
  wtasks = std::max<int64_t>(wtasks, 1);
  if (wtasks > md.ntask) wtasks = std::max<int64_t>(md.ntask, 1);
  return wtasks;
}

tt_status solve_workspace(tt_index *ix, int mode, int R, tt_dtype fdt, bool fused_rhs,
                          void **G, double **M) {
  const int RP = rp_for(R);
  const int64_t task_bytes = (int64_t)gram_task_elems(RP) * (fdt == TT_F64 ? 8 : 4);
  const int64_t wtasks = batch_tasks(ix->mode[mode], task_bytes);
  void *g = nullptr;
  tt_status st = ws_get(ix, "gram", (size_t)(wtasks * task_bytes), &g);
  if (st != TT_OK) return st;
  if (G) *G = g;
  if (M) *M = nullptr;
  if (fused_rhs) {
    void *p = nullptr;
    st = ws_get(ix, "gram_rhs", (size_t)(wtasks * RP * 8), &p);
    if (st != TT_OK) return st;
    if (M) *M = (double *)p;
  }
  return TT_OK;
}

tt_status run_solve_factor(tt_index *ix, const SolveCall &c, hipStream_t s) {
  const ModeIndex &md = ix->mode[c.mode];
  const int RP = rp_for(c.R);
  const size_t gsz = c.fdt == TT_F64 ? 8 : 4;
  const int64_t task_bytes = (int64_t)gram_task_elems(RP) * gsz;
  const int64_t wtasks = batch_tasks(md, task_bytes);
  void *Gws = nullptr;
  double *Mws = nullptr;
  tt_status st = solve_workspace(ix, c.mode, c.R, c.fdt, c.fused_rhs != 0, &Gws, &Mws);
  if (st != TT_OK) return st;

  int others[2], no = 0;
  for (int p = 0; p < ix->N; ++p)
    if (p != c.mode) others[no++] = p;

  GramDev gd;
  memset(&gd, 0, sizeof(gd));
  gd.task = md.d_task;
  gd.oidx0 = md.d_oidx[others[0]];
  gd.oidx1 = md.d_oidx[others[1]];
  gd.A0 = c.A[others[0]];
  gd.A1 = c.A[others[1]];
  gd.ldA = c.ldA;
  gd.R = c.R;
  gd.w = c.w;
  gd.w_perm = c.w_perm;
  gd.w_scale = c.w_scale;
  gd.G = Gws;
  gd.waves = ix->tune.gram_waves;
  gd.rhs_t = c.fused_rhs ? reinterpret_cast<const float *>(md.d_t) : nullptr;
  gd.M = Mws;
  gd.A_own = c.newton ? c.A[c.mode] : nullptr;
  gd.key = md.d_key;
  gd.loss = c.loss;
  gd.skip = c.skip;
  gd.A_model = c.model ? c.A[c.mode] : nullptr;
  gd.model = reinterpret_cast<float *>(c.model);

  SolveDev sd;
  memset(&sd, 0, sizeof(sd));
  sd.rows = nullptr;
  sd.row_task = md.d_row_task;
  sd.G = Gws;
  sd.R = c.R;
  sd.lambda = c.lambda;
  sd.rhs = c.rhs;
  sd.M = Mws;
  sd.X = c.X;
  sd.ldX = c.ldA;
  sd.info = c.info;
  sd.Lstore = c.Lstore;
  sd.factor_only = c.factor_only;
  sd.skip = c.skip;
  sd.own = c.newton ? c.A[c.mode] : nullptr;
  sd.own_coef = c.own_coef;
  sd.nrow = 0;
  sd.grid_max = ix->tune.solve_wgs > 0 ? (int64_t)ix->tune.solve_wgs * std::max(ix->cu_count, 1) : 0;

  const std::vector<int32_t> &rt = md.h_row_task;
  const int64_t I = md.I;
  int64_t r0 = 0;
  while (r0 < I) {
    // rows [r0, r1) whose tasks fit in the workspace
    int64_t lo = r0 + 1, hi = I;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) / 2;
      if ((int64_t)rt[mid] - rt[r0] <= wtasks) lo = mid; else hi = mid - 1;
    }
    const int64_t r1 = lo;
    gd.task_base = rt[r0];
    gd.task_end = rt[r1];
    const bool f64 = c.fdt == TT_F64;
    // FP32 / BF16 forms up to kFuseHeavyMaxRP: rows with one heavy task are
    // fused with their solve (their own class); otherwise they go with the
    // heavy tasks to the Gram kernel and with the other rows to the solve
    const bool fuse_heavy = !f64 && RP <= kFuseHeavyMaxRP;
    // each host list with the device copy its indices address
    const std::vector<int32_t> &ht = fuse_heavy ? md.h_heavy_task : md.h_heavy_task_all,
                               &mr = md.h_multi_row,
                               &re = fuse_heavy ? md.h_rest_row : md.h_rest_row_all;
    const int32_t *d_ht = fuse_heavy ? md.d_heavy_task : md.d_heavy_task_all;
    const int32_t *d_re = fuse_heavy ? md.d_rest_row : md.d_rest_row_all;
    const int64_t h0 = std::lower_bound(ht.begin(), ht.end(), (int32_t)rt[r0]) - ht.begin();
    const int64_t h1 = std::lower_bound(ht.begin(), ht.end(), (int32_t)rt[r1]) - ht.begin();
    const int64_t q0 = std::lower_bound(mr.begin(), mr.end(), (int32_t)r0) - mr.begin();
    const int64_t q1 = std::lower_bound(mr.begin(), mr.end(), (int32_t)r1) - mr.begin();
    // FP32 / BF16 forms: rows whose only task is light are solved by the
    // fused kernel; the Gram kernels take the heavy tasks and the light tasks
    // of rows with several tasks; the solve kernel takes the other rows
    GramLists gl = {};
    gl.heavy = d_ht + h0;
    gl.nheavy = h1 - h0;
    int64_t p0 = 0, p1 = 0, hs0 = 0, hs1 = 0;
    GramWork wk;
    const std::vector<int64_t> &hn = fuse_heavy ? md.h_heavy_nnz : md.h_heavy_nnz_all;
    wk.heavy_nnz = (double)(hn[h1] - hn[h0]);
    wk.reduce_tasks = 0;
    for (int64_t q = q0; q < q1; ++q) wk.reduce_tasks += rt[mr[q] + 1] - rt[mr[q]];
    if (f64) {
      wk.light_nnz = (double)(md.h_task[rt[r1]] - md.h_task[rt[r0]]) - wk.heavy_nnz;
      wk.light_tasks = (double)(rt[r1] - rt[r0]) - (double)(h1 - h0);
    } else {
      const std::vector<int32_t> &lt = md.h_light_task, &so = md.h_solo_row;
      const int64_t l0 = std::lower_bound(lt.begin(), lt.end(), (int32_t)rt[r0]) - lt.begin();
      const int64_t l1 = std::lower_bound(lt.begin(), lt.end(), (int32_t)rt[r1]) - lt.begin();
      const int64_t s0 = std::lower_bound(so.begin(), so.end(), (int32_t)r0) - so.begin();
      const int64_t s1 = std::lower_bound(so.begin(), so.end(), (int32_t)r1) - so.begin();
      p0 = std::lower_bound(re.begin(), re.end(), (int32_t)r0) - re.begin();
      p1 = std::lower_bound(re.begin(), re.end(), (int32_t)r1) - re.begin();
      gl.light = md.d_light_task + l0;
      gl.nlight = l1 - l0;
      gl.solo = md.d_solo_row + s0;
      gl.nsolo = s1 - s0;
      wk.light_tasks = (double)(l1 - l0);
      wk.light_nnz = 0;
      for (int64_t q = l0; q < l1; ++q)
        wk.light_nnz += (double)(md.h_task[lt[q] + 1] - md.h_task[lt[q]]);
      // fused solo rows: gathers of their nonzeros, the solve's own traffic
      const double Rd = c.R, fb = (double)dtype_size(c.fdt), nsolo = (double)gl.nsolo;
      const double snnz = (double)(md.h_solo_nnz[s1] - md.h_solo_nnz[s0]);
      gl.solo_bytes = snnz * (8 + (c.w ? 4 : 0) + (c.fused_rhs ? 4 : 0) + (c.model ? 4 : 0) +
                              2 * Rd * fb) +
                      nsolo * Rd * (4 + fb) +
                      (c.Lstore ? nsolo * RP * (RP + 1) / 2 * 4.0 : 0.0);
      gl.solo_flops = snnz * Rd * (Rd + 1) +
                      nsolo * (Rd * Rd * Rd / 3.0 + (c.factor_only ? 0.0 : 2.0 * Rd * Rd));
      // rows whose only task is heavy, fused with their solve
      if (fuse_heavy) {
        const std::vector<int32_t> &hs = md.h_hsolo_row;
        hs0 = std::lower_bound(hs.begin(), hs.end(), (int32_t)r0) - hs.begin();
        hs1 = std::lower_bound(hs.begin(), hs.end(), (int32_t)r1) - hs.begin();
        const double hnnz = (double)(md.h_hsolo_nnz[hs1] - md.h_hsolo_nnz[hs0]);
        const double nhs = (double)(hs1 - hs0);
        gl.hsolo = md.d_hsolo_row + hs0;
        gl.nhsolo = hs1 - hs0;
        gl.hsolo_bytes = hnnz * (8 + (c.w ? 4 : 0) + (c.fused_rhs ? 4 : 0) + (c.model ? 4 : 0) +
                                 2 * Rd * fb) +
                         nhs * Rd * (4 + fb) +
                         (c.Lstore ? nhs * RP * (RP + 1) / 2 * 4.0 : 0.0);
        gl.hsolo_flops = hnnz * Rd * (Rd + 1) +
                         nhs * (Rd * Rd * Rd / 3.0 + (c.factor_only ? 0.0 : 2.0 * Rd * Rd));
      }
    }
    hipError_t e = launch_gram(c.fdt, RP, gd, gl, md.d_multi_row + q0, q1 - q0,
                               md.d_row_task, wk, s);
    if (e != hipSuccess) return hip_fail(e, "gram kernel");
    sd.task_base = rt[r0];
    sd.r0 = r0;
    const int64_t nrest = f64 ? r1 - r0 : p1 - p0;
    sd.rows = f64 ? nullptr : d_re + p0;
    const double Rd = c.R, nrow = (double)nrest;
    {
      ProfScope ps(c.factor_only ? "cholesky_factor" : "cholesky_solve", s,
                   (double)(rt[r1] - rt[r0] - (f64 ? 0 : gl.nsolo + hs1 - hs0)) *
                           gram_task_elems(RP) *
                           (double)gsz +
                       nrow * Rd * (double)(gsz + dtype_size(c.fdt)) +
                       (c.Lstore ? nrow * RP * (RP + 1) / 2 * (double)gsz : 0.0),
                   nrow * (Rd * Rd * Rd / 3.0 + (c.factor_only ? 0.0 : 2.0 * Rd * Rd)));
      if (c.fdt == TT_F64)
        e = launch_solve_rp<double, double, double>(RP, sd, nrest, s);
      else if (c.fdt == TT_F32)
        e = launch_solve_rp<float, float, float>(RP, sd, nrest, s);
      else
        e = launch_solve_rp<float, uint16_t, float>(RP, sd, nrest, s);
    }
    if (e != hipSuccess) return hip_fail(e, "solve kernel");
    if (!f64) {
      e = launch_solo(c.fdt, RP, gd, sd, gl, s);
      if (e != hipSuccess) return hip_fail(e, "fused solve kernel");
    }
    r0 = r1;
  }
  return TT_OK;
}

hipError_t launch_apply_factor(const tt_index *ix, int mode, int R, tt_dtype fdt,
                               const void *Lstore, const void *rhs, void *X,
                               const double *skip, hipStream_t s) {
  const int64_t I = ix->mode[mode].I;
  if (I <= 0) return hipSuccess;
  const int RP = rp_for(R);
  dim3 g((unsigned)I), b(64);
  const double es = fdt == TT_F64 ? 8.0 : 4.0;
  ProfScope ps("precond_apply", s, (double)I * RP * (RP + 1) / 2 * es + (double)I * R * 2 * es,
               (double)I * 2.0 * R * R);
  const double *Ld = static_cast<const double *>(Lstore);
  const float *Lf = static_cast<const float *>(Lstore);
  if (fdt == TT_F64) {
    switch (RP) {
      case 16: k_apply_rows<double, 16><<<g, b, 0, s>>>(Ld, rhs, X, R, skip); break;
      case 32: k_apply_rows<double, 32><<<g, b, 0, s>>>(Ld, rhs, X, R, skip); break;
      default: k_apply_rows<double, 64><<<g, b, 0, s>>>(Ld, rhs, X, R, skip); break;
    }
  } else {
    switch (RP) {
      case 16: k_apply_rows<float, 16><<<g, b, 0, s>>>(Lf, rhs, X, R, skip); break;
      case 32: k_apply_rows<float, 32><<<g, b, 0, s>>>(Lf, rhs, X, R, skip); break;
      default: k_apply_rows<float, 64><<<g, b, 0, s>>>(Lf, rhs, X, R, skip); break;
    }
  }
  return hipGetLastError();
}

}  // namespace tt
