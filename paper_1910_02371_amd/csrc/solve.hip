// Solve Factor (Section 3.4): per-row Gram matrices
//     G^(i) = sum_{e in row i} w_e h_e h_e^T,   h_e = Hadamard_{p != n} A_p[i_p(e)]
// built on matrix cores, then (G^(i) + lambda I) x_i = M_i solved per row by
// an FP64 Cholesky factorization and two triangular solves (the SPD solve of
// Section 3.4; the normal equations of Section 2.2).
//
// Gram: one wave per task (a piece of <= kGramPiece nonzeros of one row).
// With H the task's rows h_e stacked, G = H^T diag(w) H is a K x R by K x R
// contraction over the nonzeros, mapped onto MFMA with the nonzero index as
// the reduction dimension: A-operand = h (R on the M index), B-operand = w h.
//   FP32/BF16 storage: v_mfma_f32_16x16x4f32 (R <= 16) or
//                      v_mfma_f32_32x32x2f32 (R <= 32, and 3 tiles for R <= 64).
//   BF16 factors are widened exactly to FP32 (a product of two bf16 values
//   is exact in FP32), so the BF16 form accumulates like the FP32 form.
//   FP64 storage: v_mfma_f64_16x16x4f64 tiles (lower triangle only).
// Each task writes its lower-triangular G (row-major RP x RP) to a batch
// workspace; rows with several tasks are summed in FP64 in task order by the
// solve kernel (deterministic).
//
// Solve: one wave per row; lane i keeps row i of S = G + lambda I in FP64
// registers and a right-looking Cholesky runs over columns, broadcasting
// L(j,k) with readlane; the forward solve stays in registers and the
// backward solve with L^T reads L from LDS.  Non-positive pivots follow
// LAPACK potrf: info = order of the failing leading minor, x = 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.h"
#include "internal.h"

namespace tt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

struct GramDev {
  const int64_t *task;        // task boundaries in the sorted stream
  int64_t task_base, task_end;
  const int32_t *oidx0, *oidx1;
  const void *A0, *A1;        // other modes' factors (order of the streams)
  int64_t ldA;
  int R;
  const void *w;              // weights in stream order (value dtype) or NULL
  const int32_t *w_perm;
  double w_scale;
  void *G;                    // workspace: (task - task_base) * RP * RP
};

template <class TR>
__device__ __forceinline__ float elem_f(const typename TR::T *A, int64_t off);
template <>
__device__ __forceinline__ float elem_f<TrF32>(const float *A, int64_t off) { return A[off]; }
template <>
__device__ __forceinline__ float elem_f<TrBF16>(const uint16_t *A, int64_t off) {
  return bf16_to_f32(A[off]);
}

template <class VT>
__device__ __forceinline__ VT weight_at(const GramDev &d, int64_t pos) {
  if (d.w == nullptr) return (VT)d.w_scale;
  int64_t q = d.w_perm ? (int64_t)d.w_perm[pos] : pos;
  return (VT)d.w_scale * reinterpret_cast<const VT *>(d.w)[q];
}

// FP32 / BF16 storage, FP32 accumulation on matrix cores.
template <class TR, int RP>
__global__ __launch_bounds__(256) void k_gram_f32(GramDev d) {
  using T = typename TR::T;
  const int lane = threadIdx.x & 63;
  const int64_t t = d.task_base + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= d.task_end) return;
  const int64_t nb = d.task[t], ne = d.task[t + 1];
  const T *A0 = reinterpret_cast<const T *>(d.A0);
  const T *A1 = reinterpret_cast<const T *>(d.A1);
  const int R = d.R;
  constexpr int NPS = (RP == 16) ? 4 : 2;     // nonzeros per MFMA step
  constexpr int MW = (RP == 16) ? 16 : 32;    // M = N of the instruction
  const int i = lane % MW;
  const int kk = lane / MW;
  f32x4 c16 = {0.f, 0.f, 0.f, 0.f};
  f32x16 c00, c01, c11;
#pragma unroll
  for (int v = 0; v < 16; ++v) { c00[v] = 0.f; c01[v] = 0.f; c11[v] = 0.f; }

  for (int64_t base = nb; base < ne; base += 64) {
    const int cnt = (int)min((int64_t)64, ne - base);
    int my0 = 0, my1 = 0;
    float myw = 0.f;
    if (lane < cnt) {
      my0 = d.oidx0[base + lane];
      my1 = d.oidx1[base + lane];
      myw = weight_at<float>(d, base + lane);
    }
    const int steps = (cnt + NPS - 1) / NPS;
    for (int st = 0; st < steps; ++st) {
      const int src = st * NPS + kk;
      const int j0 = __shfl(my0, src);
      const int j1 = __shfl(my1, src);
      const float w = __shfl(myw, src);
      float h0 = 0.f, h1 = 0.f;
      if (i < R) h0 = elem_f<TR>(A0, (int64_t)j0 * d.ldA + i) * elem_f<TR>(A1, (int64_t)j1 * d.ldA + i);
      if constexpr (RP == 64) {
        if (i + 32 < R)
          h1 = elem_f<TR>(A0, (int64_t)j0 * d.ldA + i + 32) *
               elem_f<TR>(A1, (int64_t)j1 * d.ldA + i + 32);
      }
      if constexpr (RP == 16) {
        c16 = __builtin_amdgcn_mfma_f32_16x16x4f32(h0, w * h0, c16, 0, 0, 0);
      } else {
        c00 = __builtin_amdgcn_mfma_f32_32x32x2f32(h0, w * h0, c00, 0, 0, 0);
        if constexpr (RP == 64) {
          c01 = __builtin_amdgcn_mfma_f32_32x32x2f32(h0, w * h1, c01, 0, 0, 0);
          c11 = __builtin_amdgcn_mfma_f32_32x32x2f32(h1, w * h1, c11, 0, 0, 0);
        }
      }
    }
  }
  float *G = reinterpret_cast<float *>(d.G) + (t - d.task_base) * (int64_t)(RP * RP);
  if constexpr (RP == 16) {
    // D[row][col]: col = lane % 16, row = 4 * (lane / 16) + v
#pragma unroll
    for (int v = 0; v < 4; ++v) G[(4 * (lane / 16) + v) * RP + lane % 16] = c16[v];
  } else {
    // D[row][col]: col = lane % 32, row = 8 * (v / 4) + 4 * (lane / 32) + v % 4
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 8 * (v / 4) + 4 * (lane / 32) + (v % 4);
      const int col = lane % 32;
      G[row * RP + col] = c00[v];
      if constexpr (RP == 64) {
        G[(32 + row) * RP + 32 + col] = c11[v];
        G[(32 + col) * RP + row] = c01[v];  // block (1,0) = (block (0,1))^T
      }
    }
  }
}

// FP64 storage and accumulation: 16x16x4 FP64 tiles of the lower triangle.
template <int RP>
__global__ __launch_bounds__(256) void k_gram_f64(GramDev d) {
  constexpr int TB = RP / 16;
  constexpr int NT = TB * (TB + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int64_t t = d.task_base + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= d.task_end) return;
  const int64_t nb = d.task[t], ne = d.task[t + 1];
  const double *A0 = reinterpret_cast<const double *>(d.A0);
  const double *A1 = reinterpret_cast<const double *>(d.A1);
  const int R = d.R;
  const int i = lane % 16, kk = lane / 16;
  f64x4 c[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) c[q] = (f64x4){0.0, 0.0, 0.0, 0.0};
  for (int64_t base = nb; base < ne; base += 64) {
    const int cnt = (int)min((int64_t)64, ne - base);
    int my0 = 0, my1 = 0;
    double myw = 0.0;
    if (lane < cnt) {
      my0 = d.oidx0[base + lane];
      my1 = d.oidx1[base + lane];
      myw = weight_at<double>(d, base + lane);
    }
    const int steps = (cnt + 3) / 4;
    for (int st = 0; st < steps; ++st) {
      const int src = st * 4 + kk;
      const int j0 = __shfl(my0, src);
      const int j1 = __shfl(my1, src);
      const double w = __shfl(myw, src);
      double h[TB];
#pragma unroll
      for (int a = 0; a < TB; ++a) {
        const int col = 16 * a + i;
        h[a] = col < R ? A0[(int64_t)j0 * d.ldA + col] * A1[(int64_t)j1 * d.ldA + col] : 0.0;
      }
      int q = 0;
#pragma unroll
      for (int a = 0; a < TB; ++a)
#pragma unroll
        for (int bb = 0; bb <= a; ++bb) {
          c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[a], w * h[bb], c[q], 0, 0, 0);
          ++q;
        }
    }
  }
  double *G = reinterpret_cast<double *>(d.G) + (t - d.task_base) * (int64_t)(RP * RP);
  int q = 0;
#pragma unroll
  for (int a = 0; a < TB; ++a)
#pragma unroll
    for (int bb = 0; bb <= a; ++bb) {
      // v_mfma_f64_16x16x4f64 result: D[row][col] at col = lane % 16,
      // row = 4 * v + lane / 16 (checked on the device)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 4 * v + lane / 16, col = lane % 16;
        G[(16 * a + row) * RP + 16 * bb + col] = c[q][v];
        if (a != bb) G[(16 * bb + col) * RP + 16 * a + row] = c[q][v];
      }
      ++q;
    }
}

// ---------------------------------------------------------------------------
__device__ __forceinline__ double readlane_d(double x, int l) {
  long long b = __double_as_longlong(x);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

struct SolveDev {
  const int32_t *row_task;   // I + 1
  int64_t task_base;
  int64_t r0;                // first row of the batch
  const void *G;             // Gram workspace (float or double per dtype)
  int R;
  double lambda;
  const void *rhs;           // I x R dense dtype
  void *X;                   // I x R in storage dtype, leading dim ldX
  int64_t ldX;
  int32_t *info;
  double *Lstore;            // I x RP x RP (optional)
  int factor_only;
  const double *skip;
};

// Cholesky of the lane-distributed matrix s (lane i = row i), in place:
// afterwards s[j] on lane i holds L(i, j) for j <= i.  Returns info.
template <int RP>
__device__ __forceinline__ int chol_lanes(double (&s)[RP], int lane) {
#pragma unroll
  for (int k = 0; k < RP; ++k) {
    const double dkk = readlane_d(s[k], k);
    if (!(dkk > 0.0)) return k + 1;
    const double rd = sqrt(dkk);
    const double inv = 1.0 / rd;
    const double lik = lane > k ? s[k] * inv : (lane == k ? rd : 0.0);
    s[k] = lik;
#pragma unroll
    for (int j = k + 1; j < RP; ++j) {
      const double ljk = readlane_d(lik, j);
      s[j] -= lik * ljk;
    }
  }
  return 0;
}

// Solve L L^T x = b with L held as in chol_lanes; b on lane i is b_i.
template <int RP>
__device__ __forceinline__ double chol_solve_lanes(const double (&s)[RP], double b,
                                                   int lane, double *lds) {
  // forward: L y = b (column-oriented, y kept in b)
#pragma unroll
  for (int k = 0; k < RP; ++k) {
    const double yk = readlane_d(b, k) / readlane_d(s[k], k);
    b = lane == k ? yk : (lane > k ? b - s[k] * yk : b);
  }
  // backward: L^T x = y; lane i needs L(k, i), staged row-major in LDS
#pragma unroll
  for (int j = 0; j < RP; ++j)
    if (lane < RP) lds[lane * (RP + 1) + j] = s[j];
  __syncthreads();
  double diag = 0.0;
#pragma unroll
  for (int k = 0; k < RP; ++k)
    if (k == lane) diag = s[k];
#pragma unroll
  for (int k = RP - 1; k >= 0; --k) {
    const double xk = readlane_d(b, k) / readlane_d(diag, k);
    const double lki = (lane < k) ? lds[k * (RP + 1) + lane] : 0.0;
    b = lane == k ? xk : (lane < k ? b - lki * xk : b);
  }
  return b;
}

template <class GT, class XT, class MT, int RP>
__global__ __launch_bounds__(64) void k_solve_rows(SolveDev d) {
  __shared__ double lds[RP * (RP + 1)];
  if (d.skip && *d.skip != 0.0) return;
  const int lane = threadIdx.x;
  const int64_t row = d.r0 + blockIdx.x;
  const int R = d.R;
  const int32_t t0 = d.row_task[row], t1 = d.row_task[row + 1];
  double s[RP];
#pragma unroll
  for (int j = 0; j < RP; ++j) s[j] = 0.0;
  if (lane < RP) {
    for (int32_t t = t0; t < t1; ++t) {
      const GT *g = reinterpret_cast<const GT *>(d.G) +
                    ((int64_t)t - d.task_base) * (RP * RP) + lane * RP;
#pragma unroll
      for (int j = 0; j < RP; ++j) s[j] += (double)g[j];
    }
  }
#pragma unroll
  for (int j = 0; j < RP; ++j) {
    if (lane >= R || j >= R) s[j] = (j == lane) ? 1.0 : 0.0;
    else if (j == lane) s[j] += d.lambda;
  }
  const int info = chol_lanes<RP>(s, lane);
  if (d.info && lane == 0) d.info[row] = info;
  if (d.Lstore) {
    double *L = d.Lstore + row * (int64_t)(RP * RP) + lane * RP;
    if (lane < RP) {
#pragma unroll
      for (int j = 0; j < RP; ++j) L[j] = info ? ((j == lane) ? 1.0 : 0.0) : s[j];
    }
  }
  if (d.factor_only) return;
  double x = 0.0;
  if (info == 0) {
    const double b = lane < R ? (double)reinterpret_cast<const MT *>(d.rhs)[row * R + lane] : 0.0;
    x = chol_solve_lanes<RP>(s, b, lane, lds);
  }
  if (lane < R) reinterpret_cast<XT *>(d.X)[row * d.ldX + lane] = from_double<XT>(x);
}

// Apply stored factors to a right-hand side: X = (L L^T)^{-1} rhs.
template <class MT, int RP>
__global__ __launch_bounds__(64) void k_apply_rows(const double *__restrict__ Lstore,
                                                   const void *rhs, void *X, int R,
                                                   const double *skip) {
  __shared__ double lds[RP * (RP + 1)];
  if (skip && *skip != 0.0) return;
  const int lane = threadIdx.x;
  const int64_t row = blockIdx.x;
  double s[RP];
  const double *L = Lstore + row * (int64_t)(RP * RP) + (lane < RP ? lane : 0) * RP;
#pragma unroll
  for (int j = 0; j < RP; ++j) s[j] = lane < RP ? L[j] : 0.0;
  const double b = lane < R ? (double)reinterpret_cast<const MT *>(rhs)[row * R + lane] : 0.0;
  const double x = chol_solve_lanes<RP>(s, b, lane, lds);
  if (lane < R) reinterpret_cast<MT *>(X)[row * R + lane] = (MT)x;
}

// ---------------------------------------------------------------------------
static int rp_for(int R) { return R <= 16 ? 16 : (R <= 32 ? 32 : 64); }

template <class GT, class XT, class MT>
static hipError_t launch_solve_rp(int RP, const SolveDev &d, int64_t nrow, hipStream_t s) {
  if (nrow <= 0) return hipSuccess;
  dim3 g((unsigned)nrow), b(64);
  switch (RP) {
    case 16: k_solve_rows<GT, XT, MT, 16><<<g, b, 0, s>>>(d); break;
    case 32: k_solve_rows<GT, XT, MT, 32><<<g, b, 0, s>>>(d); break;
    default: k_solve_rows<GT, XT, MT, 64><<<g, b, 0, s>>>(d); break;
  }
  return hipGetLastError();
}

static hipError_t launch_gram(tt_dtype fdt, int RP, const GramDev &d, hipStream_t s) {
  const int64_t n = d.task_end - d.task_base;
  if (n <= 0) return hipSuccess;
  dim3 g((unsigned)((n + 3) / 4)), b(256);
  if (fdt == TT_F64) {
    switch (RP) {
      case 16: k_gram_f64<16><<<g, b, 0, s>>>(d); break;
      case 32: k_gram_f64<32><<<g, b, 0, s>>>(d); break;
      default: k_gram_f64<64><<<g, b, 0, s>>>(d); break;
    }
  } else if (fdt == TT_F32) {
    switch (RP) {
      case 16: k_gram_f32<TrF32, 16><<<g, b, 0, s>>>(d); break;
      case 32: k_gram_f32<TrF32, 32><<<g, b, 0, s>>>(d); break;
      default: k_gram_f32<TrF32, 64><<<g, b, 0, s>>>(d); break;
    }
  } else {
    switch (RP) {
      case 16: k_gram_f32<TrBF16, 16><<<g, b, 0, s>>>(d); break;
      case 32: k_gram_f32<TrBF16, 32><<<g, b, 0, s>>>(d); break;
      default: k_gram_f32<TrBF16, 64><<<g, b, 0, s>>>(d); break;
    }
  }
  return hipGetLastError();
}

tt_status run_solve_factor(tt_index *ix, const SolveCall &c, hipStream_t s) {
  const ModeIndex &md = ix->mode[c.mode];
  const int RP = rp_for(c.R);
  const size_t gsz = c.fdt == TT_F64 ? 8 : 4;
  const int64_t task_bytes = (int64_t)RP * RP * gsz;
  int64_t wtasks = std::max<int64_t>(kGramBatchBytes / task_bytes, md.max_task_per_row);
  wtasks = std::max<int64_t>(wtasks, 1);
  if (wtasks > md.ntask) wtasks = std::max<int64_t>(md.ntask, 1);
  void *Gws = nullptr;
  tt_status st = ws_get(ix, "gram", (size_t)(wtasks * task_bytes), &Gws);
  if (st != TT_OK) return st;

  int others[2], no = 0;
  for (int p = 0; p < ix->N; ++p)
    if (p != c.mode) others[no++] = p;

  GramDev gd;
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

  SolveDev sd;
  sd.row_task = md.d_row_task;
  sd.G = Gws;
  sd.R = c.R;
  sd.lambda = c.lambda;
  sd.rhs = c.rhs;
  sd.X = c.X;
  sd.ldX = c.ldA;
  sd.info = c.info;
  sd.Lstore = c.Lstore;
  sd.factor_only = c.factor_only;
  sd.skip = nullptr;

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
    hipError_t e = launch_gram(c.fdt, RP, gd, s);
    if (e != hipSuccess) return hip_fail(e, "gram kernel");
    sd.task_base = rt[r0];
    sd.r0 = r0;
    // advance row pointers by offsetting the batch (row index = r0 + block)
    if (c.fdt == TT_F64)
      e = launch_solve_rp<double, double, double>(RP, sd, r1 - r0, s);
    else if (c.fdt == TT_F32)
      e = launch_solve_rp<float, float, float>(RP, sd, r1 - r0, s);
    else
      e = launch_solve_rp<float, uint16_t, float>(RP, sd, r1 - r0, s);
    if (e != hipSuccess) return hip_fail(e, "solve kernel");
    r0 = r1;
  }
  return TT_OK;
}

hipError_t launch_apply_factor(const tt_index *ix, int mode, int R, tt_dtype fdt,
                               const double *Lstore, const void *rhs, void *X,
                               const double *skip, hipStream_t s) {
  const int64_t I = ix->mode[mode].I;
  if (I <= 0) return hipSuccess;
  const int RP = rp_for(R);
  dim3 g((unsigned)I), b(64);
  if (fdt == TT_F64) {
    switch (RP) {
      case 16: k_apply_rows<double, 16><<<g, b, 0, s>>>(Lstore, rhs, X, R, skip); break;
      case 32: k_apply_rows<double, 32><<<g, b, 0, s>>>(Lstore, rhs, X, R, skip); break;
      default: k_apply_rows<double, 64><<<g, b, 0, s>>>(Lstore, rhs, X, R, skip); break;
    }
  } else {
    switch (RP) {
      case 16: k_apply_rows<float, 16><<<g, b, 0, s>>>(Lstore, rhs, X, R, skip); break;
      case 32: k_apply_rows<float, 32><<<g, b, 0, s>>>(Lstore, rhs, X, R, skip); break;
      default: k_apply_rows<float, 64><<<g, b, 0, s>>>(Lstore, rhs, X, R, skip); break;
    }
  }
  return hipGetLastError();
}

}  // namespace tt
