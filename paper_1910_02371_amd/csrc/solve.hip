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
//   FP32/BF16 storage: v_mfma_f32_16x16x4f32 tiles, four nonzeros per step,
//                      each lane reading RP / 16 consecutive columns of a row
//                      (RP (RP / 16 + 1) / 32 tiles cover the upper triangle).
//   BF16 factors are widened exactly to FP32 (a product of two bf16 values
//   is exact in FP32), so the BF16 form accumulates like the FP32 form.
//   FP64 storage: v_mfma_f64_16x16x4f64 tiles (lower triangle only).
// Each task writes the upper triangle of its G (row-major RP x RP) to a batch
// workspace; the solve kernel reads it by columns (lane i takes G[j][i] =
// G[i][j] for j <= i), so its loads are coalesced.  Rows with several tasks
// are summed in FP64 in task order (deterministic).
//
// Solve: one wave per row; lane i keeps row i of S = G + lambda I in FP64
// registers and a right-looking Cholesky runs over columns, broadcasting
// L(j,k) with readlane; the forward solve stays in registers and the
// backward solve with L^T reads L from LDS.  Non-positive pivots follow
// LAPACK potrf: info = order of the failing leading minor, x = 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
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
  int split_heavy;            // light kernel skips tasks > kGramLight
};

template <class TR>
__device__ __forceinline__ float elem_f(const typename TR::T *A, int64_t off);
template <>
__device__ __forceinline__ float elem_f<TrF32>(const float *A, int64_t off) { return A[off]; }
template <>
__device__ __forceinline__ float elem_f<TrBF16>(const uint16_t *A, int64_t off) {
  return bf16_to_f32(A[off]);
}
// Same load with a 32-bit element offset (factor matrices below 2^32 bytes),
// which lets the address be a scalar base plus a 32-bit vector offset.
template <class TR>
__device__ __forceinline__ float elem_f32off(const typename TR::T *A, uint32_t off) {
  const typename TR::T *p = reinterpret_cast<const typename TR::T *>(
      reinterpret_cast<const char *>(A) + (uint32_t)(off * (uint32_t)sizeof(typename TR::T)));
  if constexpr (sizeof(typename TR::T) == 4) return *p;
  else return bf16_to_f32(*p);
}

template <class VT>
__device__ __forceinline__ VT weight_at(const GramDev &d, int64_t pos) {
  if (d.w == nullptr) return (VT)d.w_scale;
  int64_t q = d.w_perm ? (int64_t)d.w_perm[pos] : pos;
  return (VT)d.w_scale * reinterpret_cast<const VT *>(d.w)[q];
}

// FP32 / BF16 storage, FP32 accumulation on v_mfma_f32_16x16x4f32.
// Vector-fragment layout: lane l = 16 k + i takes nonzero k of a step (four
// nonzeros per step) and columns VW*i .. VW*i + VW - 1 of its two factor rows
// (VW = RP / 16), read as one vector load.  Register v of lane (i, k) then
// holds column VW*i + v, so the register-class pair (p, q) is one 16x16x4
// MFMA whose tile entry (r, c) is G[VW*r + p][VW*c + q].  The classes
// p <= q (VW (VW + 1) / 2 tiles) cover every unordered column pair: once when
// p < q, twice when p == q (only r <= c is stored).
template <int RP>
struct GramAcc {
  static constexpr int VW = RP / 16;
  static constexpr int NT = VW * (VW + 1) / 2;
  static constexpr int NV = 4 * NT;
  f32x4 c[NT];
  __device__ void zero() {
#pragma unroll
    for (int q = 0; q < NT; ++q) c[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
  }
  __device__ float get(int v) const { return c[v / 4][v % 4]; }
  __device__ void set(int v, float x) { c[v / 4][v % 4] = x; }
};

#ifndef TT_GRAM_GS
#define TT_GRAM_GS 4          // MFMA steps whose gathers are issued together
#endif
#ifndef TT_GRAM_HEAVY_WAVES
#define TT_GRAM_HEAVY_WAVES 8 // waves of the workgroup that takes a heavy task
#endif

// VW consecutive factor entries starting at element `off`, widened to FP32.
// VEC: one aligned vector load (the caller guarantees alignment and that
// the whole vector lies inside the row); otherwise element loads.
template <class TR, int VW, bool VEC>
__device__ __forceinline__ void load_cols(const typename TR::T *A, uint32_t off, int cb,
                                          int R, float (&o)[VW]) {
  if constexpr (VEC) {
    const uint32_t e = off + (uint32_t)(cb < R ? cb : 0);
    if constexpr (std::is_same<TR, TrF32>::value) {
      if constexpr (VW == 4) {
        const float4 x = *reinterpret_cast<const float4 *>(at32(A, e));
        o[0] = x.x; o[1] = x.y; o[2] = x.z; o[3] = x.w;
      } else if constexpr (VW == 2) {
        const float2 x = *reinterpret_cast<const float2 *>(at32(A, e));
        o[0] = x.x; o[1] = x.y;
      } else {
        o[0] = *at32(A, e);
      }
    } else {
      if constexpr (VW == 4) {
        const uint2 x = *reinterpret_cast<const uint2 *>(at32(A, e));
        o[0] = __uint_as_float(x.x << 16); o[1] = __uint_as_float(x.x & 0xffff0000u);
        o[2] = __uint_as_float(x.y << 16); o[3] = __uint_as_float(x.y & 0xffff0000u);
      } else if constexpr (VW == 2) {
        const uint32_t x = *reinterpret_cast<const uint32_t *>(at32(A, e));
        o[0] = __uint_as_float(x << 16); o[1] = __uint_as_float(x & 0xffff0000u);
      } else {
        o[0] = bf16_to_f32(*at32(A, e));
      }
    }
  } else {
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      const int c = cb + v;
      const uint32_t e = off + (uint32_t)(c < R ? c : 0);
      if constexpr (std::is_same<TR, TrF32>::value) o[v] = *at32(A, e);
      else o[v] = bf16_to_f32(*at32(A, e));
    }
  }
}

template <class TR, int RP, int GS>
struct GramGroup {
  float a0[GS][RP / 16], a1[GS][RP / 16], w[GS];
};

// Nonzeros [nb, ne) of one row into acc.  The range is walked in blocks of
// 64 nonzeros (lane l loads the indices and weight of nonzero base + l,
// coalesced, one block ahead) and, inside a block, in groups of GS MFMA
// steps: the shuffles and factor-row gathers of a group are issued together,
// then its MFMAs.  Padding columns (>= R) use a clamped address and a zero
// mask, so loads are unconditional; steps past the end read lanes whose
// weight is 0.
template <class TR, int RP, bool VEC>
__device__ __forceinline__ void gram_accum(const GramDev &d, int64_t nb, int64_t ne,
                                           GramAcc<RP> &acc) {
  using T = typename TR::T;
  constexpr int VW = RP / 16;
  constexpr int GS = TT_GRAM_GS;              // steps per group
  constexpr int SPB = 16;                     // steps per 64-nonzero block
  constexpr int GPB = SPB / GS;               // groups per block
  static_assert(SPB % GS == 0, "group size must divide the block");
  const int lane = threadIdx.x & 63;
  const T *A0 = reinterpret_cast<const T *>(d.A0);
  const T *A1 = reinterpret_cast<const T *>(d.A1);
  const int R = d.R;
  const uint32_t ldA = (uint32_t)d.ldA;
  const int kk = lane >> 4;
  const int cb = VW * (lane & 15);
  float m[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) m[v] = (cb + v < R) ? 1.f : 0.f;
  const int64_t n = ne - nb;
  if (n <= 0) return;
  const int64_t nblk = (n + 63) / 64;
  const int last_cnt = (int)(n - (nblk - 1) * 64);
  const int64_t gtot = (nblk - 1) * GPB + ((last_cnt + 3) / 4 + GS - 1) / GS;

  auto load_block = [&](int64_t blk, int &j0, int &j1, float &w) {
    const int64_t e = nb + blk * 64 + lane;
    if (e < ne) {
      j0 = d.oidx0[e];
      j1 = d.oidx1[e];
      w = weight_at<float>(d, e);
    } else {
      j0 = 0; j1 = 0; w = 0.f;
    }
  };
  // `cur` registers hold the block of the group being prepared, `nxt` the
  // following block
  int cj0, cj1, nj0 = 0, nj1 = 0;
  float cw, nw = 0.f;
  load_block(0, cj0, cj1, cw);
  if (nblk > 1) load_block(1, nj0, nj1, nw);
  int64_t cblk = 0;

  GramGroup<TR, RP, GS> g;
  for (int64_t gi = 0; gi < gtot; ++gi) {
    const int64_t blk = gi / GPB;
    if (blk != cblk) {  // advance cur to blk (== cblk + 1), prefetch the next
      cj0 = nj0; cj1 = nj1; cw = nw;
      cblk = blk;
      if (blk + 1 < nblk) load_block(blk + 1, nj0, nj1, nw);
    }
    const int st0 = (int)(gi % GPB) * GS;
    int j0[GS], j1[GS];
#pragma unroll
    for (int u = 0; u < GS; ++u) {
      const int src = (st0 + u) * 4 + kk;
      j0[u] = __shfl(cj0, src);
      j1[u] = __shfl(cj1, src);
      g.w[u] = __shfl(cw, src);
    }
#pragma unroll
    for (int u = 0; u < GS; ++u) {
      load_cols<TR, VW, VEC>(A0, (uint32_t)j0[u] * ldA, cb, R, g.a0[u]);
      load_cols<TR, VW, VEC>(A1, (uint32_t)j1[u] * ldA, cb, R, g.a1[u]);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < GS; ++u) {
      float h[VW], hw[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        h[v] = g.a0[u][v] * g.a1[u][v] * m[v];
        hw[v] = g.w[u] * h[v];
      }
      int q = 0;
#pragma unroll
      for (int p = 0; p < VW; ++p)
#pragma unroll
        for (int pp = p; pp < VW; ++pp) {
          acc.c[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(h[p], hw[pp], acc.c[q], 0, 0, 0);
          ++q;
        }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Write the upper triangle of G (row-major RP x RP) from the accumulators.
// v_mfma_f32_16x16x4f32 result: lane l, register v holds D[4 (l / 16) + v][l % 16].
template <int RP>
__device__ __forceinline__ void gram_store(float *G, const GramAcc<RP> &acc) {
  constexpr int VW = RP / 16;
  const int lane = threadIdx.x & 63;
  const int c = lane & 15;
  int q = 0;
#pragma unroll
  for (int p = 0; p < VW; ++p)
#pragma unroll
    for (int pp = p; pp < VW; ++pp) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * (lane >> 4) + v;
        const int a = VW * r + p, b = VW * c + pp;
        if (p < pp || r <= c) G[min(a, b) * RP + max(a, b)] = acc.c[q][v];
      }
      ++q;
    }
}

// Light tasks: one wave per task, four tasks per workgroup; tasks with more
// than kGramLight nonzeros are left to k_gram_f32_heavy.
template <class TR, int RP, bool VEC>
__global__ __launch_bounds__(256) void k_gram_f32(GramDev d) {
  const int64_t t = d.task_base + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= d.task_end) return;
  const int64_t nb = d.task[t], ne = d.task[t + 1];
  if (d.split_heavy && ne - nb > kGramLight) return;
  GramAcc<RP> acc;
  acc.zero();
  gram_accum<TR, RP, VEC>(d, nb, ne, acc);
  gram_store<RP>(reinterpret_cast<float *>(d.G) + (t - d.task_base) * (int64_t)(RP * RP), acc);
}

// Heavy tasks: the waves of a workgroup split the task's nonzeros and add
// their accumulators through LDS in wave order (deterministic).
template <class TR, int RP, bool VEC>
__global__ __launch_bounds__(64 * TT_GRAM_HEAVY_WAVES) void k_gram_f32_heavy(
    GramDev d, const int32_t *heavy, int64_t nheavy) {
  constexpr int NV = GramAcc<RP>::NV;
  constexpr int NW = TT_GRAM_HEAVY_WAVES;
  __shared__ float buf[NV * 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = heavy[blockIdx.x];
  const int64_t nb = d.task[t], ne = d.task[t + 1];
  const int64_t per = (((ne - nb) + NW - 1) / NW + 3) & ~(int64_t)3;
  const int64_t b0 = min(ne, nb + w * per), b1 = min(ne, b0 + per);
  GramAcc<RP> acc;
  acc.zero();
  gram_accum<TR, RP, VEC>(d, b0, b1, acc);
  for (int q = 0; q < NW; ++q) {
    if (w == q) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        buf[v * 64 + lane] = (q == 0 ? 0.f : buf[v * 64 + lane]) + acc.get(v);
    }
    __syncthreads();
  }
  if (w == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc.set(v, buf[v * 64 + lane]);
    gram_store<RP>(reinterpret_cast<float *>(d.G) + (t - d.task_base) * (int64_t)(RP * RP), acc);
  }
}

// Rows with more than kReduceMin tasks: sum the upper triangles of their
// tasks' Grams entrywise in FP64, in task order, into the row's first task
// slot.
template <class GT, int RP>
__global__ __launch_bounds__(256) void k_gram_reduce(const int32_t *__restrict__ rows,
                                                     const int32_t *__restrict__ row_task,
                                                     int64_t task_base, GT *G) {
  const int64_t row = rows[blockIdx.x];
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= RP * RP || e / RP > e % RP) return;  // upper triangle only
  const int32_t t0 = row_task[row], t1 = row_task[row + 1];
  const GT *g = G + ((int64_t)t0 - task_base) * (RP * RP) + e;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const int n = t1 - t0;
  int q = 0;
  for (; q + 4 <= n; q += 4) {
    s0 += (double)g[(int64_t)q * (RP * RP)];
    s1 += (double)g[(int64_t)(q + 1) * (RP * RP)];
    s2 += (double)g[(int64_t)(q + 2) * (RP * RP)];
    s3 += (double)g[(int64_t)(q + 3) * (RP * RP)];
  }
  for (; q < n; ++q) s0 += (double)g[(int64_t)q * (RP * RP)];
  G[((int64_t)t0 - task_base) * (RP * RP) + e] = (GT)((s0 + s1) + (s2 + s3));
}

// FP64 storage and accumulation: 16x16x4 FP64 tiles of the upper triangle.
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
        for (int bb = a; bb < TB; ++bb) {
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
    for (int bb = a; bb < TB; ++bb) {
      // v_mfma_f64_16x16x4f64 result: D[row][col] at col = lane % 16,
      // row = 4 * v + lane / 16 (checked on the device); tile (a, bb) is
      // block (a, bb) of the upper triangle
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 4 * v + lane / 16, col = lane % 16;
        G[(16 * a + row) * RP + 16 * bb + col] = c[q][v];
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
  void *Lstore;              // I x RP (RP + 1) / 2 packed factors, Gram dtype (optional)
  int factor_only;
  const double *skip;
};

// Pivot of step k: 1 / sqrt(d) for d > 0.  The hardware reciprocal square
// root estimate is refined by two Newton steps y <- y + y (1 - d y^2) / 2
// (each squares the relative error, so the result is within a few ulp).
// Pivots below 2^-900 are scaled by 2^960 first and the result by 2^480
// (both exact), so d y^2 neither underflows nor overflows.
__device__ __forceinline__ double rsqrt_pivot(double d) {
  const bool tiny = d < 0x1p-900;
  const double ds = tiny ? d * 0x1p960 : d;
  double y = __builtin_amdgcn_rsq(ds);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-ds, y * y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return tiny ? y * 0x1p480 : y;
}

// Cholesky of the lane-distributed matrix s (lane i = row i), in place:
// afterwards s[j] on lane i holds L(i, j) for j <= i and 0 for j > i.
// Column k of L is published through LDS (`col`, RP doubles) and read back
// as broadcasts, so the trailing update of step k is RP-k-1 independent FMAs
// per lane (lanes above the diagonal multiply by 0).  Look-ahead: step k
// updates column k+1 first and computes pivot k+1 from it, so the pivot's
// dependent chain overlaps the rest of step k's update; the test of that
// pivot closes the step.  The workgroup is one wave, whose LDS accesses
// complete in program order, so the broadcast needs no barrier.  Returns
// info (LAPACK potrf convention: the order of the first leading minor that
// is not positive definite).
template <int RP>
__device__ __forceinline__ int chol_lanes(double (&s)[RP], int lane, double *col,
                                          double &rdiag) {
  double dkk = readlane_d(s[0], 0);
  if (!(dkk > 0.0)) return 1;
  double inv = rsqrt_pivot(dkk);
#pragma unroll
  for (int k = 0; k < RP; ++k) {
    if (lane == k) rdiag = inv;
    const double lik = lane >= k ? s[k] * inv : 0.0;
    s[k] = lik;
    if (k + 1 < RP) {
      if (lane < RP) col[lane] = lik;
      s[k + 1] -= lik * col[k + 1];
      dkk = readlane_d(s[k + 1], k + 1);
      inv = rsqrt_pivot(dkk);
#pragma unroll
      for (int j = k + 2; j < RP; ++j) s[j] -= lik * col[j];
      if (!(dkk > 0.0)) return k + 2;
    }
  }
  return 0;
}

// A copy of the lane index that the compiler cannot identify with the
// original (an empty asm statement owns it), so lane comparisons in different
// phases of a kernel are not merged and kept alive as masks across them.
__device__ __forceinline__ int opaque_lane(int lane) {
  asm volatile("" : "+v"(lane));
  return lane;
}

// Row-packed lower triangle: row i of L at i (i + 1) / 2 .. i (i + 1) / 2 + i.
// The LDS copy holds PS = RP (RP + 1) / 2 entries, a zero at PS and one
// scratch slot per lane after it, so that every lane can issue the same
// loads and stores (no lane-dependent branches around memory operations).
template <int RP>
struct Packed {
  static constexpr int PS = RP * (RP + 1) / 2;
  static constexpr int ZERO = PS;
  static constexpr int LDS = PS + 1 + 64;
};

// Lane i writes its row of L (s[j], j <= i) into the LDS copy and entries
// j > i into its scratch slot; Lp[ZERO] is set to 0.
template <int RP>
__device__ __forceinline__ void put_rows(double *Lp, const double (&s)[RP], int lane_in) {
  using P = Packed<RP>;
  const int lane = opaque_lane(lane_in);
  const int base = lane < RP ? (lane * (lane + 1)) / 2 : 0;
  const int junk = P::ZERO + 1 + lane;
#pragma unroll
  for (int j = 0; j < RP; ++j) {
    const int addr = (j <= lane && lane < RP) ? base + j : junk;
    Lp[addr] = s[j];
  }
  if (lane == 0) Lp[P::ZERO] = 0.0;
}

// Triangular solves with L read from the LDS copy; b on lane i is b_i and
// rdiag on lane i is 1 / L(i, i).  At step k every lane subtracts its
// multiplier times the broadcast pivot value; the multiplier is read from
// Lp[ZERO] (= 0) on the pivot lane and on lanes already solved, so those
// lanes keep their value and the result is b * rdiag at the end.  The
// loops are only partly unrolled: their bodies index nothing by k except
// through LDS addresses.
// Forward substitution L y = b (LT: the LDS copy's element type).
template <int RP, class LT>
__device__ __forceinline__ double fwd_lds(const LT *Lp, double b, double rdiag, int lane) {
  using P = Packed<RP>;
  const int base = lane < RP ? (lane * (lane + 1)) / 2 : 0;
#pragma unroll 8
  for (int k = 0; k < RP; ++k) {
    const double yk = readlane_d(b * rdiag, k);
    const double lik = (double)Lp[(lane > k && lane < RP) ? base + k : P::ZERO];
    b = fma(-lik, yk, b);
  }
  return b * rdiag;
}

// Backward substitution L^T x = y (lane i takes L(k, i), i < k, from row k).
template <int RP, class LT>
__device__ __forceinline__ double bwd_lds(const LT *Lp, double b, double rdiag, int lane) {
  using P = Packed<RP>;
#pragma unroll 8
  for (int k = RP - 1; k >= 0; --k) {
    const double xk = readlane_d(b * rdiag, k);
    const double lki = (double)Lp[lane < k ? (k * (k + 1)) / 2 + lane : P::ZERO];
    b = fma(-lki, xk, b);
  }
  return b * rdiag;
}

template <class GT, class XT, class MT, int RP>
__global__ __launch_bounds__(64, 2) void k_solve_rows(SolveDev d) {
  using P = Packed<RP>;
  __shared__ double Lp[P::LDS];
  __shared__ double col[RP];
  if (d.skip && *d.skip != 0.0) return;
  const int lane = threadIdx.x;
  const int64_t row = d.r0 + blockIdx.x;
  const int R = d.R;
  const int32_t t0 = d.row_task[row];
  int32_t t1 = d.row_task[row + 1];
  if (t1 - t0 > kReduceMin) t1 = t0 + 1;  // pre-reduced by k_gram_reduce
  // lane i reads column i of the task's RP x RP block: G[j][i] for j <= i
  // is the stored upper triangle (= G[i][j]); entries j > i are not written
  // by the Gram kernels and are replaced by 0 below
  double s[RP];
#pragma unroll
  for (int j = 0; j < RP; ++j) s[j] = 0.0;
  const int li = lane < RP ? lane : 0;
  for (int32_t t = t0; t < t1; ++t) {
    const GT *g = reinterpret_cast<const GT *>(d.G) +
                  ((int64_t)t - d.task_base) * (RP * RP) + li;
#pragma unroll
    for (int j = 0; j < RP; ++j) s[j] += (double)g[j * RP];
  }
  // S = G + lambda I on the R x R block, identity on the padding
  {
    const int ln = opaque_lane(lane);
    const bool pad_row = ln >= R;
#pragma unroll
    for (int j = 0; j < RP; ++j) {
      const double v = s[j] + (j == ln ? d.lambda : 0.0);
      const double kept = j > ln ? 0.0 : v;
      s[j] = (pad_row || j >= R) ? (j == ln ? 1.0 : 0.0) : kept;
    }
  }
  double rdiag = 1.0;
  const int info = chol_lanes<RP>(s, lane, col, rdiag);
  if (d.info && lane == 0) d.info[row] = info;
  if (info && d.Lstore) {
    // failed rows keep the identity (no preconditioning for that block)
#pragma unroll
    for (int j = 0; j < RP; ++j) s[j] = (j == lane) ? 1.0 : 0.0;
  }
  put_rows<RP>(Lp, s, lane);
  __syncthreads();
  if (d.Lstore) {
    GT *L = reinterpret_cast<GT *>(d.Lstore) + row * (int64_t)P::PS;
    for (int q = lane; q < P::PS; q += 64) L[q] = (GT)Lp[q];
  }
  if (d.factor_only) return;
  double x = 0.0;
  if (info == 0) {
    const double b = lane < R ? (double)reinterpret_cast<const MT *>(d.rhs)[row * R + lane] : 0.0;
    x = bwd_lds<RP, double>(Lp, fwd_lds<RP, double>(Lp, b, rdiag, lane), rdiag, lane);
  }
  if (lane < R) reinterpret_cast<XT *>(d.X)[row * d.ldX + lane] = from_double<XT>(x);
}

// Apply stored factors to a right-hand side: X = (L L^T)^{-1} rhs.  The
// factors (row-packed, RP (RP + 1) / 2 per row) are stored in the dense
// dtype MT (FP64 for the FP64 form, FP32 otherwise: they only precondition);
// they are copied into LDS in that dtype with coalesced loads and both
// triangular solves run in FP64 from there.
template <class MT, int RP>
__global__ __launch_bounds__(64) void k_apply_rows(const MT *__restrict__ Lstore,
                                                   const void *rhs, void *X, int R,
                                                   const double *skip) {
  using P = Packed<RP>;
  __shared__ MT Lp[P::LDS];
  if (skip && *skip != 0.0) return;
  const int lane = threadIdx.x;
  const int64_t row = blockIdx.x;
  const MT *L = Lstore + row * (int64_t)P::PS;
  // all loads of the row's factor are issued before the first LDS write
  constexpr int NIT = (P::PS + 63) / 64;
  MT v[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int q = lane + 64 * it;
    v[it] = L[q < P::PS ? q : 0];
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int q = lane + 64 * it;
    if (q < P::PS) Lp[q] = v[it];
  }
  if (lane == 0) Lp[P::ZERO] = MT(0);
  __syncthreads();
  const double b = lane < R ? (double)reinterpret_cast<const MT *>(rhs)[row * R + lane] : 0.0;
  const double dg = lane < RP ? (double)Lp[(lane * (lane + 3)) / 2] : 1.0;  // L(i, i)
  const double rdiag = 1.0 / dg;
  const double y = fwd_lds<RP, MT>(Lp, b, rdiag, lane);
  const double x = bwd_lds<RP, MT>(Lp, y, rdiag, lane);
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

template <class TR, int RP, bool VEC>
static void launch_gram_f32_rp(GramDev d, const int32_t *heavy, int64_t nheavy,
                               double light_bytes, double light_flops, double heavy_bytes,
                               double heavy_flops, hipStream_t s) {
  const int64_t n = d.task_end - d.task_base;
  d.split_heavy = 1;
  {
    ProfScope ps("gram_light", s, light_bytes, light_flops);
    k_gram_f32<TR, RP, VEC><<<dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s>>>(d);
  }
  if (nheavy > 0) {
    ProfScope ps("gram_heavy", s, heavy_bytes, heavy_flops);
    k_gram_f32_heavy<TR, RP, VEC>
        <<<dim3((unsigned)nheavy), dim3(64 * TT_GRAM_HEAVY_WAVES), 0, s>>>(d, heavy, nheavy);
  }
}

// Vector loads of VW = RP / 16 entries need R, ldA and both factor bases
// aligned to VW elements.
template <class TR, int RP>
static void launch_gram_f32_vec(const GramDev &d, const int32_t *heavy, int64_t nheavy,
                                double lb, double lf, double hb, double hf, hipStream_t s) {
  constexpr int VW = RP / 16;
  constexpr size_t al = VW * sizeof(typename TR::T);
  const bool vec = d.R % VW == 0 && d.ldA % VW == 0 &&
                   reinterpret_cast<uintptr_t>(d.A0) % al == 0 &&
                   reinterpret_cast<uintptr_t>(d.A1) % al == 0;
  if (vec) launch_gram_f32_rp<TR, RP, true>(d, heavy, nheavy, lb, lf, hb, hf, s);
  else launch_gram_f32_rp<TR, RP, false>(d, heavy, nheavy, lb, lf, hb, hf, s);
}

// Gram of one batch of tasks [task_base, task_end): light tasks one wave
// each, heavy tasks (the `heavy` slice) one workgroup each, then the
// pre-reduction of rows with many tasks (the `multi` slice).
struct GramWork {
  double light_nnz, heavy_nnz, light_tasks, reduce_tasks;
};

static hipError_t launch_gram(tt_dtype fdt, int RP, const GramDev &d, const int32_t *heavy,
                              int64_t nheavy, const int32_t *multi, int64_t nmulti,
                              const int32_t *row_task, const GramWork &wk, hipStream_t s) {
  const int64_t n = d.task_end - d.task_base;
  if (n <= 0) return hipSuccess;
  dim3 g((unsigned)((n + 3) / 4)), b(256);
  const double R = d.R, fb = fdt == TT_F64 ? 8 : (fdt == TT_F32 ? 4 : 2);
  const double gs = fdt == TT_F64 ? 8 : 4, pernz = 8 + (d.w ? gs : 0) + 2 * R * fb;
  const double tile = (double)RP * RP * gs;
  if (fdt == TT_F64) {
    ProfScope ps("gram_light", s, (wk.light_nnz + wk.heavy_nnz) * pernz + wk.light_tasks * tile,
                 (wk.light_nnz + wk.heavy_nnz) * R * (R + 1));
    GramDev d2 = d;
    d2.split_heavy = 0;
    switch (RP) {
      case 16: k_gram_f64<16><<<g, b, 0, s>>>(d2); break;
      case 32: k_gram_f64<32><<<g, b, 0, s>>>(d2); break;
      default: k_gram_f64<64><<<g, b, 0, s>>>(d2); break;
    }
  } else {
    const double lb = wk.light_nnz * pernz + wk.light_tasks * tile;
    const double lf = wk.light_nnz * R * (R + 1);
    const double hb = wk.heavy_nnz * pernz + (double)nheavy * tile;
    const double hf = wk.heavy_nnz * R * (R + 1);
    if (fdt == TT_F32) {
      switch (RP) {
        case 16: launch_gram_f32_vec<TrF32, 16>(d, heavy, nheavy, lb, lf, hb, hf, s); break;
        case 32: launch_gram_f32_vec<TrF32, 32>(d, heavy, nheavy, lb, lf, hb, hf, s); break;
        default: launch_gram_f32_vec<TrF32, 64>(d, heavy, nheavy, lb, lf, hb, hf, s); break;
      }
    } else {
      switch (RP) {
        case 16: launch_gram_f32_vec<TrBF16, 16>(d, heavy, nheavy, lb, lf, hb, hf, s); break;
        case 32: launch_gram_f32_vec<TrBF16, 32>(d, heavy, nheavy, lb, lf, hb, hf, s); break;
        default: launch_gram_f32_vec<TrBF16, 64>(d, heavy, nheavy, lb, lf, hb, hf, s); break;
      }
    }
  }
  if (nmulti > 0) {
    ProfScope ps("gram_reduce", s, wk.reduce_tasks * tile + (double)nmulti * tile,
                 wk.reduce_tasks * RP * RP);
    dim3 gr((unsigned)nmulti, (unsigned)((RP * RP + 255) / 256));
    if (fdt == TT_F64) {
      switch (RP) {
        case 16: k_gram_reduce<double, 16><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (double *)d.G); break;
        case 32: k_gram_reduce<double, 32><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (double *)d.G); break;
        default: k_gram_reduce<double, 64><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (double *)d.G); break;
      }
    } else {
      switch (RP) {
        case 16: k_gram_reduce<float, 16><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (float *)d.G); break;
        case 32: k_gram_reduce<float, 32><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (float *)d.G); break;
        default: k_gram_reduce<float, 64><<<gr, 256, 0, s>>>(multi, row_task, d.task_base, (float *)d.G); break;
      }
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
  gd.split_heavy = 1;

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
    const std::vector<int32_t> &ht = md.h_heavy_task, &mr = md.h_multi_row;
    const int64_t h0 = std::lower_bound(ht.begin(), ht.end(), (int32_t)rt[r0]) - ht.begin();
    const int64_t h1 = std::lower_bound(ht.begin(), ht.end(), (int32_t)rt[r1]) - ht.begin();
    const int64_t q0 = std::lower_bound(mr.begin(), mr.end(), (int32_t)r0) - mr.begin();
    const int64_t q1 = std::lower_bound(mr.begin(), mr.end(), (int32_t)r1) - mr.begin();
    GramWork wk;
    const std::vector<int64_t> &hn = md.h_heavy_nnz;
    wk.heavy_nnz = (double)(hn[h1] - hn[h0]);
    wk.light_nnz = (double)(md.h_task[rt[r1]] - md.h_task[rt[r0]]) - wk.heavy_nnz;
    wk.light_tasks = (double)(rt[r1] - rt[r0]) - (double)(h1 - h0);
    wk.reduce_tasks = 0;
    for (int64_t q = q0; q < q1; ++q) wk.reduce_tasks += rt[mr[q] + 1] - rt[mr[q]];
    hipError_t e = launch_gram(c.fdt, RP, gd, md.d_heavy_task + h0, h1 - h0,
                               md.d_multi_row + q0, q1 - q0, md.d_row_task, wk, s);
    if (e != hipSuccess) return hip_fail(e, "gram kernel");
    sd.task_base = rt[r0];
    sd.r0 = r0;
    const double Rd = c.R, nrow = (double)(r1 - r0);
    ProfScope ps(c.factor_only ? "cholesky_factor" : "cholesky_solve", s,
                 (double)(rt[r1] - rt[r0]) * RP * RP * (double)gsz +
                     nrow * Rd * (double)(gsz + dtype_size(c.fdt)) +
                     (c.Lstore ? nrow * RP * (RP + 1) / 2 * (double)gsz : 0.0),
                 nrow * (Rd * Rd * Rd / 3.0 + (c.factor_only ? 0.0 : 2.0 * Rd * Rd)));
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
