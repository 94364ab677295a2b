// Device code of Solve Factor (Section 3.4), shared by the translation
// units that instantiate its kernels: the Gram accumulation on the matrix
// cores, the FP64 blocked Cholesky and triangular solves, the kernels, and
// the host-side launch helpers of the fused Gram + solve rows (instantiated
// per factor dtype in solve_fused_f32.hip and solve_fused_bf16.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
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
  void *G;                    // workspace: (task - task_base) * gram_task_elems(RP)
  int waves;                  // waves of a heavy-task workgroup (2, 4, 8)
  const float *rhs_t;         // fused right-hand side: observed values, stream order
  double *M;                  // fused right-hand side: (task - task_base) * RP partials
  // Newton form of alternating minimization (WEIGHTED and RHS together):
  // the weights phi''(t, m) and the right-hand-side values phi'(t, m) are
  // evaluated in the pass from the model value m = <A_own[i], h_e> of each
  // nonzero of row i = key[e]
  const void *A_own;          // the updated mode's factor (leading dim ldA)
  const int32_t *key;         // sorted mode index of each nonzero
  int loss;
  const double *skip;         // when set and *skip != 0 the launch is a no-op
  // least-squares form with a model output (RHS without weights): the model
  // value <A_model[i], h_e> of every nonzero, written to model[e] in stream
  // order (TTTP of the factors as they are before the update)
  const void *A_model;
  float *model;
};

// Slot of the lower element (r, c), r >= c, in the lower-tile layout.
__device__ __forceinline__ int lower_slot(int r, int c) {
  const int I = r >> 4, J = c >> 4;
  return 256 * (I * (I + 1) / 2 + J) + 16 * (r & 15) + (c & 15);
}

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

// FP32 / BF16 storage, FP32 accumulation on v_mfma_f32_16x16x32_bf16.
// Vector-fragment layout: lane l = 16 k + i takes nonzero k of each substep
// of four nonzeros and columns VW*i .. VW*i + VW - 1 of its two factor rows
// (VW = RP / 16), read as one vector load.  Register class v of lane (i, k)
// then holds column VW*i + v, so the class pair (p, q) is one 16 x 16 MFMA
// tile (K = 32 nonzeros per step) whose entry (r, c) is
// G[VW*r + p][VW*c + q].  The classes p <= q (VW (VW + 1) / 2 tiles) cover
// every unordered column pair: once when p < q, twice when p == q (only
// r <= c is stored).
template <int RP>
struct GramAcc {
  static constexpr int VW = RP / 16;
  static constexpr int NT = VW * (VW + 1) / 2;
  static constexpr int NV = 4 * NT;
  f32x4 c[NT];
  double m[VW];  // fused right-hand side: sum of t_e h_e over this lane's nonzeros
  __device__ void zero() {
#pragma unroll
    for (int q = 0; q < NT; ++q) c[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < VW; ++v) m[v] = 0.0;
  }
  __device__ float get(int v) const { return c[v / 4][v % 4]; }
  __device__ void set(int v, float x) { c[v / 4][v % 4] = x; }
};


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

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Bits of the leading bf16 part of x (truncation): x minus this part is
// exact in FP32.
__device__ __forceinline__ uint32_t bf16_head(float x) { return __float_as_uint(x) & 0xffff0000u; }

// Two bf16 parts (in the upper halves of a and b) packed as elements
// 2t (a) and 2t + 1 (b) of an MFMA operand word.
__device__ __forceinline__ uint32_t pack_bf16(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x07060302u);
}

// Exact split of x into NP bf16 parts (NP = 3 for any FP32 value; NP = 2 is
// exact for a product of two bf16 values, which has at most 16 significant
// bits): x = sum of the parts, largest first.
template <int NP>
__device__ __forceinline__ void split_bf16(float x, uint32_t (&p)[NP]) {
  // no contraction of the caller's product into the subtractions
#pragma clang fp contract(off)
  float r = x;
#pragma unroll
  for (int i = 0; i + 1 < NP; ++i) {
    p[i] = bf16_head(r);
    r -= __uint_as_float(p[i]);
  }
  // what remains has at most 8 significant bits: a bf16 value as it is
  p[NP - 1] = __float_as_uint(r);
}

// Products of parts kept for h_a h_b^T: part i of the A side times part j of
// the B side, for i + j <= 4 (1-based; the dropped terms are below 2^-24 of
// the product).  With two parts on both sides all four products are kept,
// which is exact.
template <int PA, int PB>
struct PartPairs {
  static constexpr int N = (PA == 2 && PB == 2) ? 4 : (PA == 2 ? 5 : 6);
  __device__ static constexpr int a(int k) {
    return (PA == 2 && PB == 2) ? (k < 2 ? 0 : 1) : (k == 0 ? 0 : k == 1 ? 0 : k == 2 ? 1 : k == 3 ? 0 : k == 4 ? (PA == 3 ? 2 : 1) : 1);
  }
  __device__ static constexpr int b(int k) {
    return (PA == 2 && PB == 2) ? (k % 2) : (k == 0 ? 0 : k == 1 ? 1 : k == 2 ? 0 : k == 3 ? 2 : k == 4 ? (PA == 3 ? 0 : 1) : 1);
  }
};

// Nonzeros [nb, ne) of one row into acc, on v_mfma_f32_16x16x32_bf16.  The
// range is walked in blocks of 64 nonzeros (lane l loads the row offsets of
// the two gathered factor rows and the weight of nonzero base + l,
// coalesced, one block ahead) and steps of 32: a step is 8 substeps of 4
// nonzeros in the vector-fragment layout, so lane (i, k) holds, for column
// class p, the values h_e[VW i + p] of the 8 nonzeros e = 4 s + k
// (s = 0..7).  Those 8 values are exactly the lane's K-run of an MFMA
// operand (lanes 16 g + i take K = 8 g .. 8 g + 7), so the operands are
// built in registers with no transposition.  Each FP32 value is split
// exactly into bf16 parts (three for FP32 factors, two for BF16 factors,
// whose products have 16 significant bits) and the parts' products are
// accumulated in FP32 (PartPairs).  Without per-nonzero weights both
// operands are the parts of h; with weights the B operand is the parts of
// w h.  Columns at or beyond R read a clamped address and hold finite values
// that only reach padding entries of G, which the solve replaces by the
// identity.  Nonzeros past the end of the range (only in the last step)
// read row 0 and are zeroed by their weight or validity.
// MOD = false compiles the model output out (callers that never ask for it).
template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS, bool MOD = true>
__device__ __forceinline__ void gram_accum(const GramDev &d, int64_t nb, int64_t ne,
                                           GramAcc<RP> &acc) {
  // every instantiation (load mode, model output) rounds the same operations
  // the same way: products are not contracted into later additions
#pragma clang fp contract(off)
  using T = typename TR::T;
  constexpr int VW = RP / 16;
  constexpr bool F32 = std::is_same<TR, TrF32>::value;
  constexpr int PA = F32 ? 3 : 2;
  constexpr int PB = WEIGHTED ? 3 : PA;
  // weights and right-hand-side values from the loss at the model value
  constexpr bool NEWTON = WEIGHTED && RHS;
  using PP = PartPairs<PA, PB>;
  const int lane = threadIdx.x & 63;
  const T *A0 = reinterpret_cast<const T *>(d.A0);
  const T *A1 = reinterpret_cast<const T *>(d.A1);
  const int R = d.R;
  const uint32_t ldA = (uint32_t)d.ldA;
  const int kk = lane >> 4;
  const int cb = VW * (lane & 15);
  const int64_t n = ne - nb;
  if (n <= 0) return;
  // NEWTON, or the model output: this lane's columns of the row's own
  // factor row (0 beyond R)
  constexpr bool MODEL = MOD && RHS && !WEIGHTED;  // a model output is possible
  const bool model = MODEL && d.model != nullptr;  // uniform
  float own[VW];
  if constexpr (NEWTON || MODEL) {
    if (NEWTON || model) {
      const uint32_t row = (uint32_t)d.key[nb];
      load_cols<TR, VW, VEC>(reinterpret_cast<const T *>(NEWTON ? d.A_own : d.A_model),
                             row * ldA, cb, R, own);
#pragma unroll
      for (int v = 0; v < VW; ++v) own[v] = cb + v < R ? own[v] : 0.f;
    }
  }
  const int64_t nblk = (n + 63) / 64;
  const int64_t nst = (n + 31) / 32;
  const bool ragged = (n & 31) != 0;  // the last step has nonzeros past the end

  auto load_block = [&](int64_t blk, uint32_t &r0, uint32_t &r1, float &w, float &tv) {
    const int64_t e = nb + blk * 64 + lane;
    if (e < ne) {
      r0 = (uint32_t)d.oidx0[e] * ldA;
      r1 = (uint32_t)d.oidx1[e] * ldA;
      w = WEIGHTED ? weight_at<float>(d, e) : 1.f;
      tv = RHS ? d.rhs_t[e] : 0.f;
    } else {
      r0 = 0; r1 = 0; w = 0.f; tv = 0.f;
    }
  };
  uint32_t cr0, cr1, nr0 = 0, nr1 = 0;
  float cw, nw = 0.f, ct, nt = 0.f;
  load_block(0, cr0, cr1, cw, ct);
  if (nblk > 1) load_block(1, nr0, nr1, nw, nt);
  int64_t cblk = 0;

  // one step; only the last step of a ragged range (TAIL) has nonzeros past
  // the end, so the others carry no validity code
  auto step = [&](int64_t st, auto tail_tag) {
    constexpr bool tail = decltype(tail_tag)::value;
    const int64_t blk = st >> 1;
    if (blk != cblk) {  // advance cur to blk (== cblk + 1), prefetch the next
      cr0 = nr0; cr1 = nr1; cw = nw; ct = nt;
      cblk = blk;
      if (blk + 1 < nblk) load_block(blk + 1, nr0, nr1, nw, nt);
    }
    const int sb = 32 * (int)(st & 1) + kk;
    uint32_t r0[8], r1[8];
    float w[8], tv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      r0[u] = __shfl(cr0, sb + 4 * u);
      r1[u] = __shfl(cr1, sb + 4 * u);
      w[u] = (WEIGHTED || tail) ? __shfl(cw, sb + 4 * u) : 1.f;
      if (RHS) tv[u] = __shfl(ct, sb + 4 * u);  // 0 past the end
    }
    float a0[8][VW], a1[8][VW];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      load_cols<TR, VW, VEC>(A0, r0[u], cb, R, a0[u]);
      load_cols<TR, VW, VEC>(A1, r1[u], cb, R, a1[u]);
    }
    __builtin_amdgcn_sched_barrier(0);
    // the model output: each substep's nonzero (the 16 lanes of a DPP row
    // hold its columns) gets <own, h_e>; lane 16 k of the row stores it
    if constexpr (MODEL) {
      if (model) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          float dsum = 0.f;
#pragma unroll
          for (int v = 0; v < VW; ++v) dsum = fmaf(own[v], a0[u][v] * a1[u][v], dsum);
          const float m = group_sum<16>(dsum);
          const int64_t e = nb + cblk * 64 + sb + 4 * u;
          if ((lane & 15) == 0 && e < ne) d.model[e] = m;
        }
      }
    }
    // NEWTON: model value of each substep's nonzero (the 16 lanes of a DPP
    // row hold its columns), then phi'' as the weight and phi' as the
    // right-hand-side value; both vanish past the end of the range
    if constexpr (NEWTON) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        float dsum = 0.f;
#pragma unroll
        for (int v = 0; v < VW; ++v) dsum = fmaf(own[v], a0[u][v] * a1[u][v], dsum);
        const float m = group_sum<16>(dsum);
        const float ok = w[u];  // 1 inside the range, 0 past its end
        const float t = tv[u];
        tv[u] = ok * loss_eval<float>(EPI_DPHI, d.loss, t, m);
        w[u] = ok * loss_eval<float>(EPI_D2PHI, d.loss, t, m);
      }
    }
    // operand words: [class][part][word], word t holds substeps 2t, 2t + 1
    uint32_t opa[VW][PA][4], opb[VW][PB][4];
    // fused right-hand side: the step's 8 terms per column in FP32, then one
    // FP64 addition per step
    float mstep[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) mstep[v] = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < VW; ++v) {
        uint32_t pa[2][PA], pb[2][PB];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int u = 2 * t + q;
          float h = a0[u][v] * a1[u][v];
          if constexpr (RHS) mstep[v] = fmaf(tv[u], h, mstep[v]);
          if constexpr (WEIGHTED) {
            split_bf16<PA>(h, pa[q]);
            split_bf16<PB>(w[u] * h, pb[q]);
          } else {
            if (tail) h *= w[u];  // validity (1 or 0)
            split_bf16<PA>(h, pa[q]);
          }
        }
#pragma unroll
        for (int i = 0; i < PA; ++i) opa[v][i][t] = pack_bf16(pa[0][i], pa[1][i]);
        if constexpr (WEIGHTED) {
#pragma unroll
          for (int i = 0; i < PB; ++i) opb[v][i][t] = pack_bf16(pb[0][i], pb[1][i]);
        }
      }
    if constexpr (RHS) {
#pragma unroll
      for (int v = 0; v < VW; ++v) acc.m[v] += (double)mstep[v];
    }
    int q = 0;
#pragma unroll
    for (int p = 0; p < VW; ++p)
#pragma unroll
      for (int pp = p; pp < VW; ++pp) {
#pragma unroll
        for (int k = 0; k < PP::N; ++k) {
          const int ia = PP::a(k), ib = PP::b(k);
          const u32x4 wa = {opa[p][ia][0], opa[p][ia][1], opa[p][ia][2], opa[p][ia][3]};
          u32x4 wb;
          if constexpr (WEIGHTED)
            wb = (u32x4){opb[pp][ib][0], opb[pp][ib][1], opb[pp][ib][2], opb[pp][ib][3]};
          else
            wb = (u32x4){opa[pp][ib][0], opa[pp][ib][1], opa[pp][ib][2], opa[pp][ib][3]};
          acc.c[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf16x8, wa), __builtin_bit_cast(bf16x8, wb), acc.c[q], 0, 0, 0);
        }
        ++q;
      }
    __builtin_amdgcn_sched_barrier(0);
  };
  const int64_t nfull = ragged ? nst - 1 : nst;
  for (int64_t st = 0; st < nfull; ++st) step(st, std::false_type{});
  if (ragged) step(nst - 1, std::true_type{});
}

// Waves per SIMD the Gram kernels are compiled for: at RP = 64 the
// unweighted forms fit 3 (register-limited otherwise to 2), which hides
// more of the gather latency of each 32-nonzero step.
template <int RP, bool WEIGHTED>
struct GramOcc {
  static constexpr int value = (RP == 64 && !WEIGHTED) ? 3 : 1;
};

// Write G in the lower-tile layout from the accumulators (each unordered
// column pair once).  v_mfma_f32_16x16x32_bf16 result: lane l, register v
// holds D[4 (l / 16) + v][l % 16].
template <int RP>
__device__ __forceinline__ void gram_store(float *G, const GramAcc<RP> &acc, float scale) {
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
        if (p < pp || r <= c) G[lower_slot(max(a, b), min(a, b))] = acc.c[q][v] * scale;
      }
      ++q;
    }
}

// Light tasks of rows with several tasks (the `tasks` list): one wave per
// task, four tasks per workgroup.  Rows whose only task is light form their
// Gram inside k_solve_solo; tasks above the light threshold (tuning
// gram_light) go to k_gram_f32_heavy.
// Fused right-hand side of one task: lanes l, l + 16, l + 32, l + 48 hold
// the same columns for different nonzeros; their FP64 sums are added in a
// fixed butterfly and lanes 0..15 store the task's RP partial entries.
template <int RP>
__device__ __forceinline__ void rhs_store(double *M, const GramAcc<RP> &acc, int lane) {
  constexpr int VW = RP / 16;
#pragma unroll
  for (int v = 0; v < VW; ++v) {
    double x = acc.m[v];
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    if (lane < 16) M[VW * lane + v] = x;
  }
}

// MOD (the Gram kernels and k_gram_solve_heavy): compiled with the model
// output; the launches take the variant without it when none is asked for,
// which keeps its registers free for the gathers.
template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS, bool MOD>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(GramOcc<RP, WEIGHTED>::value))) void k_gram_f32(
    GramDev d, const int32_t *tasks, int64_t ntasks) {
  if (d.skip && *d.skip != 0.0) return;
  const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= ntasks) return;
  const int64_t t = tasks[q];
  const int64_t nb = d.task[t], ne = d.task[t + 1];
  GramAcc<RP> acc;
  acc.zero();
  gram_accum<TR, RP, VEC, WEIGHTED, RHS, MOD>(d, nb, ne, acc);
  gram_store<RP>(reinterpret_cast<float *>(d.G) + (t - d.task_base) * (int64_t)gram_task_elems(RP), acc,
                 d.w ? 1.f : (float)d.w_scale);
  if constexpr (RHS) rhs_store<RP>(d.M + (t - d.task_base) * (int64_t)RP, acc, threadIdx.x & 63);
}

// Heavy tasks: the waves of a workgroup split the task's nonzeros and add
// their accumulators through LDS in wave order (deterministic).
template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS, int NW, bool MOD>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(GramOcc<RP, WEIGHTED>::value))) void k_gram_f32_heavy(
    GramDev d, const int32_t *heavy, int64_t nheavy) {
  constexpr int NV = GramAcc<RP>::NV;
  constexpr int VW = RP / 16;
  __shared__ float buf[NV * 64];
  __shared__ double mbuf[RHS ? VW * 64 : 1];
  if (d.skip && *d.skip != 0.0) return;  // uniform over the workgroup
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = heavy[blockIdx.x];
  const int64_t nb = d.task[t], ne = d.task[t + 1];
  const int64_t per = (((ne - nb) + NW - 1) / NW + 3) & ~(int64_t)3;
  const int64_t b0 = min(ne, nb + w * per), b1 = min(ne, b0 + per);
  GramAcc<RP> acc;
  acc.zero();
  gram_accum<TR, RP, VEC, WEIGHTED, RHS, MOD>(d, b0, b1, acc);
  for (int q = 0; q < NW; ++q) {
    if (w == q) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        buf[v * 64 + lane] = (q == 0 ? 0.f : buf[v * 64 + lane]) + acc.get(v);
      if constexpr (RHS) {
#pragma unroll
        for (int v = 0; v < VW; ++v)
          mbuf[v * 64 + lane] = (q == 0 ? 0.0 : mbuf[v * 64 + lane]) + acc.m[v];
      }
    }
    __syncthreads();
  }
  if (w == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc.set(v, buf[v * 64 + lane]);
    gram_store<RP>(reinterpret_cast<float *>(d.G) + (t - d.task_base) * (int64_t)gram_task_elems(RP), acc,
                 d.w ? 1.f : (float)d.w_scale);
    if constexpr (RHS) {
#pragma unroll
      for (int v = 0; v < VW; ++v) acc.m[v] = mbuf[v * 64 + lane];
      rhs_store<RP>(d.M + (t - d.task_base) * (int64_t)RP, acc, lane);
    }
  }
}

// Rows with more than kReduceMin tasks: sum their tasks' fused right-hand
// side partials in FP64 into the first task's slot.  The 256 threads take
// the row's tasks in 4 strided sets of 64 lanes (lane = column), each with 4
// independent partial sums, combined in a fixed order (deterministic).
template <int RP>
__global__ __launch_bounds__(256) void k_rhs_reduce(const int32_t *__restrict__ rows,
                                                    const int32_t *__restrict__ row_task,
                                                    int64_t task_base, double *M,
                                                    const double *skip) {
  __shared__ double part[4][64];
  if (skip && *skip != 0.0) return;
  const int64_t row = rows[blockIdx.x];
  const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int32_t t0 = row_task[row], t1 = row_task[row + 1];
  double *m = M + ((int64_t)t0 - task_base) * RP;
  const int n = t1 - t0;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (c < RP) {
    int q = g;
    for (; q + 12 < n; q += 16) {
      s0 += m[(int64_t)q * RP + c];
      s1 += m[(int64_t)(q + 4) * RP + c];
      s2 += m[(int64_t)(q + 8) * RP + c];
      s3 += m[(int64_t)(q + 12) * RP + c];
    }
    for (; q < n; q += 4) s0 += m[(int64_t)q * RP + c];
  }
  part[g][c] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (g == 0 && c < RP) m[c] = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
}

// Rows with more than kReduceMin tasks: sum their tasks' Grams entrywise
// (lower-tile layout) in FP64, in task order, into the row's first task slot.
template <class GT, int RP>
__global__ __launch_bounds__(256) void k_gram_reduce(const int32_t *__restrict__ rows,
                                                     const int32_t *__restrict__ row_task,
                                                     int64_t task_base, GT *G,
                                                     const double *skip) {
  constexpr int SZ = 128 * (RP / 16) * (RP / 16 + 1);
  if (skip && *skip != 0.0) return;
  const int64_t row = rows[blockIdx.x];
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= SZ) return;
  const int32_t t0 = row_task[row], t1 = row_task[row + 1];
  const GT *g = G + ((int64_t)t0 - task_base) * SZ + e;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  const int n = t1 - t0;
  int q = 0;
  for (; q + 4 <= n; q += 4) {
    s0 += (double)g[(int64_t)q * SZ];
    s1 += (double)g[(int64_t)(q + 1) * SZ];
    s2 += (double)g[(int64_t)(q + 2) * SZ];
    s3 += (double)g[(int64_t)(q + 3) * SZ];
  }
  for (; q < n; ++q) s0 += (double)g[(int64_t)q * SZ];
  G[((int64_t)t0 - task_base) * SZ + e] = (GT)((s0 + s1) + (s2 + s3));
}

// FP64 storage and accumulation: 16x16x4 FP64 tiles of the upper triangle.
template <int RP>
__global__ __launch_bounds__(256) void k_gram_f64(GramDev d) {
  constexpr int TB = RP / 16;
  constexpr int NT = TB * (TB + 1) / 2;
  if (d.skip && *d.skip != 0.0) return;
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
  double *G = reinterpret_cast<double *>(d.G) + (t - d.task_base) * (int64_t)gram_task_elems(RP);
  int q = 0;
#pragma unroll
  for (int a = 0; a < TB; ++a)
#pragma unroll
    for (int bb = a; bb < TB; ++bb) {
      // v_mfma_f64_16x16x4f64 result: D[row][col] at col = lane % 16,
      // row = 4 * v + lane / 16 (checked on the device); tile (a, bb) is
      // block (a, bb) of the upper triangle, stored transposed as the lower
      // element (16 bb + col, 16 a + row)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 4 * v + lane / 16, col = lane % 16;
        if (a < bb || col >= row) G[lower_slot(16 * bb + col, 16 * a + row)] = c[q][v];
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
  const int32_t *rows;       // rows of the launch (NULL: r0 + position)
  int64_t nrow;              // rows of the launch; the grid strides over them
  int64_t grid_max;          // host side: 0, or the persistent grid size
  const int32_t *row_task;   // I + 1
  int64_t task_base;
  int64_t r0;                // first row of the batch
  const void *G;             // Gram workspace (float or double per dtype)
  int R;
  double lambda;
  const void *rhs;           // I x R dense dtype
  const double *M;           // fused right-hand side partials per task, or NULL
  void *X;                   // I x R in storage dtype, leading dim ldX
  int64_t ldX;
  int32_t *info;
  void *Lstore;              // I x RP (RP + 1) / 2 packed factors, Gram dtype (optional)
  int factor_only;
  const double *skip;
  // Newton form of alternating minimization: the fused right-hand side M
  // holds the row gradients' loss part, and the system is solved for
  // -(M_i + own_coef * own[i]) (own: the updated factor, leading dim ldX)
  const void *own;
  double own_coef;
};

// Right-hand side of lane i (< R) in the Newton form: -(m + c own[row, i]).
template <class XT>
__device__ __forceinline__ double newton_rhs(const SolveDev &d, int64_t row, int lane, double m) {
  const XT u = reinterpret_cast<const XT *>(d.own)[row * d.ldX + lane];
  return -(m + d.own_coef * to_double<XT>(u));
}

// Pivot of step k: 1 / sqrt(d) for d > 0 (d is the broadcast pivot, the
// same on every lane).  The hardware reciprocal square root estimate is
// refined by NIT Newton steps y <- y + y (1 - d y^2) / 2, each of which
// squares the relative error: two give a result within a few ulp; one, from
// the estimate's ~2^-22, leaves ~2^-43, which is what the FP32 and BF16
// forms' solves use (a relative error below 1e-12 in each column of L is a
// backward error of the same size, far below their tolerance).  Pivots
// below 2^-900 are scaled by 2^960 first and the result by 2^480 (both
// exact), so d y^2 neither underflows nor overflows.
template <int NIT>
__device__ __forceinline__ double rsqrt_newton(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const double e = fma(-d, y * y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}
template <int NIT>
__device__ __forceinline__ double rsqrt_pivot(double d) {
  // selects rather than a branch: one estimate and refinement per pivot
  const bool tiny = d < 0x1p-900;
  const double y = rsqrt_newton<NIT>(tiny ? d * 0x1p960 : d);
  return tiny ? y * 0x1p480 : y;
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

// Panel buffer of the blocked Cholesky: four columns of PP doubles (column
// c at c * PP, then 64 scratch slots).  PP is RP + 16 rounded so that
// 2 PP = 32 (mod 64): the 16-lane groups of a half-wave that read
// neighbouring columns fall on disjoint LDS bank halves.
template <int RP>
struct PanelBuf {
  static constexpr int PP = RP == 16 ? 48 : RP + 16;
  static constexpr int SCR = 4 * PP;
  static constexpr int SIZE = 4 * PP + 64;
};

// Backward substitution L^T x = y as bwd_lds, with lane i's column
// L(k > i, i) copied from LDS into registers first (the factorization's
// accumulator registers are free by then), so the steps touch no memory.
template <int RP>
__device__ __forceinline__ double bwd_regs(const double *Lp, double b, double rdiag, int lane) {
  using P = Packed<RP>;
  double lcol[RP];
#pragma unroll
  for (int k = 0; k < RP; ++k) lcol[k] = Lp[lane < k ? (k * (k + 1)) / 2 + lane : P::ZERO];
#pragma unroll
  for (int k = RP - 1; k >= 0; --k) {
    const double xk = readlane_d(b * rdiag, k);
    b = fma(-lcol[k], xk, b);
  }
  return b * rdiag;
}

// Blocked Cholesky of one row's S = G + lambda I on the matrix cores.
// S lives in NT accumulator tiles (lower tiles, layout of the Gram
// workspace): lane l, register v of tile (I, J) holds
// S(16 I + 4 v + l / 16, 16 J + l % 16).  For each panel of four columns
// k0 .. k0 + 3 (inside column block J = k0 / 16):
//   1. the lanes holding the panel's columns write them to the LDS panel
//      buffer Pn (column-major, PanelBuf);
//   2. lane i reads row i of the panel and the panel is factored on the
//      lanes (pivot from the diagonal lane, reciprocal square root, the
//      three in-panel updates with broadcast multipliers);
//   3. the factored panel L_p goes back to Pn and into the row-packed LDS
//      copy Lp of L;
//   4. the trailing update S(I, J') -= L_p(I) L_p(J')^T for J <= J' <= I
//      runs as v_mfma_f64_16x16x4f64 with K = the panel's four columns,
//      operand L_p(I) read from Pn (lane l: L(16 I + l % 16, k0 + l / 16)).
// Entries of already factored columns in a tile are updated too but never
// read again.  The workgroup is one wave, whose LDS accesses complete in
// program order, so the buffers need no barriers.  Returns info (LAPACK
// potrf convention) and leaves 1 / L(i, i) in rdiag on lane i.
// FWD: the forward substitution L y = b runs with the factorization (lane i
// holds b_i; at pivot k, y_k = b_k / L(k, k) is broadcast and lanes i > k
// subtract L(i, k) y_k, the multiplier they have just computed), so b
// holds y on return.
// The row's Gram is the sum of `ntask` consecutive tile-layout matrices at
// gbase (task workspace, or the LDS copy of a Gram formed in the kernel).
// REGL (the FP32 and BF16 forms' solo-row kernels): one Newton step per
// pivot (rsqrt_pivot); no LDS copy of L; after each panel's trailing update
// the factored columns are written back from the panel buffer into the
// tiles of column block J (replacing what the update left there), so on
// return tile (I, J)
// holds L in the accumulator layout, zero above the diagonal (bwd_acc,
// store_acc read it from there).
template <int RP>
constexpr int chol_nt() {
  return (RP / 16) * (RP / 16 + 1) / 2;
}

// S = sum of the task Grams + lambda I in the accumulator tiles (identity on
// the padding rows and columns, zero above the diagonal).
template <class GT, int RP>
__device__ __forceinline__ void chol_load(f64x4 (&acc)[chol_nt<RP>()], const GT *gbase,
                                          int ntask, int R, double lambda, int lane) {
  constexpr int NB = RP / 16;
  constexpr int NT = NB * (NB + 1) / 2;
  constexpr int SZ = 256 * NT;
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = (f64x4){0.0, 0.0, 0.0, 0.0};
  for (int t = 0; t < ntask; ++t) {
    const GT *g = gbase + (int64_t)t * SZ + lane;
#pragma unroll
    for (int q = 0; q < NT; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[q][v] += (double)g[256 * q + 64 * v];
  }
  // the Gram may live in LDS that the factorization overwrites: no later
  // memory access moves above these loads (a wave's LDS accesses complete in
  // program order)
  asm volatile("" ::: "memory");
  {
    // shift, identity on the padding, zero above the diagonal of the
    // diagonal tiles (those slots are not written by the Gram kernels)
    const int ln = opaque_lane(lane);
    const int rr = ln >> 4, cc = ln & 15;
    // the diagonal (and the unwritten upper slots) only occur in the
    // diagonal tiles I == J
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double x = acc[I * (I + 1) / 2 + I][v];
        x = (4 * v + rr < cc) ? 0.0 : x;
        x += (4 * v + rr == cc) ? lambda : 0.0;
        acc[I * (I + 1) / 2 + I][v] = x;
      }
    if (R < RP) {  // uniform: padding rows and columns become the identity
#pragma unroll
      for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * I + 4 * v + rr, c = 16 * J + cc;
            const double x = acc[I * (I + 1) / 2 + J][v];
            acc[I * (I + 1) / 2 + J][v] = (r >= R || c >= R) ? (r == c ? 1.0 : 0.0) : x;
          }
    }
  }
}

template <int RP, bool FWD, bool REGL>
__device__ __forceinline__ int chol_core(f64x4 (&acc)[chol_nt<RP>()], int lane, double *Lp,
                                         double *Pn, double &rdiag, double &b) {
  constexpr int NB = RP / 16;
  using P = Packed<RP>;
  using PB = PanelBuf<RP>;
  // every lane of the wave is a row when RP = 64: the lane < RP tests fold
  constexpr bool FULL = RP == 64;
  const int base = (FULL || lane < RP) ? (lane * (lane + 1)) / 2 : 0;
#pragma unroll
  for (int p = 0; p < RP / 4; ++p) {
    const int k0 = 4 * p, J = k0 / 16, c0 = k0 % 16;
    {
      // 1. panel columns to Pn (lanes whose column is outside the panel
      // write to their scratch slot)
      const int ln = opaque_lane(lane);
      const int cc = ln & 15, rr = ln >> 4;
      const bool mine = (unsigned)(cc - c0) < 4u;
#pragma unroll
      for (int I = J; I < NB; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int addr = mine ? (cc - c0) * PB::PP + 16 * I + 4 * v + rr : PB::SCR + ln;
          Pn[addr] = acc[I * (I + 1) / 2 + J][v];
        }
    }
    // 2. factor the panel on the lanes
    double x[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double xv = Pn[c * PB::PP + lane];  // in bounds for every lane
      x[c] = (FULL || lane < RP) ? xv : 0.0;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = k0 + c;
      const double dkk = readlane_d(x[c], k);
      if (!(dkk > 0.0)) return k + 1;
      const double inv = rsqrt_pivot<REGL ? 1 : 2>(dkk);
      if (lane == k) rdiag = inv;
      const double lik = lane >= k ? x[c] * inv : 0.0;
      x[c] = lik;
      if constexpr (FWD) {
        // lik is exactly 0 on the lanes above k, which keep their b
        const double yk = readlane_d(b, k) * inv;
        b = lane == k ? yk : fma(-lik, yk, b);
      }
#pragma unroll
      for (int c2 = c + 1; c2 < 4; ++c2) x[c2] = fma(-lik, readlane_d(lik, k0 + c2), x[c2]);
    }
    // 3. the factored panel to Pn and to the row-packed copy of L
    {
      const int ln = opaque_lane(lane);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        Pn[(FULL || ln < RP) ? c * PB::PP + ln : PB::SCR + ln] = x[c];
        if constexpr (!REGL)
          Lp[(k0 + c <= ln && (FULL || ln < RP)) ? base + k0 + c : P::ZERO + 1 + ln] = x[c];
      }
    }
    // 4. trailing update on the matrix cores
    if (k0 + 4 < RP) {
      double a[NB];
#pragma unroll
      for (int I = J; I < NB; ++I) a[I] = Pn[(lane >> 4) * PB::PP + 16 * I + (lane & 15)];
#pragma unroll
      for (int I = J; I < NB; ++I)
#pragma unroll
        for (int J2 = J; J2 <= I; ++J2)
          acc[I * (I + 1) / 2 + J2] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              -a[I], a[J2], acc[I * (I + 1) / 2 + J2], 0, 0, 0);
    }
    if constexpr (REGL) {
      // 5. the factored panel into the tiles of column block J (lanes whose
      // column is outside the panel read their scratch slot and keep theirs)
      const int ln = opaque_lane(lane);
      const int cc = ln & 15, rr = ln >> 4;
      const bool mine = (unsigned)(cc - c0) < 4u;
#pragma unroll
      for (int I = J; I < NB; ++I)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double y = Pn[mine ? (cc - c0) * PB::PP + 16 * I + 4 * v + rr : PB::SCR + ln];
          acc[I * (I + 1) / 2 + J][v] = mine ? y : acc[I * (I + 1) / 2 + J][v];
        }
    }
  }
  return 0;
}

template <class GT, int RP, bool FWD>
__device__ __forceinline__ int chol_tiles(const SolveDev &d, const GT *gbase, int ntask,
                                          int lane, double *Lp, double *Pn,
                                          double &rdiag, double &b) {
  f64x4 acc[chol_nt<RP>()];
  chol_load<GT, RP>(acc, gbase, ntask, d.R, d.lambda, lane);
  return chol_core<RP, FWD, false>(acc, lane, Lp, Pn, rdiag, b);
}

// Buffer of bwd_acc: a diagonal tile row-major (256), a zero, the block's x.
struct BwdBuf {
  static constexpr int ZERO = 256;
  static constexpr int X = 264;
  static constexpr int SIZE = 280;
};

// Backward substitution L^T x = y with L in the accumulator tiles (lane l,
// register v of tile (I, J): L(16 I + 4 v + l / 16, 16 J + l % 16)); lane i
// holds y_i in b and 1 / L(i, i) in rdiag.  Column blocks from the last:
// the diagonal tile goes to the LDS buffer T row-major and the block's 16
// unknowns are solved one after the other (x_k broadcast, lanes c < k of
// the block subtract L(k, c) x_k, the other lanes a zero); then the block's
// x goes to T, and for every block G above it the lanes form their part of
// sum_r L(r, c) x_r over the rows r of block J in tile (J, G), the four
// lane groups add theirs (two butterfly steps) and the lanes of block G
// subtract it.  Returns x_i on lane i.
template <int RP>
__device__ __forceinline__ double bwd_acc(const f64x4 (&acc)[chol_nt<RP>()], double *T,
                                          double b, double rdiag, int lane) {
  constexpr int NB = RP / 16;
  using BB = BwdBuf;
  const int ln = opaque_lane(lane);
  const int rr = ln >> 4, cc = ln & 15;
  // earlier LDS reads (the factorization's) stay before these writes
  asm volatile("" ::: "memory");
  if (lane == 0) T[BB::ZERO] = 0.0;
#pragma unroll
  for (int J = NB - 1; J >= 0; --J) {
    const int dq = J * (J + 1) / 2 + J;
#pragma unroll
    for (int v = 0; v < 4; ++v) T[(4 * v + rr) * 16 + cc] = acc[dq][v];
    asm volatile("" ::: "memory");
    const bool inblk = rr == J;
#pragma unroll 4
    for (int k = 15; k >= 0; --k) {
      const double xk = readlane_d(b * rdiag, 16 * J + k);
      const double lkc = T[(inblk && cc < k) ? k * 16 + cc : BB::ZERO];
      b = fma(-lkc, xk, b);
    }
    if (J > 0) {
      asm volatile("" ::: "memory");
      T[inblk ? BB::X + cc : BB::ZERO + 1 + (ln & 3)] = b * rdiag;
      asm volatile("" ::: "memory");
      double xs[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) xs[v] = T[BB::X + 4 * v + rr];
#pragma unroll
      for (int G = 0; G < J; ++G) {
        const int q = J * (J + 1) / 2 + G;
        double p = acc[q][0] * xs[0];
#pragma unroll
        for (int v = 1; v < 4; ++v) p = fma(acc[q][v], xs[v], p);
        p += __shfl_xor(p, 16);
        p += __shfl_xor(p, 32);
        b = rr == G ? b - p : b;
      }
      // the next block's tile overwrites T: these reads stay before it
      asm volatile("" ::: "memory");
    }
  }
  return b * rdiag;
}

// L from the tiles to the row-packed factor store (RP (RP + 1) / 2 floats
// per row), staged in LDS (Lf: PS + 64 floats) so that the global stores
// are coalesced; info != 0 stores the identity.
template <int RP>
__device__ __forceinline__ void store_acc(const f64x4 (&acc)[chol_nt<RP>()], float *Lf,
                                          float *L, int info, int lane) {
  constexpr int NB = RP / 16;
  constexpr int PS = Packed<RP>::PS;
  const int ln = opaque_lane(lane);
  const int rr = ln >> 4, cc = ln & 15;
  asm volatile("" ::: "memory");
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J <= I; ++J)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * I + 4 * v + rr, c = 16 * J + cc;
        const bool diag = r == c;
        const float y = info ? (diag ? 1.f : 0.f) : (float)acc[I * (I + 1) / 2 + J][v];
        Lf[c <= r ? (r * (r + 1)) / 2 + c : PS + ln] = y;
      }
  asm volatile("" ::: "memory");
  for (int q = lane; q < PS; q += 64) L[q] = Lf[q];
}

// One row of k_solve_rows.
template <class GT, class XT, class MT, int RP>
__device__ __forceinline__ void solve_row(const SolveDev &d, int64_t row, int lane, double *Lp,
                                          double *Pn) {
  using P = Packed<RP>;
  const int R = d.R;
  const int32_t t0 = d.row_task[row];
  int32_t t1 = d.row_task[row + 1];
  if (t1 - t0 > kReduceMin) t1 = t0 + 1;  // pre-reduced by k_gram_reduce
  if (lane == 0) Lp[P::ZERO] = 0.0;
  double rdiag = 1.0;
  // right-hand side (lane i holds b_i); the forward substitution runs inside
  // the factorization
  double b = 0.0;
  if (!d.factor_only) {
    if (d.M) {
      // fused right-hand side: the row's task partials (pre-reduced into the
      // first task for rows with more than kReduceMin tasks), in task order
      if (lane < R) {
        for (int32_t t = t0; t < t1; ++t) b += d.M[((int64_t)t - d.task_base) * RP + lane];
        if (d.own) b = newton_rhs<XT>(d, row, lane, b);
      }
    } else if (lane < R) {
      b = (double)reinterpret_cast<const MT *>(d.rhs)[row * R + lane];
    }
  }
  constexpr int SZ = gram_task_elems(RP);
  const GT *gbase = reinterpret_cast<const GT *>(d.G) + ((int64_t)t0 - d.task_base) * SZ;
  const int info = d.factor_only
                       ? chol_tiles<GT, RP, false>(d, gbase, t1 - t0, lane, Lp, Pn, rdiag, b)
                       : chol_tiles<GT, RP, true>(d, gbase, t1 - t0, lane, Lp, Pn, rdiag, b);
  if (d.info && lane == 0) d.info[row] = info;
  if (info && d.Lstore) {
    // failed rows keep the identity (no preconditioning for that block)
    for (int q = lane; q < P::PS; q += 64) Lp[q] = 0.0;
    if (lane < RP) Lp[(lane * (lane + 3)) / 2] = 1.0;
  }
  if (d.Lstore) {
    GT *L = reinterpret_cast<GT *>(d.Lstore) + row * (int64_t)P::PS;
    for (int q = lane; q < P::PS; q += 64) L[q] = (GT)Lp[q];
  }
  if (d.factor_only) return;
  // b holds y = L^{-1} rhs; backward substitution L^T x = y
  const double x = info == 0 ? bwd_regs<RP>(Lp, b, rdiag, lane) : 0.0;
  if (lane < R) reinterpret_cast<XT *>(d.X)[row * d.ldX + lane] = from_double<XT>(x);
}

// PERSIST: a grid smaller than the row count, each workgroup taking every
// gridDim.x-th row in order (one wave per workgroup, so the LDS is reused
// across rows without barriers); otherwise one workgroup per row.
template <class GT, class XT, class MT, int RP, bool PERSIST>
__global__ __launch_bounds__(64) void k_solve_rows(SolveDev d) {
  using P = Packed<RP>;
  __shared__ double Lp[P::LDS];
  __shared__ double Pn[PanelBuf<RP>::SIZE];
  if (d.skip && *d.skip != 0.0) return;
  if constexpr (PERSIST) {
    for (int64_t idx = blockIdx.x; idx < d.nrow; idx += gridDim.x) {
      // the lane index is re-derived per row (opaque), so the per-lane
      // constants of the unrolled factorization are not held across rows
      const int lane = opaque_lane(threadIdx.x);
      solve_row<GT, XT, MT, RP>(d, d.rows ? (int64_t)d.rows[idx] : d.r0 + idx, lane, Lp, Pn);
      asm volatile("" ::: "memory");
    }
  } else {
    const int64_t idx = blockIdx.x;
    solve_row<GT, XT, MT, RP>(d, d.rows ? (int64_t)d.rows[idx] : d.r0 + idx, threadIdx.x, Lp,
                              Pn);
  }
}

// The tail of a fused Gram + solve: the row's whole Gram (and fused
// right-hand side) is in one wave's accumulators; store the Gram in the tile
// layout into the LDS that the factorization later reuses for L, factor,
// and solve or store the factors.
template <class TR, int RP, bool RHS, bool FO>
__device__ __forceinline__ void solve_from_acc(const GramDev &g, const SolveDev &d, int64_t row,
                                               int lane, double *Lp, double *Pn,
                                               const GramAcc<RP> &acc) {
  using P = Packed<RP>;
  using XT = typename TR::T;
  constexpr int VW = RP / 16;
  static_assert(gram_task_elems(RP) <= 2 * P::PS, "the Gram fits below Lp[ZERO]");
  const int R = d.R;
  // earlier LDS reads (a previous row's, one wave, program order) stay before
  // these writes
  asm volatile("" ::: "memory");
  float *Gl = reinterpret_cast<float *>(Lp);
  gram_store<RP>(Gl, acc, g.w ? 1.f : (float)g.w_scale);
  double b = 0.0;
  if constexpr (RHS) {
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      double x = acc.m[v];
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
      if (lane < 16) Pn[VW * lane + v] = x;
    }
    const double bv = Pn[lane < RP ? lane : 0];
    b = lane < R ? bv : 0.0;
    if (d.own && lane < R) b = newton_rhs<XT>(d, row, lane, b);
  } else if (!FO && lane < R) {
    b = (double)reinterpret_cast<const float *>(d.rhs)[row * R + lane];
  }
  asm volatile("" ::: "memory");
  if (lane == 0) Lp[P::ZERO] = 0.0;
  double rdiag = 1.0;
  const int info = chol_tiles<float, RP, !FO>(d, Gl, 1, lane, Lp, Pn, rdiag, b);
  if (d.info && lane == 0) d.info[row] = info;
  if (info && d.Lstore) {
    for (int q = lane; q < P::PS; q += 64) Lp[q] = 0.0;
    if (lane < RP) Lp[(lane * (lane + 3)) / 2] = 1.0;
  }
  if (d.Lstore) {
    float *L = reinterpret_cast<float *>(d.Lstore) + row * (int64_t)P::PS;
    for (int q = lane; q < P::PS; q += 64) L[q] = (float)Lp[q];
  }
  if constexpr (!FO) {
    const double x = info == 0 ? bwd_regs<RP>(Lp, b, rdiag, lane) : 0.0;
    if (lane < R) reinterpret_cast<XT *>(d.X)[row * d.ldX + lane] = from_double<XT>(x);
  }
}

// LDS of the push-through solve at padded size KP (doubles): K's tiles,
// then (same place) the panel buffer and the backward-solve buffer, then H
// (KP rows of 64 floats).
template <int KP>
struct PushLds {
  static constexpr int K = chol_nt<KP>() * 128;
  static constexpr int PB = PanelBuf<KP>::SIZE > BwdBuf::SIZE ? PanelBuf<KP>::SIZE : BwdBuf::SIZE;
  static constexpr int H = K > PB ? K : PB;
  static constexpr int SIZE = H + KP * 32;
};

// LDS of a k_solve_solo workgroup (doubles): the largest of the Gram in the
// tile layout, the panel buffer, the backward-solve buffer, the factor
// staging (PS + 64 floats) and, for the push-through solves (PUSH), their
// buffers.
template <int RP, bool PUSH>
struct SoloLds {
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int FAC = cmax(cmax(gram_task_elems(RP) / 2, PanelBuf<RP>::SIZE),
                                  cmax(BwdBuf::SIZE, (Packed<RP>::PS + 64 + 1) / 2));
  static constexpr int DOUBLES = PUSH ? cmax(FAC, cmax(PushLds<16>::SIZE, PushLds<32>::SIZE)) : FAC;
};

// Rows of at most 32 nonzeros take the push-through solve in the unweighted
// fused least-squares update at padded rank 64.
template <int RP, bool WEIGHTED, bool RHS, bool FO>
constexpr bool solo_push() {
  return RP == 64 && RHS && !WEIGHTED && !FO;
}

// solve_from_acc with L kept in the accumulator tiles (chol_core REGL) and
// one LDS block `lds` that holds in turn the right-hand side reduction, the
// Gram in the tile layout, the panel buffer, the factor staging and the
// backward-solve buffer (one wave: its LDS accesses complete in program
// order; the empty asm statements keep the compiler from moving them).
template <class TR, int RP, bool RHS, bool FO>
__device__ __forceinline__ void solve_from_acc_regl(const GramDev &g, const SolveDev &d,
                                                    int64_t row, int lane, double *lds,
                                                    const GramAcc<RP> &acc) {
  using XT = typename TR::T;
  constexpr int VW = RP / 16;
  const int R = d.R;
  // earlier LDS reads (a previous row's) stay before these writes
  asm volatile("" ::: "memory");
  double b = 0.0;
  if constexpr (RHS) {
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      double x = acc.m[v];
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
      if (lane < 16) lds[VW * lane + v] = x;
    }
    const double bv = lds[lane < RP ? lane : 0];
    b = lane < R ? bv : 0.0;
    if (d.own && lane < R) b = newton_rhs<XT>(d, row, lane, b);
  } else if (!FO && lane < R) {
    b = (double)reinterpret_cast<const float *>(d.rhs)[row * R + lane];
  }
  // the Gram overwrites the right-hand side buffer
  asm volatile("" ::: "memory");
  float *Gl = reinterpret_cast<float *>(lds);
  gram_store<RP>(Gl, acc, g.w ? 1.f : (float)g.w_scale);
  asm volatile("" ::: "memory");
  f64x4 L[chol_nt<RP>()];
  chol_load<float, RP>(L, Gl, 1, R, d.lambda, lane);
  double rdiag = 1.0;
  const int info = chol_core<RP, !FO, true>(L, lane, nullptr, lds, rdiag, b);
  if (d.info && lane == 0) d.info[row] = info;
  if (d.Lstore)
    store_acc<RP>(L, reinterpret_cast<float *>(lds),
                  reinterpret_cast<float *>(d.Lstore) + row * (int64_t)Packed<RP>::PS, info, lane);
  if constexpr (!FO) {
    const double x = info == 0 ? bwd_acc<RP>(L, lds, b, rdiag, lane) : 0.0;
    if (lane < R) reinterpret_cast<XT *>(d.X)[row * d.ldX + lane] = from_double<XT>(x);
  }
}

// Rows of the fused least-squares update with k <= KP nonzeros (KP = 16 or
// 32) at ranks above 32.  With H the k x R matrix of the rows h_e and c the
// constant weight, (c H^T H + lambda I)^{-1} H^T t = H^T (c H H^T +
// lambda I)^{-1} t for lambda > 0 (push-through identity), so the row's R x
// R system reduces to a k x k one.  K = H H^T is formed on the matrix cores
// from the same exact bf16 splits as the Gram (the contraction now runs
// over the R columns: lane 16 g + i holds columns 8 g .. 8 g + 7 of h_e,
// e = 16 I + i, which is its operand K-run for the tiles of row block I),
// stored in the tile layout, factored (L kept in the accumulator tiles) and
// solved at padded size KP (rows e >= k are the identity), and x = H^T y is
// summed in FP64 from an LDS copy of H.  LDS (`lds`, PushLds<KP>): K's
// tiles, then the panel buffer and the backward-solve buffer in the same
// place, and H after them.
template <class TR, int KP, bool VEC>
__device__ __forceinline__ void solve_pushthrough(const GramDev &g, const SolveDev &d,
                                                  int64_t row, int64_t nb, int k, int lane,
                                                  double *lds) {
  using T = typename TR::T;
  using XT = typename TR::T;
  constexpr bool F32 = std::is_same<TR, TrF32>::value;
  constexpr int PA = F32 ? 3 : 2;
  using PP = PartPairs<PA, PA>;
  constexpr int NB = KP / 16;
  constexpr int NT = NB * (NB + 1) / 2;
  float *Kl = reinterpret_cast<float *>(lds);
  float *Hl = reinterpret_cast<float *>(lds + PushLds<KP>::H);
  const T *A0 = reinterpret_cast<const T *>(g.A0);
  const T *A1 = reinterpret_cast<const T *>(g.A1);
  const int R = d.R;
  const uint32_t ldA = (uint32_t)g.ldA;
  const int gq = lane >> 4, i = lane & 15;
  // earlier LDS reads (a previous row's, one wave, program order) stay before
  // these writes
  asm volatile("" ::: "memory");
  uint32_t op[NB][2][PA][4];
#pragma unroll
  for (int I = 0; I < NB; ++I) {
    const int e = 16 * I + i;
    const bool ok = e < k;
    const int64_t ec = nb + (ok ? e : 0);
    const uint32_t r0 = (uint32_t)g.oidx0[ec] * ldA, r1 = (uint32_t)g.oidx1[ec] * ldA;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int cb = 32 * s + 8 * gq;
      float a0[8], a1[8];
      load_cols<TR, 4, VEC>(A0, r0, cb, R, *reinterpret_cast<float(*)[4]>(a0));
      load_cols<TR, 4, VEC>(A0, r0, cb + 4, R, *reinterpret_cast<float(*)[4]>(a0 + 4));
      load_cols<TR, 4, VEC>(A1, r1, cb, R, *reinterpret_cast<float(*)[4]>(a1));
      load_cols<TR, 4, VEC>(A1, r1, cb + 4, R, *reinterpret_cast<float(*)[4]>(a1 + 4));
      uint32_t pt[8][PA];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float h = (ok && cb + j < R) ? a0[j] * a1[j] : 0.f;
        Hl[e * 64 + cb + j] = h;
        split_bf16<PA>(h, pt[j]);
      }
#pragma unroll
      for (int ii = 0; ii < PA; ++ii)
#pragma unroll
        for (int w = 0; w < 4; ++w) op[I][s][ii][w] = pack_bf16(pt[2 * w][ii], pt[2 * w + 1][ii]);
    }
  }
  // the model output: lane e < k forms <own row, h_e> from the LDS copy of H
  // (FP64 sum, rounded once; the own row is read before this row's update)
  if (g.model != nullptr) {
    asm volatile("" ::: "memory");
    if (lane < k) {
      const T *own = reinterpret_cast<const T *>(g.A_model) + row * (int64_t)ldA;
      double mm = 0.0;
      for (int c = 0; c < R; ++c)
        mm = fma((double)Hl[lane * 64 + c], (double)elem_f<TR>(own, c), mm);
      g.model[nb + lane] = (float)mm;
    }
  }
  f32x4 acc[NT];
#pragma unroll
  for (int q = 0; q < NT; ++q) acc[q] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int I = 0; I < NB; ++I)
#pragma unroll
    for (int J = 0; J <= I; ++J)
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int kk = 0; kk < PP::N; ++kk) {
          const int ia = PP::a(kk), ib = PP::b(kk);
          const u32x4 wa = {op[I][s][ia][0], op[I][s][ia][1], op[I][s][ia][2], op[I][s][ia][3]};
          const u32x4 wb = {op[J][s][ib][0], op[J][s][ib][1], op[J][s][ib][2], op[J][s][ib][3]};
          const int q = I * (I + 1) / 2 + J;
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf16x8, wa), __builtin_bit_cast(bf16x8, wb), acc[q], 0, 0, 0);
        }
  // tile (I, J), register v of lane l: K[16 I + 4 (l / 16) + v][16 J + l % 16],
  // stored row-major in its tile
  const float c = g.w ? 1.f : (float)g.w_scale;
#pragma unroll
  for (int q = 0; q < NT; ++q)
#pragma unroll
    for (int v = 0; v < 4; ++v) Kl[256 * q + 16 * (4 * gq + v) + i] = acc[q][v] * c;
  asm volatile("" ::: "memory");
  double b = lane < k ? (double)g.rhs_t[nb + lane] : 0.0;
  double rdiag = 1.0;
  f64x4 L[NT];
  // rows and columns k .. KP - 1 become the identity
  chol_load<float, KP>(L, Kl, 1, k, d.lambda, lane);
  const int info = chol_core<KP, true, true>(L, lane, nullptr, lds, rdiag, b);
  if (d.info && lane == 0) d.info[row] = info;
  const double y = info == 0 ? bwd_acc<KP>(L, lds, b, rdiag, lane) : 0.0;
  double x = 0.0;
  for (int e = 0; e < k; ++e) x = fma((double)Hl[e * 64 + lane], readlane_d(y, e), x);
  if (lane < R) reinterpret_cast<XT *>(d.X)[row * d.ldX + lane] = from_double<XT>(x);
}

template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS, bool FO, bool MOD>
__device__ __forceinline__ void solve_solo_row(const GramDev &g, const SolveDev &d, int64_t row,
                                               int lane, double *lds) {
  const int32_t t = d.row_task[row];
  if constexpr (solo_push<RP, WEIGHTED, RHS, FO>()) {
    // the least-squares update of a row with at most 32 nonzeros: its k x k
    // system (uniform over the wave)
    const int64_t nb = g.task[t], n = g.task[t + 1] - nb;
    if (d.lambda > 0.0 && d.own == nullptr && n <= 32) {
      if (n <= 16)
        solve_pushthrough<TR, 16, VEC>(g, d, row, nb, (int)n, lane, lds);
      else
        solve_pushthrough<TR, 32, VEC>(g, d, row, nb, (int)n, lane, lds);
      return;
    }
  }
  GramAcc<RP> acc;
  acc.zero();
  gram_accum<TR, RP, VEC, WEIGHTED, RHS, MOD>(g, g.task[t], g.task[t + 1], acc);
  solve_from_acc_regl<TR, RP, RHS, FO>(g, d, row, lane, lds, acc);
}

// Rows whose only Gram task is light (FP32 and BF16 forms): the wave forms
// the row's Gram on the matrix cores (gram_accum), stages it in the tile
// layout in LDS, loads it into the FP64 accumulator tiles and factors and
// solves it there (solve_from_acc_regl: L stays in the tiles), so the Gram
// never goes to the workspace.  The fused right-hand side is reduced over
// the four nonzero groups with the butterfly of rhs_store.  PERSIST as in
// k_solve_rows.
// MOD: the fused update also writes the model values.  Waves per SIMD the
// kernel is compiled for: the variants with a model output, per-nonzero
// weights or the persistent loop need more registers (two), the factor-only
// one fits four (10 KB of LDS at RP = 64), the others three.
#ifndef TT_SOLO_FO_WAVES
#define TT_SOLO_FO_WAVES 4
#endif
template <bool WEIGHTED, bool RHS, bool FO, bool PERSIST, bool MOD>
constexpr int solo_waves() {
  return (PERSIST || MOD || WEIGHTED) ? 2 : (FO && !RHS) ? TT_SOLO_FO_WAVES : 3;
}

template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS, bool FO, bool PERSIST, bool MOD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(
    solo_waves<WEIGHTED, RHS, FO, PERSIST, MOD>()))) void k_solve_solo(GramDev g, SolveDev d) {
  __shared__ double lds[SoloLds<RP, solo_push<RP, WEIGHTED, RHS, FO>()>::DOUBLES];
  if (d.skip && *d.skip != 0.0) return;
  if constexpr (PERSIST) {
    for (int64_t idx = blockIdx.x; idx < d.nrow; idx += gridDim.x) {
      const int lane = opaque_lane(threadIdx.x);  // per row (see k_solve_rows)
      solve_solo_row<TR, RP, VEC, WEIGHTED, RHS, FO, MOD>(g, d, d.rows[idx], lane, lds);
      asm volatile("" ::: "memory");
    }
  } else {
    solve_solo_row<TR, RP, VEC, WEIGHTED, RHS, FO, MOD>(g, d, d.rows[blockIdx.x], threadIdx.x, lds);
  }
}

// Rows whose only Gram task is heavy (FP32 and BF16 forms): the task's
// nonzeros are split over the workgroup's four waves as in
// k_gram_f32_heavy and their accumulators are added in LDS in wave order;
// then wave 0 factors and solves (or stores the factors of) the row from
// the summed accumulators, so neither the Gram nor the right-hand side
// passes through the workspace.  While wave 0 factors, the other waves have
// left and the compute unit's other workgroups keep gathering.  The LDS of
// the wave reduction is reused for the factorization.
template <int RP>
struct HeavySoloLds {
  static constexpr int NV = GramAcc<RP>::NV;
  static constexpr int RED = NV * 64 * 4 + (RP / 16) * 64 * 8;  // floats, then doubles
  static constexpr int FAC = (Packed<RP>::LDS + PanelBuf<RP>::SIZE) * 8;
  static constexpr int DOUBLES = ((RED > FAC ? RED : FAC) + 7) / 8;
};

template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS, bool FO, bool MOD>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(RP == 64 ? 2 : 4))) void k_gram_solve_heavy(GramDev g,
                                                                               SolveDev d) {
  using L = HeavySoloLds<RP>;
  constexpr int NW = 4;
  constexpr int NV = L::NV;
  constexpr int VW = RP / 16;
  __shared__ double lds[L::DOUBLES];
  float *buf = reinterpret_cast<float *>(lds);
  double *mbuf = lds + NV * 64 / 2;
  if (d.skip && *d.skip != 0.0) return;  // uniform over the workgroup
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row = d.rows[blockIdx.x];
  const int32_t t = d.row_task[row];
  const int64_t nb = g.task[t], ne = g.task[t + 1];
  const int64_t per = (((ne - nb) + NW - 1) / NW + 3) & ~(int64_t)3;
  const int64_t b0 = min(ne, nb + w * per), b1 = min(ne, b0 + per);
  GramAcc<RP> acc;
  acc.zero();
  gram_accum<TR, RP, VEC, WEIGHTED, RHS, MOD>(g, b0, b1, acc);
  for (int q = 0; q < NW; ++q) {
    if (w == q) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        buf[v * 64 + lane] = (q == 0 ? 0.f : buf[v * 64 + lane]) + acc.get(v);
      if constexpr (RHS) {
#pragma unroll
        for (int v = 0; v < VW; ++v)
          mbuf[v * 64 + lane] = (q == 0 ? 0.0 : mbuf[v * 64 + lane]) + acc.m[v];
      }
    }
    __syncthreads();
  }
  if (w != 0) return;
#pragma unroll
  for (int v = 0; v < NV; ++v) acc.set(v, buf[v * 64 + lane]);
  if constexpr (RHS) {
#pragma unroll
    for (int v = 0; v < VW; ++v) acc.m[v] = mbuf[v * 64 + lane];
  }
  // the factorization reuses the reduction buffers (one wave from here on:
  // its LDS accesses complete in program order)
  double *Lp = lds;
  double *Pn = lds + Packed<RP>::LDS;
  solve_from_acc<TR, RP, RHS, FO>(g, d, row, lane, Lp, Pn, acc);
}

// Apply stored factors to a right-hand side: X = (L L^T)^{-1} rhs.  The
// factors (row-packed, RP (RP + 1) / 2 per row) are stored in the dense
// dtype MT (FP64 for the FP64 form, FP32 otherwise: they only precondition);
// they are copied into LDS in that dtype with coalesced loads and both
// triangular solves run in FP64 from there.
//
// apply_row solves one row with one wave (lane = threadIdx.x mod 64) and
// the wave's own LDS block Lp; a single wave orders its LDS accesses by
// program order, so only the compiler has to be kept from moving the reads
// of the copy above its writes.
template <class MT, int RP>
__device__ __forceinline__ void apply_row(const MT *__restrict__ Lstore, const void *rhs,
                                          void *X, int R, int64_t row, MT *Lp) {
  using P = Packed<RP>;
  const int lane = threadIdx.x & 63;
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
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  const double b = lane < R ? (double)reinterpret_cast<const MT *>(rhs)[row * R + lane] : 0.0;
  const double dg = lane < RP ? (double)Lp[(lane * (lane + 3)) / 2] : 1.0;  // L(i, i)
  const double rdiag = 1.0 / dg;
  double x;
  if constexpr (sizeof(MT) == 4) {
    // FP32 factors: lane i first copies its row L(i, k < i) and its column
    // L(k > i, i) from LDS into registers (zeros elsewhere), so the two
    // substitutions below touch no memory: each step is the broadcast of
    // y_k (x_k) and one FMA per lane
    MT lrow[RP], lcol[RP];
    const int base = lane < RP ? (lane * (lane + 1)) / 2 : 0;
#pragma unroll
    for (int k = 0; k < RP; ++k) {
      lrow[k] = Lp[(lane > k && lane < RP) ? base + k : P::ZERO];
      lcol[k] = Lp[lane < k ? (k * (k + 1)) / 2 + lane : P::ZERO];
    }
    double bb = b;
#pragma unroll
    for (int k = 0; k < RP; ++k) {
      const double yk = readlane_d(bb * rdiag, k);
      bb = fma(-(double)lrow[k], yk, bb);
    }
    bb *= rdiag;
#pragma unroll
    for (int k = RP - 1; k >= 0; --k) {
      const double xk = readlane_d(bb * rdiag, k);
      bb = fma(-(double)lcol[k], xk, bb);
    }
    x = bb * rdiag;
  } else {
    const double y = fwd_lds<RP, MT>(Lp, b, rdiag, lane);
    x = bwd_lds<RP, MT>(Lp, y, rdiag, lane);
  }
  if (lane < R) reinterpret_cast<MT *>(X)[row * R + lane] = (MT)x;
}

template <class MT, int RP>
__global__ __launch_bounds__(64) void k_apply_rows(const MT *__restrict__ Lstore,
                                                   const void *rhs, void *X, int R,
                                                   const double *skip) {
  __shared__ MT Lp[Packed<RP>::LDS];
  if (skip && *skip != 0.0) return;
  apply_row<MT, RP>(Lstore, rhs, X, R, blockIdx.x, Lp);
}

// ---------------------------------------------------------------------------
static inline int rp_for(int R) { return R <= 16 ? 16 : (R <= 32 ? 32 : 64); }

// One workgroup per row, or a persistent grid of d.grid_max workgroups.
static inline unsigned solve_grid(const SolveDev &d) {
  return (unsigned)(d.grid_max > 0 ? std::min<int64_t>(d.nrow, d.grid_max) : d.nrow);
}

// One batch of the FP32 / BF16 forms: heavy tasks and light tasks of rows
// with several tasks (Gram into the workspace), and the fused Gram + solve
// of the rows whose only task is light (solo) or heavy (hsolo).
struct GramLists {
  const int32_t *heavy, *light, *solo, *hsolo;
  int64_t nheavy, nlight, nsolo, nhsolo;
  double light_bytes, light_flops, heavy_bytes, heavy_flops, solo_bytes, solo_flops,
      hsolo_bytes, hsolo_flops;
};

// Rows whose only Gram task is heavy are fused with their solve up to this
// padded rank.
#ifndef TT_FUSE_HEAVY_MAX_RP
#define TT_FUSE_HEAVY_MAX_RP 32
#endif
constexpr int kFuseHeavyMaxRP = TT_FUSE_HEAVY_MAX_RP;

template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS>
static void launch_solo_rp(const GramDev &d, const SolveDev &sd, const GramLists &gl,
                           hipStream_t s) {
  if (gl.nsolo <= 0) return;
  ProfScope ps(sd.factor_only ? "gram_factor_light" : "gram_solve_light", s, gl.solo_bytes,
               gl.solo_flops);
  SolveDev sd2 = sd;
  sd2.rows = gl.solo;
  sd2.nrow = gl.nsolo;
  const dim3 grid(solve_grid(sd2)), block(64);
  const bool pers = grid.x < (unsigned)gl.nsolo;
#define TT_SOLO(FO, MOD)                                                               \
  do {                                                                                 \
    if (pers) k_solve_solo<TR, RP, VEC, WEIGHTED, RHS, FO, true, MOD><<<grid, block, 0, s>>>(d, sd2); \
    else k_solve_solo<TR, RP, VEC, WEIGHTED, RHS, FO, false, MOD><<<grid, block, 0, s>>>(d, sd2); \
  } while (0)
  if constexpr (RHS) {
    // the fused right-hand side always comes with a solve
    bool mod = false;
    if constexpr (!WEIGHTED) {
      mod = d.model != nullptr;
      if (mod) TT_SOLO(false, true);
    }
    if (!mod) TT_SOLO(false, false);
  } else {
    if (sd.factor_only) TT_SOLO(true, false);
    else TT_SOLO(false, false);
  }
#undef TT_SOLO
}


template <class TR, int RP, bool VEC, bool WEIGHTED, bool RHS>
static void launch_hsolo_rp(const GramDev &d, const SolveDev &sd, const GramLists &gl,
                            hipStream_t s) {
  if (gl.nhsolo <= 0) return;
  ProfScope ps(sd.factor_only ? "gram_factor_heavy" : "gram_solve_heavy", s, gl.hsolo_bytes,
               gl.hsolo_flops);
  SolveDev sd2 = sd;
  sd2.rows = gl.hsolo;
  sd2.nrow = gl.nhsolo;
  const dim3 grid((unsigned)gl.nhsolo), block(256);
  if constexpr (RHS) {
    // the fused right-hand side always comes with a solve
    bool mod = false;
    if constexpr (!WEIGHTED) {
      mod = d.model != nullptr;
      if (mod) k_gram_solve_heavy<TR, RP, VEC, WEIGHTED, RHS, false, true><<<grid, block, 0, s>>>(d, sd2);
    }
    if (!mod) k_gram_solve_heavy<TR, RP, VEC, WEIGHTED, RHS, false, false><<<grid, block, 0, s>>>(d, sd2);
  } else {
    if (sd.factor_only)
      k_gram_solve_heavy<TR, RP, VEC, WEIGHTED, RHS, true, false><<<grid, block, 0, s>>>(d, sd2);
    else
      k_gram_solve_heavy<TR, RP, VEC, WEIGHTED, RHS, false, false><<<grid, block, 0, s>>>(d, sd2);
  }
}

// Vector loads of VW = RP / 16 entries need R, ldA and the factor bases
// aligned to VW elements.
template <class TR, int RP>
static inline bool gram_vec_ok(const GramDev &d) {
  constexpr int VW = RP / 16;
  constexpr size_t al = VW * sizeof(typename TR::T);
  return d.R % VW == 0 && d.ldA % VW == 0 && reinterpret_cast<uintptr_t>(d.A0) % al == 0 &&
         reinterpret_cast<uintptr_t>(d.A1) % al == 0 &&
         reinterpret_cast<uintptr_t>(d.A_own) % al == 0;
}

// The Gram kernels' forms: weighted Grams (the Gauss-Newton
// preconditioner) never carry a fused right-hand side; the Newton form of
// alternating minimization (A_own set) has both, from the loss at the model
// value.  F is called with the (VEC, WEIGHTED, RHS) of the launch.
template <class TR, int RP, class F>
static inline void gram_form(const GramDev &d, F &&f) {
  const bool vec = gram_vec_ok<TR, RP>(d);
  if (d.A_own) {
    if (vec) f(std::true_type{}, std::true_type{}, std::true_type{});
    else f(std::false_type{}, std::true_type{}, std::true_type{});
  } else if (d.w) {
    if (vec) f(std::true_type{}, std::true_type{}, std::false_type{});
    else f(std::false_type{}, std::true_type{}, std::false_type{});
  } else if (d.M) {
    if (vec) f(std::true_type{}, std::false_type{}, std::true_type{});
    else f(std::false_type{}, std::false_type{}, std::true_type{});
  } else {
    if (vec) f(std::true_type{}, std::false_type{}, std::false_type{});
    else f(std::false_type{}, std::false_type{}, std::false_type{});
  }
}

// The fused Gram + solve rows of one batch: solo rows (one light task, a
// wave each) and heavy solo rows (one heavy task, a workgroup each).
template <class TR>
hipError_t launch_fused_rows(int RP, const GramDev &d, const SolveDev &sd, const GramLists &gl,
                             hipStream_t s) {
  auto run = [&](auto rp) {
    constexpr int P = decltype(rp)::value;
    gram_form<TR, P>(d, [&](auto v, auto w, auto h) {
      constexpr bool V = decltype(v)::value, W = decltype(w)::value, H = decltype(h)::value;
      launch_solo_rp<TR, P, V, W, H>(d, sd, gl, s);
      launch_hsolo_rp<TR, P, V, W, H>(d, sd, gl, s);
    });
  };
  switch (RP) {
    case 16: run(std::integral_constant<int, 16>{}); break;
    case 32: run(std::integral_constant<int, 32>{}); break;
    default: run(std::integral_constant<int, 64>{}); break;
  }
  return hipGetLastError();
}
hipError_t launch_fused_rows_f32(int RP, const GramDev &d, const SolveDev &sd,
                                 const GramLists &gl, hipStream_t s);
hipError_t launch_fused_rows_bf16(int RP, const GramDev &d, const SolveDev &sd,
                                  const GramLists &gl, hipStream_t s);

}  // namespace tt
