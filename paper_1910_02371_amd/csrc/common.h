// Device-side helpers shared by the libtt kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tt {

// ---------------------------------------------------------------------------
// Storage traits.  T = factor storage type, VT = per-nonzero value type,
// AT = accumulation type, V = elements per 16-byte lane fragment.
// ---------------------------------------------------------------------------
struct TrF64 {
  using T = double;
  using VT = double;
  using AT = double;
  static constexpr int V = 2;
};
struct TrF32 {
  using T = float;
  using VT = float;
  using AT = float;
  static constexpr int V = 4;
};
struct TrBF16 {
  using T = uint16_t;
  using VT = float;
  using AT = float;
  static constexpr int V = 8;
};

__device__ __forceinline__ float bf16_to_f32(uint32_t b) {
  return __uint_as_float(b << 16);
}

// IEEE round-to-nearest-even of a binary32 value to bfloat16; NaN is kept
// NaN (quiet bit forced).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <class X>
__device__ __forceinline__ X to_acc(X v) { return v; }

// Convert a double result to storage type.
template <class T>
__device__ __forceinline__ T from_double(double v);
template <>
__device__ __forceinline__ double from_double<double>(double v) { return v; }
template <>
__device__ __forceinline__ float from_double<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ uint16_t from_double<uint16_t>(double v) {
  return f32_to_bf16_rne((float)v);
}

template <class T>
__device__ __forceinline__ double to_double(T v);
template <>
__device__ __forceinline__ double to_double<double>(double v) { return v; }
template <>
__device__ __forceinline__ double to_double<float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double to_double<uint16_t>(uint16_t v) {
  return (double)bf16_to_f32(v);
}

// ---------------------------------------------------------------------------
// Factor-row fragment loads: lane `c0 / V` of a group reads elements
// [c0, c0 + V) of row `row`.  VEC: one 16-byte load (requires R % V == 0,
// 16-byte aligned rows); otherwise element loads with the bound r < R.
// Elements at or beyond R read as 0.
// ---------------------------------------------------------------------------
template <class TR, bool VEC>
__device__ __forceinline__ void load_frag(const typename TR::T *__restrict__ A,
                                          int64_t ldA, int64_t row, int c0,
                                          int R, typename TR::AT (&o)[TR::V]);

// Element pointer from a uniform base and a 32-bit element offset (every
// factor and dense block is below 2^32 bytes, checked on the host), so the
// address is a scalar base plus one 32-bit vector offset.
template <class X>
__device__ __forceinline__ const X *at32(const X *base, uint32_t elem) {
  return reinterpret_cast<const X *>(reinterpret_cast<const char *>(base) +
                                     (uint32_t)(elem * (uint32_t)sizeof(X)));
}
template <class X>
__device__ __forceinline__ X *at32(X *base, uint32_t elem) {
  return reinterpret_cast<X *>(reinterpret_cast<char *>(base) +
                               (uint32_t)(elem * (uint32_t)sizeof(X)));
}

template <>
__device__ __forceinline__ void load_frag<TrF32, true>(const float *__restrict__ A,
                                                      int64_t ldA, int64_t row,
                                                      int c0, int R,
                                                      float (&o)[4]) {
  if (c0 < R) {
    float4 v = *reinterpret_cast<const float4 *>(at32(A, (uint32_t)row * (uint32_t)ldA + c0));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else {
    o[0] = o[1] = o[2] = o[3] = 0.f;
  }
}
template <>
__device__ __forceinline__ void load_frag<TrF32, false>(const float *__restrict__ A,
                                                       int64_t ldA, int64_t row,
                                                       int c0, int R,
                                                       float (&o)[4]) {
  const float *p = at32(A, (uint32_t)row * (uint32_t)ldA + c0);
#pragma unroll
  for (int j = 0; j < 4; ++j) o[j] = (c0 + j < R) ? p[j] : 0.f;
}
template <>
__device__ __forceinline__ void load_frag<TrF64, true>(const double *__restrict__ A,
                                                      int64_t ldA, int64_t row,
                                                      int c0, int R,
                                                      double (&o)[2]) {
  if (c0 < R) {
    double2 v = *reinterpret_cast<const double2 *>(at32(A, (uint32_t)row * (uint32_t)ldA + c0));
    o[0] = v.x; o[1] = v.y;
  } else {
    o[0] = o[1] = 0.0;
  }
}
template <>
__device__ __forceinline__ void load_frag<TrF64, false>(const double *__restrict__ A,
                                                       int64_t ldA, int64_t row,
                                                       int c0, int R,
                                                       double (&o)[2]) {
  const double *p = at32(A, (uint32_t)row * (uint32_t)ldA + c0);
#pragma unroll
  for (int j = 0; j < 2; ++j) o[j] = (c0 + j < R) ? p[j] : 0.0;
}
template <>
__device__ __forceinline__ void load_frag<TrBF16, true>(const uint16_t *__restrict__ A,
                                                       int64_t ldA, int64_t row,
                                                       int c0, int R,
                                                       float (&o)[8]) {
  if (c0 < R) {
    uint4 v = *reinterpret_cast<const uint4 *>(at32(A, (uint32_t)row * (uint32_t)ldA + c0));
    o[0] = __uint_as_float(v.x << 16); o[1] = __uint_as_float(v.x & 0xffff0000u);
    o[2] = __uint_as_float(v.y << 16); o[3] = __uint_as_float(v.y & 0xffff0000u);
    o[4] = __uint_as_float(v.z << 16); o[5] = __uint_as_float(v.z & 0xffff0000u);
    o[6] = __uint_as_float(v.w << 16); o[7] = __uint_as_float(v.w & 0xffff0000u);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = 0.f;
  }
}
template <>
__device__ __forceinline__ void load_frag<TrBF16, false>(const uint16_t *__restrict__ A,
                                                        int64_t ldA, int64_t row,
                                                        int c0, int R,
                                                        float (&o)[8]) {
  const uint16_t *p = at32(A, (uint32_t)row * (uint32_t)ldA + c0);
#pragma unroll
  for (int j = 0; j < 8; ++j) o[j] = (c0 + j < R) ? bf16_to_f32(p[j]) : 0.f;
}

// Dense (accumulation-type) row fragment with row stride R: V elements
// [c0, c0 + V) of row `row`; elements at or beyond R read as 0.
template <class AT, int V, bool VEC>
__device__ __forceinline__ void load_dense(const AT *__restrict__ X, int64_t row, int c0,
                                           int R, AT (&o)[V]) {
  const AT *p = at32(X, (uint32_t)row * (uint32_t)R + c0);
  if constexpr (VEC) {
    if (c0 < R) {
      if constexpr (sizeof(AT) == 4) {
#pragma unroll
        for (int q = 0; q < V / 4; ++q) {
          float4 v = reinterpret_cast<const float4 *>(p)[q];
          o[4 * q] = v.x; o[4 * q + 1] = v.y; o[4 * q + 2] = v.z; o[4 * q + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < V / 2; ++q) {
          double2 v = reinterpret_cast<const double2 *>(p)[q];
          o[2 * q] = v.x; o[2 * q + 1] = v.y;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j) o[j] = AT(0);
    }
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) o[j] = (c0 + j < R) ? p[j] : AT(0);
  }
}

// Butterfly sum over aligned groups of G lanes (G a power of two <= 64);
// every lane of the group receives the total.
template <int G, class X>
__device__ __forceinline__ X group_sum(X v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Elementwise loss maps (least squares and Poisson log link).
enum { LOSS_LS = 0, LOSS_POISSON_LOG = 1 };
enum { EPI_NONE = 0, EPI_RESID = 1, EPI_PHI = 2, EPI_DPHI = 3, EPI_D2PHI = 4 };

template <class AT>
__device__ __forceinline__ AT loss_eval(int epi, int loss, AT t, AT m) {
  if (epi == EPI_RESID) return t - m;
  if (loss == LOSS_LS) {
    AT d = m - t;
    if (epi == EPI_PHI) return d * d;
    if (epi == EPI_DPHI) return AT(2) * d;
    return AT(2);
  }
  AT e = exp(m);
  if (epi == EPI_PHI) return e - t * m;
  if (epi == EPI_DPHI) return e - t;
  return e;
}

}  // namespace tt
