// Device-side helpers shared by the libtt kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace tt {

// ---------------------------------------------------------------------------
// Storage traits.  T = factor storage type, VT = per-nonzero value type,
// AT = accumulation type, V = elements per lane fragment (16 bytes for FP64
// and FP32, 8 bytes for BF16, so BF16 keeps the FP32 lane layout).
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
  static constexpr int V = 4;  // 8-byte fragments: the lane layout of the FP32 form
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
// [c0, c0 + V) of row `row`.  VEC: one vector load (requires 16-byte (BF16:
// 8-byte) aligned rows and a leading dimension of at least R rounded up to
// V; with R % V != 0 the caller masks per element, PARTIAL); otherwise
// element loads.  Elements at or beyond R
// read as 0.  The loads are unconditional (out-of-range lanes read column 0
// or R - 1 of the row and select 0 afterwards), so no branch separates a
// load from its use and the compiler can keep many gathers in flight.
// ---------------------------------------------------------------------------

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

template <class T>
__device__ __forceinline__ float widen_f(T x);
template <>
__device__ __forceinline__ float widen_f<float>(float x) { return x; }
template <>
__device__ __forceinline__ float widen_f<uint16_t>(uint16_t x) { return bf16_to_f32(x); }

// Traits of dense accumulation-type rows (X blocks of the matvec): the FP32
// or FP64 storage traits of the same lane layout.
template <class AT> struct DenseTrSel;
template <> struct DenseTrSel<float> { using type = TrF32; };
template <> struct DenseTrSel<double> { using type = TrF64; };
template <class AT> using DenseTr = typename DenseTrSel<AT>::type;

// A fragment as loaded (before widening and masking).  Gathers keep the raw
// form until the values are used, so that the compiler does not fold the
// masking into a branch around the load.
template <class TR, bool VEC>
struct FragRaw {
  typename TR::AT v[TR::V];
};
template <>
struct FragRaw<TrF32, true> { float4 v; };
template <>
struct FragRaw<TrF64, true> { double2 v; };
template <>
struct FragRaw<TrBF16, true> { uint2 v; };

template <class TR, bool VEC>
__device__ __forceinline__ void gather_frag(const typename TR::T *__restrict__ A,
                                            int64_t ldA, int64_t row, int c0, int R,
                                            FragRaw<TR, VEC> &f) {
  using T = typename TR::T;
  using AT = typename TR::AT;
  const uint32_t rb = (uint32_t)row * (uint32_t)ldA;
  if constexpr (VEC) {
    const uint32_t e = rb + (uint32_t)(c0 < R ? c0 : 0);
    f.v = *reinterpret_cast<const decltype(f.v) *>(at32(A, e));
  } else {
#pragma unroll
    for (int j = 0; j < TR::V; ++j) {
      const int c = c0 + j;
      const T x = *at32(A, rb + (uint32_t)(c < R ? c : R - 1));
      if constexpr (std::is_same<TR, TrF64>::value) f.v[j] = x;
      else f.v[j] = widen_f<T>(x);
    }
  }
}

// PARTIAL (vector fragments only): R need not be a multiple of V; the
// fragment holding column R - 1 reads past it (inside the row's leading
// dimension) and each element is masked on its own column.
template <class TR, bool VEC, bool PARTIAL = false>
__device__ __forceinline__ void widen_frag(const FragRaw<TR, VEC> &f, int c0, int R,
                                           typename TR::AT (&o)[TR::V]) {
  using AT = typename TR::AT;
  if constexpr (VEC && PARTIAL) {
    AT w[TR::V];
    widen_frag<TR, true, false>(f, c0, R, w);
#pragma unroll
    for (int j = 0; j < TR::V; ++j) o[j] = c0 + j < R ? w[j] : AT(0);
  } else if constexpr (VEC) {
    const bool ok = c0 < R;
    if constexpr (std::is_same<TR, TrF32>::value) {
      o[0] = ok ? f.v.x : 0.f; o[1] = ok ? f.v.y : 0.f;
      o[2] = ok ? f.v.z : 0.f; o[3] = ok ? f.v.w : 0.f;
    } else if constexpr (std::is_same<TR, TrF64>::value) {
      o[0] = ok ? f.v.x : 0.0; o[1] = ok ? f.v.y : 0.0;
    } else {
      o[0] = ok ? __uint_as_float(f.v.x << 16) : 0.f;
      o[1] = ok ? __uint_as_float(f.v.x & 0xffff0000u) : 0.f;
      o[2] = ok ? __uint_as_float(f.v.y << 16) : 0.f;
      o[3] = ok ? __uint_as_float(f.v.y & 0xffff0000u) : 0.f;
    }
  } else {
#pragma unroll
    for (int j = 0; j < TR::V; ++j) o[j] = c0 + j < R ? f.v[j] : AT(0);
  }
}

template <class TR, bool VEC, bool PARTIAL = false>
__device__ __forceinline__ void load_frag(const typename TR::T *__restrict__ A,
                                          int64_t ldA, int64_t row, int c0, int R,
                                          typename TR::AT (&o)[TR::V]) {
  FragRaw<TR, VEC> f;
  gather_frag<TR, VEC>(A, ldA, row, c0, R, f);
  widen_frag<TR, VEC, PARTIAL>(f, c0, R, o);
}

// Dense (accumulation-type) row fragment with row stride R: V elements
// [c0, c0 + V) of row `row`; elements at or beyond R read as 0 (loads are
// unconditional as above).
template <class AT, int V, bool VEC>
__device__ __forceinline__ void load_dense(const AT *__restrict__ X, int64_t row, int c0,
                                           int R, AT (&o)[V]) {
  const uint32_t rb = (uint32_t)row * (uint32_t)R;
  if constexpr (VEC) {
    const bool ok = c0 < R;
    const AT *p = at32(X, rb + (uint32_t)(ok ? c0 : 0));
    if constexpr (sizeof(AT) == 4) {
#pragma unroll
      for (int q = 0; q < V / 4; ++q) {
        const float4 v = reinterpret_cast<const float4 *>(p)[q];
        o[4 * q] = ok ? v.x : 0.f; o[4 * q + 1] = ok ? v.y : 0.f;
        o[4 * q + 2] = ok ? v.z : 0.f; o[4 * q + 3] = ok ? v.w : 0.f;
      }
    } else {
#pragma unroll
      for (int q = 0; q < V / 2; ++q) {
        const double2 v = reinterpret_cast<const double2 *>(p)[q];
        o[2 * q] = ok ? v.x : 0.0; o[2 * q + 1] = ok ? v.y : 0.0;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int c = c0 + j;
      const AT x = *at32(X, rb + (uint32_t)(c < R ? c : R - 1));
      o[j] = c < R ? x : AT(0);
    }
  }
}

// Lane permutations inside 16-lane rows (DPP controls): swap neighbours,
// swap pairs, mirror each half row, mirror the row.
enum : int { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140 };

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of G lanes (G a power of two <= 64); every lane of
// the group receives the total.  Inside a 16-lane row the partners come from
// DPP moves (two quad swaps, then the half-row and row mirrors, each of
// which pairs the lane with a lane of the other half); wider groups add
// butterfly steps across rows.  Every lane adds the same two operands at
// each step (in either order), so all lanes of a group get the same bits.
template <int G, class X>
__device__ __forceinline__ X group_sum(X v) {
  if constexpr (G >= 2) v += dpp_move<DPP_XOR1>(v);
  if constexpr (G >= 4) v += dpp_move<DPP_XOR2>(v);
  if constexpr (G >= 8) v += dpp_move<DPP_HALF_MIRROR>(v);
  if constexpr (G >= 16) v += dpp_move<DPP_MIRROR>(v);
#pragma unroll
  for (int o = 16; o < G; o <<= 1) v += __shfl_xor(v, o);
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
