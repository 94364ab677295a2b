// Device pieces shared by the dense helper kernels (vec.hip) and the
// persistent conjugate-gradient loop: fixed-order FP64 block reductions,
// the elementwise PCG updates and the scalar steps of PCG (Section 2.5).
// Each piece is written once so that both forms compute bit-identical
// results.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tt {

constexpr int VT_THREADS = 256;
constexpr int RED_BLOCKS = 1024;  // max partials of a two-level reduction

// Block-level FP64 sum of a 256-thread workgroup in a fixed order (wave
// butterfly, then the four waves in order).  Every thread calls it and
// receives the sum.
__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double part[VT_THREADS / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < VT_THREADS / 64; ++w) s += part[w];
  __syncthreads();
  return s;
}

// Second level of a two-level reduction: n partials summed by one
// workgroup (thread t takes partials t, t + 256, ...).
__device__ __forceinline__ double sum_parts_block(const double *parts, int64_t n) {
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += VT_THREADS) v += parts[i];
  return block_sum_d(v);
}

// First level of the dot product x.y over n values: partial vb of np, the
// grid-stride share of a (virtual) workgroup vb in a grid of np.
template <class X>
__device__ __forceinline__ double dot_part_block(const X *x, const X *y, int64_t n, int64_t vb,
                                                 int64_t np) {
  double v = 0.0;
  for (int64_t i = vb * VT_THREADS + threadIdx.x; i < n; i += np * VT_THREADS)
    v += (double)x[i] * (double)y[i];
  return block_sum_d(v);
}

template <class Y>
__device__ __forceinline__ Y scaled(double a, double x) {
  return (Y)(a * x);
}

// x_i += alpha p_i; r_i -= alpha q_i
template <class X>
__device__ __forceinline__ void axpy2_at(X *x, const X *p, X *r, const X *q, int64_t i,
                                         double a) {
  x[i] = (X)((double)x[i] + a * (double)p[i]);
  r[i] = (X)((double)r[i] - a * (double)q[i]);
}

// z_i + beta p_i
template <class X>
__device__ __forceinline__ X xpby_at(const X *p, const X *z, int64_t i, double b) {
  return (X)((double)z[i] + b * (double)p[i]);
}

// PCG scalar slots (device doubles).
enum {
  SC_RZ = 0, SC_PHP = 1, SC_RR = 2, SC_R0 = 3, SC_RZNEW = 4, SC_DONE = 5,
  SC_ITERS = 6, SC_ALPHA = 7, SC_BETA = 8, SC_REL = 9
};

// Scalar steps of PCG on the slots above.
//  stage 0 (after z0 = P^{-1} r0, rz = r.z, rr = r.r): r0 = sqrt(rr); done if r0 == 0
//  stage 1 (after pHp = p.Hp): alpha = rz / pHp
//  stage 2 (after rr = r.r): rel = sqrt(rr) / r0; iters += 1; done if rel <= tol
//  stage 3 (after rznew = r.z): beta = rznew / rz; rz = rznew
__device__ __forceinline__ void pcg_stage(double *sc, int stage, double tol) {
  if (stage == 0) {
    sc[SC_R0] = sqrt(sc[SC_RR]);
    sc[SC_ITERS] = 0.0;
    sc[SC_REL] = 1.0;
    sc[SC_DONE] = (sc[SC_R0] == 0.0) ? 1.0 : 0.0;
    if (sc[SC_R0] == 0.0) sc[SC_REL] = 0.0;
    return;
  }
  if (sc[SC_DONE] != 0.0) return;
  if (stage == 1) {
    sc[SC_ALPHA] = sc[SC_RZ] / sc[SC_PHP];
  } else if (stage == 2) {
    const double rel = sqrt(sc[SC_RR]) / sc[SC_R0];
    sc[SC_REL] = rel;
    sc[SC_ITERS] += 1.0;
    if (rel <= tol) sc[SC_DONE] = 1.0;
  } else if (stage == 3) {
    sc[SC_BETA] = sc[SC_RZNEW] / sc[SC_RZ];
    sc[SC_RZ] = sc[SC_RZNEW];
  }
}

}  // namespace tt
