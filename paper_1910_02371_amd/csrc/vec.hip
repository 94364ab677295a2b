// Dense helper kernels: fills, row scaling (regularization terms), FP64
// reductions with a fixed order, and the vector/scalar steps of the
// preconditioned conjugate gradient used by the Gauss-Newton iteration
// (Section 2.5).  Reductions are two-level (per-block FP64 partials, then one
// block summing the partials in index order), so results are deterministic.
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"
#include "vec_impl.h"

namespace tt {

static int grid_cap(int64_t n, int cap) {
  int64_t g = (n + VT_THREADS - 1) / VT_THREADS;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

template <class X>
__global__ void k_fill(X *p, int64_t n, X v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill(void *p, int64_t n, tt_dtype dense, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dense == TT_F64)
    k_fill<double><<<grid_cap(n, 8192), VT_THREADS, 0, s>>>((double *)p, n, v);
  else
    k_fill<float><<<grid_cap(n, 8192), VT_THREADS, 0, s>>>((float *)p, n, (float)v);
  return hipGetLastError();
}

template <class XT, class YT>
__global__ void k_scale_rows(YT *y, const XT *x, int64_t ldx, int64_t I, int R, double a) {
  const int64_t n = I * R;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / R;
    const int r = (int)(i - row * R);
    y[i] = scaled<YT>(a, to_double<XT>(x[row * ldx + r]));
  }
}

hipError_t launch_scale_rows(void *y, const void *x, tt_dtype xdt, int64_t ldx,
                             int64_t I, int R, double a, tt_dtype ydt, hipStream_t s) {
  const int64_t n = I * R;
  if (n <= 0) return hipSuccess;
  const int g = grid_cap(n, 8192);
  if (ydt == TT_F64) {
    k_scale_rows<double, double><<<g, VT_THREADS, 0, s>>>((double *)y, (const double *)x,
                                                          ldx, I, R, a);
  } else if (xdt == TT_F32) {
    k_scale_rows<float, float><<<g, VT_THREADS, 0, s>>>((float *)y, (const float *)x, ldx,
                                                        I, R, a);
  } else if (xdt == TT_BF16) {
    k_scale_rows<uint16_t, float><<<g, VT_THREADS, 0, s>>>((float *)y, (const uint16_t *)x,
                                                           ldx, I, R, a);
  } else {
    k_scale_rows<double, float><<<g, VT_THREADS, 0, s>>>((float *)y, (const double *)x,
                                                         ldx, I, R, a);
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(VT_THREADS) void k_sum_doubles(const double *parts, int64_t n,
                                                             double *out, int accumulate,
                                                             const double *skip) {
  if (skip && *skip != 0.0) return;
  const double s = sum_parts_block(parts, n);
  if (threadIdx.x == 0) *out = accumulate ? *out + s : s;
}

hipError_t launch_sum_doubles(const double *parts, int64_t n, double *out, int accumulate,
                              hipStream_t s, const double *skip) {
  k_sum_doubles<<<1, VT_THREADS, 0, s>>>(parts, n, out, accumulate, skip);
  return hipGetLastError();
}

template <class XT>
__global__ void k_sumsq_rows(const XT *A, int64_t ldA, int64_t I, int R, double scale,
                             double *parts, const double *skip) {
  if (skip && *skip != 0.0) return;
  const int64_t n = I * R;
  double v = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / R;
    const double a = to_double<XT>(A[row * ldA + (i - row * R)]);
    v += a * a;
  }
  const double s = block_sum_d(v);
  if (threadIdx.x == 0) parts[blockIdx.x] = scale * s;
}

int64_t sumsq_parts_needed(int64_t I, int R) { return grid_cap(I * (int64_t)R, RED_BLOCKS); }

hipError_t launch_sumsq_rows(const void *A, tt_dtype fdt, int64_t ldA, int64_t I, int R,
                             double scale, double *parts, int64_t *nparts, hipStream_t s,
                             const double *skip) {
  const int g = grid_cap(I * (int64_t)R, RED_BLOCKS);
  *nparts = g;
  if (fdt == TT_F64)
    k_sumsq_rows<double><<<g, VT_THREADS, 0, s>>>((const double *)A, ldA, I, R, scale, parts,
                                                  skip);
  else if (fdt == TT_F32)
    k_sumsq_rows<float><<<g, VT_THREADS, 0, s>>>((const float *)A, ldA, I, R, scale, parts,
                                                 skip);
  else
    k_sumsq_rows<uint16_t><<<g, VT_THREADS, 0, s>>>((const uint16_t *)A, ldA, I, R, scale,
                                                    parts, skip);
  return hipGetLastError();
}

template <class X>
__global__ __launch_bounds__(VT_THREADS) void k_dot_parts(const X *x, const X *y, int64_t n,
                                                          double *parts) {
  const double s = dot_part_block(x, y, n, blockIdx.x, gridDim.x);
  if (threadIdx.x == 0) parts[blockIdx.x] = s;
}

int64_t dot_parts_needed(int64_t n) { return grid_cap(n, RED_BLOCKS); }

hipError_t launch_dot_parts(const void *x, const void *y, int64_t n, tt_dtype dense,
                            double *parts, int64_t *nparts, hipStream_t s) {
  const int g = grid_cap(n, RED_BLOCKS);
  *nparts = g;
  if (dense == TT_F64)
    k_dot_parts<double><<<g, VT_THREADS, 0, s>>>((const double *)x, (const double *)y, n, parts);
  else
    k_dot_parts<float><<<g, VT_THREADS, 0, s>>>((const float *)x, (const float *)y, n, parts);
  return hipGetLastError();
}

// x += alpha p; r -= alpha q   (skipped once converged)
template <class X>
__global__ void k_axpy2(X *x, const X *p, X *r, const X *q, int64_t n, const double *sc) {
  if (sc[SC_DONE] != 0.0) return;
  const double a = sc[SC_ALPHA];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    axpy2_at(x, p, r, q, i, a);
}

hipError_t launch_axpy2(void *x, const void *p, void *r, const void *q, int64_t n,
                        tt_dtype dense, const double *sc, int ia, hipStream_t s) {
  (void)ia;
  const int g = grid_cap(n, 8192);
  if (dense == TT_F64)
    k_axpy2<double><<<g, VT_THREADS, 0, s>>>((double *)x, (const double *)p, (double *)r,
                                             (const double *)q, n, sc);
  else
    k_axpy2<float><<<g, VT_THREADS, 0, s>>>((float *)x, (const float *)p, (float *)r,
                                            (const float *)q, n, sc);
  return hipGetLastError();
}

// p = z + beta p   (skipped once converged)
template <class X>
__global__ void k_xpby(X *p, const X *z, int64_t n, const double *sc) {
  if (sc[SC_DONE] != 0.0) return;
  const double b = sc[SC_BETA];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = xpby_at(p, z, i, b);
}

hipError_t launch_xpby(void *p, const void *z, int64_t n, tt_dtype dense, const double *sc,
                       int ib, hipStream_t s) {
  (void)ib;
  const int g = grid_cap(n, 8192);
  if (dense == TT_F64)
    k_xpby<double><<<g, VT_THREADS, 0, s>>>((double *)p, (const double *)z, n, sc);
  else
    k_xpby<float><<<g, VT_THREADS, 0, s>>>((float *)p, (const float *)z, n, sc);
  return hipGetLastError();
}

__global__ void k_pcg_scalar(double *sc, int stage, double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  pcg_stage(sc, stage, tol);
}

hipError_t launch_pcg_scalar(double *sc, int stage, double tol, hipStream_t s) {
  k_pcg_scalar<<<1, 64, 0, s>>>(sc, stage, tol);
  return hipGetLastError();
}

__global__ void k_pcg_stats(const double *sc, const double *f0, double *stats) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  stats[0] = sc[SC_ITERS];
  stats[1] = sc[SC_REL];
  stats[2] = sc[SC_R0];
  stats[3] = f0 ? *f0 : 0.0;
}

hipError_t launch_pcg_stats(const double *sc, const double *f0, double *stats, hipStream_t s) {
  k_pcg_stats<<<1, 64, 0, s>>>(sc, f0, stats);
  return hipGetLastError();
}

// A[i, r] += dx[i * R + r]  (storage dtype; bfloat16 rounded to nearest even)
template <class T, class D>
__global__ void k_add_to_factor(T *A, int64_t ldA, int64_t I, int R, const D *dx,
                                const double *skip) {
  if (skip && *skip != 0.0) return;
  const int64_t n = I * R;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / R;
    T *p = A + row * ldA + (i - row * R);
    *p = from_double<T>(to_double<T>(*p) + (double)dx[i]);
  }
}

hipError_t launch_add_to_factor(void *A, tt_dtype fdt, int64_t ldA, int64_t I, int R,
                                const void *dx, hipStream_t s, const double *skip) {
  const int64_t n = I * R;
  if (n <= 0) return hipSuccess;
  const int g = grid_cap(n, 8192);
  if (fdt == TT_F64)
    k_add_to_factor<double, double><<<g, VT_THREADS, 0, s>>>((double *)A, ldA, I, R,
                                                             (const double *)dx, skip);
  else if (fdt == TT_F32)
    k_add_to_factor<float, float><<<g, VT_THREADS, 0, s>>>((float *)A, ldA, I, R,
                                                           (const float *)dx, skip);
  else
    k_add_to_factor<uint16_t, float><<<g, VT_THREADS, 0, s>>>((uint16_t *)A, ldA, I, R,
                                                              (const float *)dx, skip);
  return hipGetLastError();
}

// A[i, r] += D[i, r] over I rows, both in the factor dtype with their own
// leading dimensions; the sum is formed in FP64 and rounded once.
template <class T>
__global__ void k_add_rows(T *A, int64_t ldA, const T *D, int64_t ldD, int64_t I, int R,
                           const double *skip) {
  if (skip && *skip != 0.0) return;
  const int64_t n = I * R;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / R;
    const int r = (int)(i - row * R);
    T *p = A + row * ldA + r;
    *p = from_double<T>(to_double<T>(*p) + to_double<T>(D[row * ldD + r]));
  }
}

hipError_t launch_add_rows(void *A, int64_t ldA, const void *D, int64_t ldD, tt_dtype fdt,
                           int64_t I, int R, hipStream_t s, const double *skip) {
  const int64_t n = I * R;
  if (n <= 0) return hipSuccess;
  const int g = grid_cap(n, 8192);
  if (fdt == TT_F64)
    k_add_rows<double><<<g, VT_THREADS, 0, s>>>((double *)A, ldA, (const double *)D, ldD, I, R,
                                                skip);
  else if (fdt == TT_F32)
    k_add_rows<float><<<g, VT_THREADS, 0, s>>>((float *)A, ldA, (const float *)D, ldD, I, R,
                                               skip);
  else
    k_add_rows<uint16_t><<<g, VT_THREADS, 0, s>>>((uint16_t *)A, ldA, (const uint16_t *)D, ldD,
                                                  I, R, skip);
  return hipGetLastError();
}

// Newton-iteration bookkeeping of alternating minimization, one mode at a
// time: sc[0] = ||D||_F^2, sc[1] = ||A_n||_F^2, sc[2] = converged flag,
// sc[count] = iterations run.  Unless the mode has converged, count the
// iteration just run and, with `check`, set the flag when
// ||D||_F <= tol ||A_n||_F.
__global__ void k_gam_flag(double *sc, double tol, int count, int check) {
  if (threadIdx.x != 0 || sc[2] != 0.0) return;
  sc[count] += 1.0;
  if (check && sqrt(sc[0]) <= tol * sqrt(sc[1])) sc[2] = 1.0;
}

hipError_t launch_gam_flag(double *sc, double tol, int count, int check, hipStream_t s) {
  k_gam_flag<<<1, 64, 0, s>>>(sc, tol, count, check);
  return hipGetLastError();
}

}  // namespace tt
