// CCD++ coordinate minimization (Section 2.3, least squares): the passes of
// one column update.  For column r, mode n:
//     u_i <- sum_e rhohat_e h_e / (lambda + sum_e h_e^2),   e in row i,
// with h_e the product of the other modes' column-r entries (current
// values: modes updated earlier in the column are new) and rhohat the
// residual without column r's rank-1 term (old values of all modes).  The
// residual rho = t - model is kept in every mode's sorted order, so each
// pass streams its own copy; factor columns are read from contiguous
// vectors of (old, current) pairs, which stay in the caches.  Column r - 1
// leaves every copy to be moved from its old to its new rank-1 term; mode
// n's pass of column r applies that move to its own copy as it streams it
// (two sets of pair vectors, columns r - 1 and r), so each column costs one
// read-modify-write pass per mode.  After the sweep's last column the
// copies are stale: the next sweep recomputes them.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace tt {

// Old and current value of one factor column entry, kept side by side so
// that a gather fetches both from one cache line.
template <class AT> struct Pair2;
template <> struct Pair2<float> { using type = float2; };
template <> struct Pair2<double> { using type = double2; };

// Column r of an I x ldA factor into its (old, current) pair vector.
template <class T, class AT>
__global__ void k_ccd_column(const T *__restrict__ A, int64_t ldA, int64_t I, int r,
                             typename Pair2<AT>::type *__restrict__ pr) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I;
       i += (int64_t)gridDim.x * blockDim.x) {
    const AT v = (AT)to_double<T>(A[i * ldA + r]);
    pr[i] = {v, v};
  }
}

// One wave per Gram task (a piece of <= gram_piece nonzeros of one row):
// FP64 partial sums of rhohat_e h_e and h_e^2 over the task, lanes striding
// over its nonzeros, then a fixed butterfly.  With the previous column's
// pairs (qn, q0, q1 non-NULL) each residual is first moved from that
// column's old to its new rank-1 term and stored back.
template <class AT, class VT>
__global__ __launch_bounds__(256) void k_ccd_tasks(
    const int64_t *__restrict__ task, int64_t ntask, const int32_t *__restrict__ key,
    const int32_t *__restrict__ o0, const int32_t *__restrict__ o1, VT *__restrict__ rho,
    const typename Pair2<AT>::type *__restrict__ pn,
    const typename Pair2<AT>::type *__restrict__ p0,
    const typename Pair2<AT>::type *__restrict__ p1,
    const typename Pair2<AT>::type *__restrict__ qn,
    const typename Pair2<AT>::type *__restrict__ q0,
    const typename Pair2<AT>::type *__restrict__ q1, double *__restrict__ part) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (t >= ntask) return;
  const int64_t nb = task[t], ne = task[t + 1];
  const int32_t row = key[nb];  // one row per task
  const double own_old = (double)pn[row].x;
  const bool move = qn != nullptr;
  const auto un = move ? qn[row] : typename Pair2<AT>::type{};
  double num = 0.0, den = 0.0;
  for (int64_t e = nb + lane; e < ne; e += 64) {
    const int32_t i0 = o0[e], i1 = o1[e];
    VT r = rho[e];
    if (move) {
      const auto a = q0[i0];
      const auto b = q1[i1];
      const double told = (double)un.x * (double)a.x * (double)b.x;
      const double tnew = (double)un.y * (double)a.y * (double)b.y;
      r = (VT)(((double)r + told) - tnew);
      rho[e] = r;
    }
    const auto a = p0[i0];
    const auto b = p1[i1];
    const double h = (double)a.y * (double)b.y;
    const double rhat = (double)r + own_old * ((double)a.x * (double)b.x);
    num = fma(rhat, h, num);
    den = fma(h, h, den);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    num += __shfl_xor(num, o);
    den += __shfl_xor(den, o);
  }
  if (lane == 0) {
    part[2 * t] = num;
    part[2 * t + 1] = den;
  }
}

// One wave per row: the row's task partials summed in FP64 (lanes stride
// over the tasks, then a fixed butterfly), the rank-1 solve
// (lambda + den) x = num (LAPACK convention: a non-positive pivot gives
// info 1 and x = 0), x stored into column r of the factor (storage dtype)
// and, as stored, as the current value of the pair vector.
template <class T, class AT>
__global__ __launch_bounds__(256) void k_ccd_rows(const int32_t *__restrict__ row_task,
                                                  int64_t I, const double *__restrict__ part,
                                                  double lambda, T *A, int64_t ldA, int r,
                                                  typename Pair2<AT>::type *__restrict__ pr,
                                                  int32_t *info) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < I;
       i += (int64_t)gridDim.x * 4) {
    double num = 0.0, den = 0.0;
    for (int32_t t = row_task[i] + lane; t < row_task[i + 1]; t += 64) {
      num += part[2 * t];
      den += part[2 * t + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      num += __shfl_xor(num, o);
      den += __shfl_xor(den, o);
    }
    if (lane == 0) {
      const double piv = lambda + den;
      const bool ok = piv > 0.0;
      const T x = from_double<T>(ok ? num / piv : 0.0);
      A[i * ldA + r] = x;
      pr[i].y = (AT)to_double<T>(x);
      if (info) info[i] = ok ? 0 : 1;
    }
  }
}

static unsigned grid_for_n(int64_t n, int64_t cap = 65536) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

template <class T, class AT, class VT>
static hipError_t ccd_column_t(const tt_index *ix, int r, void *const *d_A, int64_t ldA,
                               double lambda, void *const *rho, void *const *pairs,
                               void *const *prev, double *part, int32_t *d_info,
                               hipStream_t s) {
  using P2 = typename Pair2<AT>::type;
  const int N = ix->N;
  for (int n = 0; n < N; ++n) {
    const ModeIndex &md = ix->mode[n];
    ProfScope ps("ccd_column", s, (double)md.I * (sizeof(T) + sizeof(P2)), 0.0);
    if (md.I > 0)
      k_ccd_column<T, AT><<<grid_for_n(md.I), 256, 0, s>>>((const T *)d_A[n], ldA, md.I, r,
                                                           (P2 *)pairs[n]);
  }
  int64_t off = 0;
  for (int n = 0; n < N; ++n) {
    const ModeIndex &md = ix->mode[n];
    int q0 = -1, q1 = -1;
    for (int p = 0; p < N; ++p)
      if (p != n) (q0 < 0 ? q0 : q1) = p;
    if (md.ntask > 0) {
      ProfScope ps("ccd_mode_pass", s,
                   (double)ix->m * (4.0 * 2 + sizeof(VT) * (prev ? 2 : 1)),
                   (double)ix->m * (prev ? 14.0 : 8.0));
      k_ccd_tasks<AT, VT><<<(unsigned)((md.ntask + 3) / 4), 256, 0, s>>>(
          md.d_task, md.ntask, md.d_key, md.d_oidx[q0], md.d_oidx[q1], (VT *)rho[n],
          (const P2 *)pairs[n], (const P2 *)pairs[q0], (const P2 *)pairs[q1],
          prev ? (const P2 *)prev[n] : nullptr, prev ? (const P2 *)prev[q0] : nullptr,
          prev ? (const P2 *)prev[q1] : nullptr, part);
    }
    ProfScope ps("ccd_rows", s, (double)md.ntask * 16 + (double)md.I * (sizeof(T) + sizeof(AT)),
                 (double)md.ntask * 2);
    if (md.I > 0)
      k_ccd_rows<T, AT><<<grid_for_n(64 * md.I, 262144), 256, 0, s>>>(
          md.d_row_task, md.I, part, lambda, (T *)d_A[n], ldA, r, (P2 *)pairs[n],
          d_info ? d_info + off : nullptr);
    off += md.I;
  }
  return hipGetLastError();
}

hipError_t launch_ccd_column(const tt_index *ix, int r, void *const *d_A, int64_t ldA,
                             tt_dtype fdt, double lambda, void *const *rho, void *const *pairs,
                             void *const *prev, double *part, int32_t *d_info, hipStream_t s) {
  if (fdt == TT_F64)
    return ccd_column_t<double, double, double>(ix, r, d_A, ldA, lambda, rho, pairs, prev,
                                                part, d_info, s);
  if (fdt == TT_F32)
    return ccd_column_t<float, float, float>(ix, r, d_A, ldA, lambda, rho, pairs, prev, part,
                                             d_info, s);
  return ccd_column_t<uint16_t, float, float>(ix, r, d_A, ldA, lambda, rho, pairs, prev, part,
                                              d_info, s);
}

}  // namespace tt
