// CCD++ coordinate minimization (Section 2.3, least squares): the passes of
// one column update.  For column r, mode n:
//     u_i <- sum_e rhohat_e h_e / (lambda + sum_e h_e^2),   e in row i,
// with h_e the product of the other modes' column-r entries (current
// values: modes updated earlier in the column are new) and rhohat the
// residual without column r's rank-1 term (old values of all modes).  The
// residual rho = t - model is kept in every mode's sorted order, so each
// pass streams its own copy.  Column r - 1 leaves every copy to be moved
// from its old to its new rank-1 term; mode n's pass of column r applies
// that move to its own copy as it streams it, so each column costs one
// read-modify-write pass per mode.  After the sweep's last column the
// copies are stale: the next sweep recomputes them.
//
// Factor entries are gathered from one record per row holding column
// r - 1's old and new value and column r's old and current value: the
// gathers of a pass hit random rows of the other factors, so each costs a
// whole cache line, and one record per row fetches the four values with
// one line (the largest mode's records, 7.7 MB at 480K rows, do not stay
// in L2).  With the CCD++ layout of a mode (tuning ccd_xcd) its pass runs
// over the stream regrouped by bucket of the largest other mode's index,
// and each XCD only gathers the records of its bucket's rows, which fit its
// L2; the residual copy of that mode follows the layout's order.  When the
// smaller other mode's records fit in 48 KiB (tuning ccd_lds) every
// workgroup of the pass reads them from an LDS copy.  A row's rank-1 solve
// is done by its task's wave when the row has a single task, else by
// k_ccd_rows from the tasks' partial sums.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace tt {

// (column r - 1 old, column r - 1 new, column r old, column r current)
template <class AT> struct Rec4;
template <> struct Rec4<float> { using type = float4; };
template <> struct Rec4<double> { using type = double4; };

// Start of column r: every record moves its column-r values into the
// column r - 1 slots and takes column r of the I x ldA factor.
template <class T, class AT>
__global__ void k_ccd_column(const T *__restrict__ A, int64_t ldA, int64_t I, int r,
                             typename Rec4<AT>::type *__restrict__ rec) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < I;
       i += (int64_t)gridDim.x * blockDim.x) {
    const AT v = (AT)to_double<T>(A[i * ldA + r]);
    const auto q = rec[i];
    rec[i] = {q.z, q.w, v, v};
  }
}

// One group of GL lanes (GL = 64: a wave) per Gram task (a piece of <=
// gram_piece nonzeros of one row): FP64 partial sums of rhohat_e h_e and
// h_e^2 over the task, lanes striding over its nonzeros, then a fixed
// butterfly.  With `move` each residual is first moved from column r - 1's
// old to its new rank-1 term and stored back.  (A task per quarter wave was
// measured slower on short rows: the passes are bound by the gathers'
// cache-line transfers, not by the number of waves.)
// Rows with a single task (row_task[i + 1] - row_task[i] == 1) are solved by
// that task's wave right away (RowSolve), exactly as k_ccd_rows would from
// the one partial; k_ccd_rows skips them.
template <class T, class AT>
struct RowSolve {
  const int32_t *row_task;
  double lambda;
  T *A;
  int64_t ldA;
  int r;
  typename Rec4<AT>::type *rec;  // the pass's own mode's records
  int32_t *info;
};

// The rank-1 solve of row i from its sums (LAPACK convention: a non-positive
// pivot gives info 1 and x = 0); x goes to column r of the factor (storage
// dtype) and, as stored, to the current value of the record.
template <class T, class AT>
__device__ __forceinline__ void ccd_solve_row(const RowSolve<T, AT> &rs, int64_t i, double num,
                                              double den) {
  const double piv = rs.lambda + den;
  const bool ok = piv > 0.0;
  const T x = from_double<T>(ok ? num / piv : 0.0);
  rs.A[i * rs.ldA + rs.r] = x;
  rs.rec[i].w = (AT)to_double<T>(x);
  if (rs.info) rs.info[i] = ok ? 0 : 1;
}

template <class T, class AT, class VT, int GL, int LS>
__device__ __forceinline__ void ccd_task(int64_t t, int64_t ntask, const int64_t *__restrict__ task,
                                         const int32_t *__restrict__ key,
                                         const int32_t *__restrict__ o0,
                                         const int32_t *__restrict__ o1, VT *__restrict__ rho,
                                         const typename Rec4<AT>::type *rn,
                                         const typename Rec4<AT>::type *__restrict__ r0,
                                         const typename Rec4<AT>::type *__restrict__ r1,
                                         const typename Rec4<AT>::type *st, int move,
                                         double *__restrict__ part, const RowSolve<T, AT> &rs) {
  const int lane = threadIdx.x % GL;
  // (no early return: every lane of the wave takes part in the butterfly)
  const bool live = t >= 0 && t < ntask;
  const int64_t nb = live ? task[t] : 0, ne = live ? task[t + 1] : 0;
  const int32_t own_row = live ? key[nb] : 0;  // one row per task
  const auto un = live ? rn[own_row] : typename Rec4<AT>::type{};
  const double own_old = (double)un.z;
  // each lane takes nonzeros lane, lane + GL, ... in order, U at a time:
  // all their loads and gathers are issued before the first is used
  constexpr int U = 4;
  using R4 = typename Rec4<AT>::type;
  double num = 0.0, den = 0.0;
  for (int64_t e0 = nb + lane; e0 < ne; e0 += GL * U) {
    int32_t i0[U], i1[U];
    VT r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + GL * u < ne ? e0 + GL * u : nb;  // in range
      i0[u] = o0[e];
      i1[u] = o1[e];
      r[u] = rho[e];
    }
    R4 a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // LS: that side's records come from the workgroup's LDS copy
      a[u] = LS == 0 ? st[i0[u]] : r0[i0[u]];
      b[u] = LS == 1 ? st[i1[u]] : r1[i1[u]];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = e0 + GL * u;
      if (e < ne) {
        if (move) {
          const double told = (double)un.x * (double)a[u].x * (double)b[u].x;
          const double tnew = (double)un.y * (double)a[u].y * (double)b[u].y;
          r[u] = (VT)(((double)r[u] + told) - tnew);
          rho[e] = r[u];
        }
        const double h = (double)a[u].w * (double)b[u].w;
        const double rhat = (double)r[u] + own_old * ((double)a[u].z * (double)b[u].z);
        num = fma(rhat, h, num);
        den = fma(h, h, den);
      }
    }
  }
#pragma unroll
  for (int o = GL / 2; o > 0; o >>= 1) {
    num += __shfl_xor(num, o);
    den += __shfl_xor(den, o);
  }
  if (live && lane == 0) {
    if (rs.row_task[own_row + 1] - rs.row_task[own_row] == 1) {
      ccd_solve_row<T, AT>(rs, own_row, num, den);
    } else {
      part[2 * t] = num;
      part[2 * t + 1] = den;
    }
  }
}

extern __shared__ double4 ccd_lds[];

// Wave q of workgroup j takes slot 4 j + q (task = the slot, or the one the
// schedule gives).  LS = 0 or 1: the workgroup first copies the nstage
// records of that side (r0 or r1) into LDS, then its waves loop over slots
// 4 (j + k gridDim.x) + q; with a schedule the grid is a multiple of 8, so
// the workgroup stays on the XCD the schedule meant for those slots.  (The
// records staged are the small side's, which mostly hit the L1 cache
// otherwise: the copy saves ~7 % of such a pass; the other side's gathers
// from L2 remain the bound.)
template <class T, class AT, class VT, int GL, int LS>
__global__ __launch_bounds__(256) void k_ccd_tasks(
    const int64_t *__restrict__ task, int64_t ntask, const int32_t *__restrict__ sched,
    int64_t nslot, const int32_t *__restrict__ key, const int32_t *__restrict__ o0,
    const int32_t *__restrict__ o1, VT *__restrict__ rho,
    const typename Rec4<AT>::type *rn,  // the own mode's records (rs.rec)
    const typename Rec4<AT>::type *__restrict__ r0,
    const typename Rec4<AT>::type *__restrict__ r1, int64_t nstage, int move,
    double *__restrict__ part, RowSolve<T, AT> rs) {
  static_assert(GL == 64, "one-wave slots, four per workgroup");
  using R4 = typename Rec4<AT>::type;
  R4 *st = reinterpret_cast<R4 *>(ccd_lds);
  if constexpr (LS >= 0) {
    const R4 *src = LS == 0 ? r0 : r1;
    for (int64_t i = threadIdx.x; i < nstage; i += blockDim.x) st[i] = src[i];
    __syncthreads();
  }
  const int64_t stride = LS >= 0 ? 4 * (int64_t)gridDim.x : nslot;
  for (int64_t slot = (int64_t)blockIdx.x * 4 + threadIdx.x / GL; slot < nslot; slot += stride) {
    const int64_t t = sched ? (int64_t)sched[slot] : slot;
    ccd_task<T, AT, VT, GL, LS>(t, ntask, task, key, o0, o1, rho, rn, r0, r1, st, move, part,
                                rs);
  }
}

// One wave per row with several tasks or none (single-task rows were solved
// by their task's wave): the row's task partials summed in FP64 (lanes
// stride over the tasks, then a fixed butterfly) and the rank-1 solve
// (lambda + den) x = num (ccd_solve_row).
template <class T, class AT>
__global__ __launch_bounds__(256) void k_ccd_rows(int64_t I, const double *__restrict__ part,
                                                  RowSolve<T, AT> rs) {
  const int lane = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < I;
       i += (int64_t)gridDim.x * 4) {
    const int32_t t0 = rs.row_task[i], t1 = rs.row_task[i + 1];
    if (t1 - t0 == 1) continue;  // uniform over the wave
    double num = 0.0, den = 0.0;
    for (int32_t t = t0 + lane; t < t1; t += 64) {
      num += part[2 * t];
      den += part[2 * t + 1];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      num += __shfl_xor(num, o);
      den += __shfl_xor(den, o);
    }
    if (lane == 0) ccd_solve_row<T, AT>(rs, i, num, den);
  }
}

static unsigned grid_for_n(int64_t n, int64_t cap = 65536) {
  int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

template <class T, class AT, class VT>
static hipError_t ccd_column_t(const tt_index *ix, int r, void *const *d_A, int64_t ldA,
                               double lambda, void *const *rho, void *const *recs,
                               const CcdLayout *const *lay, double *part, int32_t *d_info,
                               hipStream_t s) {
  using R4 = typename Rec4<AT>::type;
  const int N = ix->N;
  for (int n = 0; n < N; ++n) {
    const ModeIndex &md = ix->mode[n];
    ProfScope ps("ccd_column", s, (double)md.I * (sizeof(T) + 2 * sizeof(R4)), 0.0);
    if (md.I > 0)
      k_ccd_column<T, AT><<<grid_for_n(md.I), 256, 0, s>>>((const T *)d_A[n], ldA, md.I, r,
                                                           (R4 *)recs[n]);
  }
  int64_t off = 0;
  for (int n = 0; n < N; ++n) {
    const ModeIndex &md = ix->mode[n];
    int q0 = -1, q1 = -1;
    for (int p = 0; p < N; ++p)
      if (p != n) (q0 < 0 ? q0 : q1) = p;
    // the mode's own stream and tasks, or its CCD++ layout
    const CcdLayout *L = lay ? lay[n] : nullptr;
    const int64_t ntask = L ? L->ntask : md.ntask;
    if (ntask > 0) {
      ProfScope ps("ccd_mode_pass", s, (double)ix->m * (4.0 * 2 + sizeof(VT) * (r > 0 ? 2 : 1)),
                   (double)ix->m * (r > 0 ? 14.0 : 8.0));
      const int32_t *key = L ? L->d_key : md.d_key;
      const int32_t *a0 = L ? L->d_oidx[q0] : md.d_oidx[q0];
      const int32_t *a1 = L ? L->d_oidx[q1] : md.d_oidx[q1];
      const int64_t *tk = L ? L->d_task : md.d_task;
      const int32_t *sched = L ? L->d_sched : nullptr;
      // slots: with the layout's schedule four per scheduled workgroup (one
      // wave per task), else one per task
      const int64_t nslot = L ? 4 * L->nsched : ntask;
      // the smaller other mode's records in LDS when they fit
      const int qs = ix->mode[q0].I <= ix->mode[q1].I ? q0 : q1;
      const int64_t nstage = ix->mode[qs].I;
      const int64_t stage_bytes = nstage * (int64_t)sizeof(R4);
      const bool lds = ix->tune.ccd_lds != 0 && stage_bytes <= kCcdLdsBytes;
      const R4 *rq0 = (const R4 *)recs[q0], *rq1 = (const R4 *)recs[q1];
      const int mv = r > 0 ? 1 : 0;
      const RowSolve<T, AT> rs{L ? L->d_row_task : md.d_row_task, lambda, (T *)d_A[n], ldA, r,
                               (R4 *)recs[n], d_info ? d_info + off : nullptr};
      if (lds) {
        // as many workgroups as are resident at once (registers and LDS
        // copies), a multiple of 8 in all: the workgroups loop over the
        // slots, so a second round would only lengthen the pass
        const size_t shm = (size_t)std::max<int64_t>(stage_bytes, 16);
        auto kern = qs == q0 ? &k_ccd_tasks<T, AT, VT, 64, 0> : &k_ccd_tasks<T, AT, VT, 64, 1>;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, shm) != hipSuccess ||
            per_cu < 1)
          per_cu = 1;
        int64_t grid = std::min<int64_t>((nslot + 3) / 4, (int64_t)per_cu * std::max(ix->cu_count, 8));
        grid = std::max<int64_t>(8, grid / 8 * 8);
        kern<<<(unsigned)grid, 256, shm, s>>>(tk, ntask, sched, nslot, key, a0, a1, (VT *)rho[n],
                                              (const R4 *)recs[n], rq0, rq1, nstage, mv, part,
                                              rs);
      } else {
        k_ccd_tasks<T, AT, VT, 64, -1><<<(unsigned)((nslot + 3) / 4), 256, 0, s>>>(
            tk, ntask, sched, nslot, key, a0, a1, (VT *)rho[n], (const R4 *)recs[n], rq0, rq1, 0,
            mv, part, rs);
      }
    }
    ProfScope ps("ccd_rows", s, (double)ntask * 16 + (double)md.I * (sizeof(T) + sizeof(AT)),
                 (double)ntask * 2);
    if (md.I > 0) {
      // rows with several tasks or none (the others were solved in the pass)
      const RowSolve<T, AT> rs{L ? L->d_row_task : md.d_row_task, lambda, (T *)d_A[n], ldA, r,
                               (R4 *)recs[n], d_info ? d_info + off : nullptr};
      k_ccd_rows<T, AT><<<grid_for_n(64 * md.I, 262144), 256, 0, s>>>(md.I, part, rs);
    }
    off += md.I;
  }
  return hipGetLastError();
}

hipError_t launch_ccd_column(const tt_index *ix, int r, void *const *d_A, int64_t ldA,
                             tt_dtype fdt, double lambda, void *const *rho, void *const *recs,
                             const CcdLayout *const *lay, double *part, int32_t *d_info,
                             hipStream_t s) {
  if (fdt == TT_F64)
    return ccd_column_t<double, double, double>(ix, r, d_A, ldA, lambda, rho, recs, lay, part,
                                                d_info, s);
  if (fdt == TT_F32)
    return ccd_column_t<float, float, float>(ix, r, d_A, ldA, lambda, rho, recs, lay, part,
                                             d_info, s);
  return ccd_column_t<uint16_t, float, float>(ix, r, d_A, ldA, lambda, rho, recs, lay, part,
                                              d_info, s);
}

}  // namespace tt
