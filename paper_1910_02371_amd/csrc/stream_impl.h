// Streaming kernels over one mode's sorted nonzero stream (included by the
// per-dtype translation units stream_f32.hip, stream_bf16.hip,
// stream_f64.hip).
//
// One workgroup (256 threads) takes one chunk of the partition built with
// the index: either whole rows totalling <= CHUNK nonzeros, or one piece of
// a heavy row.  The chunk's sorted mode indices, other-mode indices and
// per-nonzero values are staged into LDS with coalesced loads.  The chunk is
// split into NG = 256 / G contiguous sub-ranges, one per group of G lanes;
// a group holds R on its lanes (V elements per lane, one 16-byte (8-byte for
// BF16) fragment of each factor row) and walks its sub-range in order, gathering the factor
// rows of the other modes.  Rows that begin and end inside a sub-range are
// written directly; pieces cut by sub-range boundaries are combined by an
// in-order scan over the groups; pieces of heavy rows go to FP64 carry slots
// reduced afterwards in a fixed order.  Results are deterministic.
//
// Operations (Section 3.3 TTTP, Section 3.2 MTTKRP, Table 1 / Appendix A
// gradient, Section 2.5 Gauss-Newton matvec):
//   OP_TTTP   out_e = epilogue(s_e or t_e, sum_r prod_n A_n[i_n(e), r])
//   OP_MTTKRP Y[i] += s_e * h_e,            h_e = prod_{p != n} A_p[i_p(e)]
//   OP_GRAD   Y[i] += phi'(t_e, <A_n[i], h_e>) * h_e  (optionally storing phi'')
//   OP_GN     Y[i] += w_e * z_e * h_e,  z_e = <X_n[i], h_e> + <A_n[i], dh_e>,
//             dh_e = sum_{p != n} X_p[i_p(e)] * prod_{q != n, p} A_q[i_q(e)]
//             (optionally also stores w_e * z_e per nonzero, for the other
//             modes' blocks of the same product)
//   OP_NEWTON Y[i] += s_e * dh_e   (the phi' terms of the full Hessian
//             product, Section 2.5 / Appendix A, with s = phi')
#pragma once
#include <hip/hip_runtime.h>

#include "common.h"
#include "internal.h"

namespace tt {

constexpr int ST_THREADS = 256;
constexpr int ST_UNROLL = 4;

// Gather source for a mode that TTTP skips: the row is read (so that the
// gather phase has no branch) and then replaced by ones.
static __device__ double g_skip_row[64];

struct StreamDev {
  const int64_t *chunk;
  const int32_t *chunk_slot;
  const int32_t *key;
  const int32_t *oidx[3];   // streams of the other modes, in mode order
  const void *A_own;        // may be NULL for TTTP (mode skipped)
  const void *A_oth[3];     // may be NULL for TTTP (mode skipped)
  const void *X_own;
  const void *X_oth[3];
  const void *s;            // per-nonzero values (value dtype) or NULL
  const int32_t *s_perm;
  double w_const;
  int R;
  int64_t ldA;
  int epi, loss;
  void *out;
  const int32_t *out_perm;
  int accumulate;
  double *sum_parts;
  double *carry;
  const double *skip;       // when set and *skip != 0 the launch is a no-op
  void *zout;               // per nonzero in sorted order, or NULL: OP_GN w_e * z_e,
                            // OP_GRAD phi''(t_e, m_e)
};

// Device arguments of a streaming pass and its load mode (the VM parameter
// of k_stream), as launch_stream sets them up.
StreamDev stream_dev(StreamOp op, const StreamCall &c, int *vm);

template <class TR, int G, int CHUNK>
struct StreamSmem {
  using VT = typename TR::VT;
  using AT = typename TR::AT;
  static constexpr int NG = ST_THREADS / G;
  static constexpr int RP = G * TR::V;
  int32_t key[CHUNK + 2];
  int32_t oi[2][CHUNK];
  VT val[CHUNK];
  union {
    struct {
      AT piece[NG][2][RP];
      int32_t prow[NG][2];
      int32_t pfl[NG][2];
    } seg;
    struct {
      VT out[CHUNK];
      double part[ST_THREADS / 64];
    } tttp;
  } u;
};

template <class TR, int G, bool VEC>
__device__ __forceinline__ void store_row(void *out, int64_t row, int c0, int R,
                                          int accumulate,
                                          const typename TR::AT (&v)[TR::V]) {
  using AT = typename TR::AT;
  constexpr int V = TR::V;
  AT *o = at32(reinterpret_cast<AT *>(out), (uint32_t)row * (uint32_t)R + c0);
  if (c0 >= R) return;
  if constexpr (VEC) {
    if constexpr (sizeof(AT) == 4) {
#pragma unroll
      for (int q = 0; q < V / 4; ++q) {
        float4 *p4 = reinterpret_cast<float4 *>(o) + q;
        float4 a = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        if (accumulate) {
          float4 b = *p4;
          a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
        }
        *p4 = a;
      }
    } else {
      double2 *p2 = reinterpret_cast<double2 *>(o);
      double2 a = make_double2(v[0], v[1]);
      if (accumulate) {
        double2 b = *p2;
        a.x += b.x; a.y += b.y;
      }
      *p2 = a;
    }
  } else {
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (c0 + j < R) o[j] = accumulate ? o[j] + v[j] : v[j];
  }
}

template <class TR>
__device__ __forceinline__ typename TR::VT load_value(const StreamDev &a, int64_t pos) {
  using VT = typename TR::VT;
  if (a.s == nullptr) return (VT)a.w_const;
  int64_t q = a.s_perm ? (int64_t)a.s_perm[pos] : pos;
  return reinterpret_cast<const VT *>(a.s)[q];
}

// VM selects the loads: 0 element loads everywhere; 1 factor rows as vector
// fragments masked per element (R not a multiple of V, leading dimension
// padded to one) with element loads of the dense blocks (row stride R);
// 2 vector fragments everywhere (R a multiple of V).
//
// stream_chunk processes chunk k with the calling workgroup (256 threads)
// and its LDS block sm; the caller separates two calls on one block with a
// workgroup barrier.
template <class TR, int N, int G, int VM, int OP, int CHUNK>
__device__ __forceinline__ void stream_chunk(const StreamDev &a, int64_t k,
                                             StreamSmem<TR, G, CHUNK> &sm) {
  using T = typename TR::T;
  using VT = typename TR::VT;
  using AT = typename TR::AT;
  constexpr int V = TR::V;
  constexpr bool VA = VM >= 1;              // factor rows as fragments
  constexpr bool VD = VM == 2;              // dense blocks as fragments
  constexpr bool PART = VA && !VD;          // per-element masks on factor rows
  constexpr int NO = N - 1;
  constexpr int NG = ST_THREADS / G;
  static_assert(NO <= 2, "order 3 streams");

  const int tid = threadIdx.x;
  const int64_t b = a.chunk[k];
  const int len = (int)(a.chunk[k + 1] - b);
  const int slot = a.chunk_slot[k];
  if (len <= 0 || len > CHUNK) return;  // partition invariant: 0 < len <= CHUNK
  const bool use_val = (OP == OP_TTTP) ? (a.s != nullptr) : true;

  // ---- stage the chunk into LDS (coalesced) ------------------------------
  for (int i = tid; i < len; i += ST_THREADS) {
    sm.key[i + 1] = a.key[b + i];
#pragma unroll
    for (int p = 0; p < NO; ++p) sm.oi[p][i] = a.oidx[p][b + i];
    if (use_val) sm.val[i] = load_value<TR>(a, b + i);
  }
  if (tid == 0) {
    sm.key[0] = -1;
    sm.key[len + 1] = -1;
  }
  if constexpr (OP != OP_TTTP) {
    if (tid < 2 * NG) (&sm.u.seg.pfl[0][0])[tid] = 0;
  }
  __syncthreads();

  const int g = tid / G;
  const int c0 = (tid % G) * V;
  const int L = (len + NG - 1) / NG;
  const int e0 = min(len, g * L);
  const int e1 = min(len, e0 + L);
  const int R = a.R;
  const int64_t ldA = a.ldA;
  const T *Aown = reinterpret_cast<const T *>(a.A_own);
  const AT *Xown = reinterpret_cast<const AT *>(a.X_own);
  const T *Ao[2] = {reinterpret_cast<const T *>(a.A_oth[0]),
                    NO > 1 ? reinterpret_cast<const T *>(a.A_oth[1]) : nullptr};
  const AT *Xo[2] = {reinterpret_cast<const AT *>(a.X_oth[0]),
                     NO > 1 ? reinterpret_cast<const AT *>(a.X_oth[1]) : nullptr};

  AT acc[V];
#pragma unroll
  for (int j = 0; j < V; ++j) acc[j] = AT(0);
  AT own[V], xown[V];
  double tsum = 0.0;  // TTTP partial sum (FP64)

  auto load_own = [&](int row) {
    if constexpr (OP == OP_TTTP || OP == OP_GRAD || OP == OP_GN) {
      if (Aown) {
        load_frag<TR, VA, PART>(Aown, ldA, row, c0, R, own);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j) own[j] = (c0 + j < R) ? AT(1) : AT(0);
      }
    }
    if constexpr (OP == OP_GN) load_dense<AT, V, VD>(Xown, row, c0, R, xown);
  };

  bool first_piece = true;
  auto emit = [&](int row, bool ol, bool orr) {
    if constexpr (OP != OP_TTTP) {
      if (!ol && !orr && slot < 0) {
        store_row<TR, G, VD>(a.out, row, c0, R, a.accumulate, acc);
      } else {
        int which = first_piece ? 0 : 1;
#pragma unroll
        for (int j = 0; j < V; ++j) sm.u.seg.piece[g][which][c0 + j] = acc[j];
        if (c0 == 0) {
          sm.u.seg.prow[g][which] = row;
          sm.u.seg.pfl[g][which] = (ol ? 1 : 0) | (orr ? 2 : 0) | 4;
        }
      }
    }
    first_piece = false;
  };

  if (e0 < e1) {
    int cur = sm.key[e0 + 1];
    bool ol = sm.key[e0] == cur;
    load_own(cur);
    for (int eb = e0; eb < e1; eb += ST_UNROLL) {
      // gathers of ST_UNROLL nonzeros, issued back to back and kept raw until
      // used; slots past the end of the sub-range reload its last nonzero and
      // are skipped below
      FragRaw<TR, VA> ra[ST_UNROLL][2];
      FragRaw<DenseTr<AT>, VD> rx[ST_UNROLL][2];
#pragma unroll
      for (int u = 0; u < ST_UNROLL; ++u) {
        const int e = min(eb + u, e1 - 1);
#pragma unroll
        for (int p = 0; p < NO; ++p) {
          const int ip = sm.oi[p][e];
          if constexpr (OP == OP_TTTP) {
            const bool skip = Ao[p] == nullptr;
            gather_frag<TR, VA>(skip ? reinterpret_cast<const T *>(g_skip_row) : Ao[p], ldA,
                                 skip ? 0 : ip, c0, R, ra[u][p]);
          } else {
            gather_frag<TR, VA>(Ao[p], ldA, ip, c0, R, ra[u][p]);
          }
          if constexpr (OP == OP_GN || OP == OP_NEWTON)
            gather_frag<DenseTr<AT>, VD>(Xo[p], R, ip, c0, R, rx[u][p]);
        }
      }
#pragma unroll
      for (int u = 0; u < ST_UNROLL; ++u) {
        const int e = eb + u;
        AT fa[2][V], fx[2][V];
#pragma unroll
        for (int p = 0; p < NO; ++p) {
          if (OP == OP_TTTP && Ao[p] == nullptr) {
#pragma unroll
            for (int j = 0; j < V; ++j) fa[p][j] = (c0 + j < R) ? AT(1) : AT(0);
          } else {
            widen_frag<TR, VA, PART>(ra[u][p], c0, R, fa[p]);
          }
          if constexpr (OP == OP_GN || OP == OP_NEWTON)
            widen_frag<DenseTr<AT>, VD>(rx[u][p], c0, R, fx[p]);
        }
        if (e < e1) {
          const int row = sm.key[e + 1];
          if (row != cur) {
            emit(cur, ol, false);
#pragma unroll
            for (int j = 0; j < V; ++j) acc[j] = AT(0);
            cur = row;
            ol = false;
            load_own(cur);
          }
          // h = Hadamard product of the other modes' fragments
          AT h[V];
#pragma unroll
          for (int j = 0; j < V; ++j) {
            h[j] = fa[0][j];
#pragma unroll
            for (int p = 1; p < NO; ++p) h[j] *= fa[p][j];
          }
          if constexpr (OP == OP_MTTKRP) {
            const AT sv = (AT)sm.val[e];
#pragma unroll
            for (int j = 0; j < V; ++j) acc[j] += sv * h[j];
          } else if constexpr (OP == OP_GRAD) {
            AT d = AT(0);
#pragma unroll
            for (int j = 0; j < V; ++j) d += own[j] * h[j];
            const AT mval = group_sum<G>(d);
            const AT dp = loss_eval<AT>(EPI_DPHI, a.loss, (AT)sm.val[e], mval);
#pragma unroll
            for (int j = 0; j < V; ++j) acc[j] += dp * h[j];
            if (a.zout != nullptr && c0 == 0)
              reinterpret_cast<VT *>(a.zout)[b + e] =
                  (VT)loss_eval<AT>(EPI_D2PHI, a.loss, (AT)sm.val[e], mval);
          } else if constexpr (OP == OP_GN) {
            // sums of two products are written as explicit fused
            // multiply-adds: left to contraction, the compiler may fuse
            // either product, and differently in different load modes
            AT zz = AT(0);
#pragma unroll
            for (int j = 0; j < V; ++j) {
              AT dh;
              if constexpr (NO == 1) {
                dh = fx[0][j];
              } else {
                dh = fma(fx[0][j], fa[1][j], fa[0][j] * fx[1][j]);
              }
              zz += fma(own[j], dh, xown[j] * h[j]);
            }
            const AT z = group_sum<G>(zz);
            const AT wz = (AT)sm.val[e] * z;
#pragma unroll
            for (int j = 0; j < V; ++j) acc[j] += wz * h[j];
            if (a.zout != nullptr && c0 == 0) reinterpret_cast<VT *>(a.zout)[b + e] = (VT)wz;
          } else if constexpr (OP == OP_NEWTON) {
            const AT sv = (AT)sm.val[e];
#pragma unroll
            for (int j = 0; j < V; ++j) {
              AT dh;
              if constexpr (NO == 1) {
                dh = fx[0][j];
              } else {
                dh = fma(fx[0][j], fa[1][j], fa[0][j] * fx[1][j]);
              }
              acc[j] += sv * dh;
            }
          } else {  // OP_TTTP
            AT d = AT(0);
#pragma unroll
            for (int j = 0; j < V; ++j) d += own[j] * h[j];
            const AT mval = group_sum<G>(d);
            AT o;
            if (a.epi == EPI_NONE)
              o = use_val ? (AT)sm.val[e] * mval : mval;
            else
              o = loss_eval<AT>(a.epi, a.loss, (AT)sm.val[e], mval);
            if (c0 == 0) {
              sm.u.tttp.out[e] = (VT)o;
              tsum += (double)(VT)o;
            }
          }
        }
      }
    }
    if constexpr (OP != OP_TTTP) emit(cur, ol, sm.key[e1 + 1] == cur);
  }
  __syncthreads();

  if constexpr (OP == OP_TTTP) {
    VT *out = reinterpret_cast<VT *>(a.out);
    for (int i = tid; out != nullptr && i < len; i += ST_THREADS) {
      const int64_t dst = a.out_perm ? (int64_t)a.out_perm[b + i] : b + i;
      out[dst] = sm.u.tttp.out[i];
    }
    if (a.sum_parts) {
      // fixed-order FP64 reduction: wave butterfly, then waves in order
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) tsum += __shfl_xor(tsum, o);
      if ((tid & 63) == 0) sm.u.tttp.part[tid >> 6] = tsum;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < ST_THREADS / 64; ++w) s += sm.u.tttp.part[w];
        a.sum_parts[k] = s;
      }
    }
  } else {
    // in-order scan over the groups' open pieces (group 0's lanes)
    if (g == 0) {
      AT run[V];
#pragma unroll
      for (int j = 0; j < V; ++j) run[j] = AT(0);
      int run_row = -1;
      bool active = false;
      auto finalize = [&]() {
        if (slot >= 0) {
          double *cs = a.carry + (int64_t)slot * StreamSmem<TR, G, CHUNK>::RP + c0;
#pragma unroll
          for (int j = 0; j < V; ++j) cs[j] = (double)run[j];
        } else {
          store_row<TR, G, VD>(a.out, run_row, c0, R, a.accumulate, run);
        }
        active = false;
      };
      for (int gg = 0; gg < NG; ++gg) {
        const int f0 = sm.u.seg.pfl[gg][0];
        if (f0) {
          if ((f0 & 1) && active) {
#pragma unroll
            for (int j = 0; j < V; ++j) run[j] += sm.u.seg.piece[gg][0][c0 + j];
          } else {
#pragma unroll
            for (int j = 0; j < V; ++j) run[j] = sm.u.seg.piece[gg][0][c0 + j];
            run_row = sm.u.seg.prow[gg][0];
            active = true;
          }
          if (!(f0 & 2)) finalize();
        }
        const int f1 = sm.u.seg.pfl[gg][1];
        if (f1) {
#pragma unroll
          for (int j = 0; j < V; ++j) run[j] = sm.u.seg.piece[gg][1][c0 + j];
          run_row = sm.u.seg.prow[gg][1];
          active = true;
          if (!(f1 & 2)) finalize();
        }
      }
      if (active) finalize();
    }
  }
}

template <class TR, int N, int G, int VM, int OP, int CHUNK>
__global__ __launch_bounds__(ST_THREADS) void k_stream(StreamDev a) {
  __shared__ StreamSmem<TR, G, CHUNK> sm;
  if (a.skip && *a.skip != 0.0) return;
  stream_chunk<TR, N, G, VM, OP, CHUNK>(a, blockIdx.x, sm);
}

// Heavy rows, first level: each block sums one segment of <= kSegSlots
// consecutive carry slots (strided over 256/RP partial lanes, then a fixed
// tree) into an FP64 partial.
__device__ __forceinline__ void carry_partial_seg(const int32_t *__restrict__ seg,
                                                  const double *__restrict__ carry, int RP,
                                                  double *__restrict__ partial, int g,
                                                  double (&part)[256]) {
  const int tid = threadIdx.x;
  const int lanes = 256 / RP;
  const int r = tid % RP, q = tid / RP;
  const int s0 = seg[g], s1 = seg[g + 1];
  double s = 0.0;
  for (int sl = s0 + q; sl < s1; sl += lanes) s += carry[(int64_t)sl * RP + r];
  part[tid] = s;
  __syncthreads();
  for (int w = lanes / 2; w > 0; w >>= 1) {
    if (q < w) part[tid] += part[tid + w * RP];
    __syncthreads();
  }
  if (q == 0) partial[(int64_t)g * RP + r] = part[tid];
}

static __global__ __launch_bounds__(256) void k_carry_partial(const int32_t *__restrict__ seg,
                                                       const double *__restrict__ carry,
                                                       int RP, double *__restrict__ partial,
                                                       const double *skip) {
  __shared__ double part[256];
  if (skip && *skip != 0.0) return;
  carry_partial_seg(seg, carry, RP, partial, blockIdx.x, part);
}

// Heavy rows, second level: sum the FP64 partials of each heavy row in order
// (strided over 256/RP partial lanes, then a fixed tree) and store.
template <class AT>
__device__ __forceinline__ void heavy_fixup_row(const int32_t *__restrict__ hrow,
                                                const int32_t *__restrict__ hslot,
                                                const double *__restrict__ carry, int RP, int R,
                                                void *out, int accumulate, int h,
                                                double (&part)[256]) {
  const int tid = threadIdx.x;
  const int lanes = 256 / RP;
  const int r = tid % RP, q = tid / RP;
  const int s0 = hslot[h], s1 = hslot[h + 1];
  double s = 0.0;
  if (q < lanes)
    for (int sl = s0 + q; sl < s1; sl += lanes) s += carry[(int64_t)sl * RP + r];
  part[tid] = s;
  __syncthreads();
  for (int w = lanes / 2; w > 0; w >>= 1) {
    if (q < w) part[tid] += part[tid + w * RP];
    __syncthreads();
  }
  if (q == 0 && r < R) {
    AT *o = reinterpret_cast<AT *>(out) + (int64_t)hrow[h] * R + r;
    double v = part[tid];
    *o = accumulate ? (AT)((double)*o + v) : (AT)v;
  }
}

template <class AT>
__global__ __launch_bounds__(256) void k_heavy_fixup(const int32_t *__restrict__ hrow,
                                                     const int32_t *__restrict__ hslot,
                                                     const double *__restrict__ carry,
                                                     int RP, int R, void *out,
                                                     int accumulate, const double *skip) {
  __shared__ double part[256];
  if (skip && *skip != 0.0) return;
  heavy_fixup_row<AT>(hrow, hslot, carry, RP, R, out, accumulate, blockIdx.x, part);
}

template <class TR, int N, int G, int VM, int CHUNK>
hipError_t launch_stream_t(StreamOp op, const StreamDev &d, int64_t nchunk,
                           hipStream_t s) {
  if (nchunk <= 0) return hipSuccess;
  dim3 grid((unsigned)nchunk), block(ST_THREADS);
  switch (op) {
    case OP_TTTP: k_stream<TR, N, G, VM, OP_TTTP, CHUNK><<<grid, block, 0, s>>>(d); break;
    case OP_MTTKRP: k_stream<TR, N, G, VM, OP_MTTKRP, CHUNK><<<grid, block, 0, s>>>(d); break;
    case OP_GRAD: k_stream<TR, N, G, VM, OP_GRAD, CHUNK><<<grid, block, 0, s>>>(d); break;
    case OP_GN: k_stream<TR, N, G, VM, OP_GN, CHUNK><<<grid, block, 0, s>>>(d); break;
    case OP_NEWTON: k_stream<TR, N, G, VM, OP_NEWTON, CHUNK><<<grid, block, 0, s>>>(d); break;
  }
  return hipGetLastError();
}

// The vector paths have one instantiation per supported chunk size (the LDS
// footprint sets the occupancy); the element path, for unaligned factors,
// uses the largest, which serves every chunk size.
template <class TR, int G, int VM>
hipError_t launch_stream_vm(StreamOp op, const StreamDev &d, int64_t nchunk, int chunk,
                            hipStream_t s) {
  switch (chunk) {
    case 512: return launch_stream_t<TR, 3, G, VM, 512>(op, d, nchunk, s);
    case 1024: return launch_stream_t<TR, 3, G, VM, 1024>(op, d, nchunk, s);
    default: return launch_stream_t<TR, 3, G, VM, 2048>(op, d, nchunk, s);
  }
}

template <class TR, int G>
hipError_t launch_stream_g(StreamOp op, const StreamDev &d, int64_t nchunk, int vm,
                           int chunk, hipStream_t s) {
  if (vm == 2) return launch_stream_vm<TR, G, 2>(op, d, nchunk, chunk, s);
  if (vm == 1) return launch_stream_vm<TR, G, 1>(op, d, nchunk, chunk, s);
  return launch_stream_t<TR, 3, G, 0, 2048>(op, d, nchunk, s);
}

}  // namespace tt
