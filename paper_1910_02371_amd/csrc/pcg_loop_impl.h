// The conjugate-gradient loop of the Gauss-Newton step (Section 2.5, the
// implicit PCG of its Section 4 implementation) as one persistent kernel
// (included by pcg_loop_f32.hip, pcg_loop_bf16.hip, pcg_loop_f64.hip).
//
// Launched one by one, every CG iteration is about twenty dependent kernels
// (the three passes of the Gauss-Newton product, three dot products with
// their sums and scalar steps, the two vector updates, the preconditioner);
// on tensors of a few 10^5 nonzeros the launches, not the work, set the
// time.  Here a grid of a few workgroups per compute unit runs all
// iterations; the phases of an iteration are separated by grid barriers:
//
//   GN pass (zmode order) | carries | MTTKRP passes of the other two modes
//   (together) | carries | p.Hp partials | alpha; x += alpha p,
//   r -= alpha q with the r.r partials | convergence test;
//   z = P^{-1} r | r.z partials | beta; p = z + beta p, q = lambda2 p
//
// Every phase runs the same device code as the separate kernels (the
// per-chunk streaming body, the carry reductions, the per-row
// preconditioner solve, the elementwise updates) over the same work
// partition, and each dot product is reduced in the same two-level order,
// so the iterates are bit-identical to the launch-by-launch loop.  The
// scalars (alpha, beta, norms, convergence) are computed redundantly by
// every workgroup from the same partials; block 0 stores them at the end.
//
// Grid barrier: two-level monotone arrival counters and a generation word
// (all zeroed before the launch).  Thread 0 of each workgroup arrives with
// agent-scope release order (the last arriver of each level acquires the
// others' writes) and waits until the generation reaches the barrier's
// number, then fences with acquire order; workgroup barriers before and
// after order the other threads.  Arrivals spread over one counter per
// group of workgroups, since same-address atomics serialize.  All
// workgroups are resident at once (the grid is capped by the occupancy
// query), so every wait ends; a wait that still exceeds a spin bound sets
// an abort flag that makes every workgroup leave: the step is then not
// applied, and the stored statistics read iterations = -1 and a NaN
// residual.
//
// Measured on MI355X: a barrier costs a few microseconds, about as much as
// a dependent kernel launch, and a phase with more work chunks than
// resident workgroups takes several rounds of per-chunk latency, so the
// loop pays only where every phase fits in one round (tuning pcg_wgs).
#pragma once
#include <hip/hip_runtime.h>

#include "pcg_loop.h"
#include "solve_impl.h"
#include "stream_impl.h"
#include "vec_impl.h"

namespace tt {

// Barrier words (pcg_loop.h): the generation, the abort flag, the
// top-level arrivals and one arrival counter per group of kBarGroup
// workgroups, each on its own 128-byte line.  A workgroup adds one to its
// group's counter; the last of the group adds one to the top-level
// counter; the last group publishes the new generation.  Every counter
// only grows, so after barrier e a group's counter is e x (its size).
__device__ __forceinline__ bool grid_sync(unsigned *bar, unsigned &epoch, int *lds_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    ++epoch;
    const unsigned nb = gridDim.x;
    const unsigned g = blockIdx.x / kBarGroup;
    const unsigned ngroups = (nb + kBarGroup - 1) / kBarGroup;
    const unsigned gsize = min((unsigned)kBarGroup, nb - g * kBarGroup);
    // arrivals release this workgroup's writes; only the last arriver of a
    // level acquires the others' before passing them on
    const unsigned a = __hip_atomic_fetch_add(&bar[kBarFirstGroup + kBarStride * g], 1u,
                                              __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    if (a + 1 == epoch * gsize) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const unsigned t = __hip_atomic_fetch_add(&bar[kBarTop], 1u, __ATOMIC_RELEASE,
                                                __HIP_MEMORY_SCOPE_AGENT);
      if (t + 1 == epoch * ngroups) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(&bar[kBarGen], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    int ok = 1;
    unsigned spins = 0;
    while (__hip_atomic_load(&bar[kBarGen], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      if (__hip_atomic_load(&bar[kBarAbort], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
          ++spins > kPcgSpinLimit) {
        __hip_atomic_store(&bar[kBarAbort], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *lds_ok = ok;
  }
  __syncthreads();
  return *lds_ok != 0;
}

template <class TR, int G>
struct PcgSmem {
  using X = typename TR::AT;
  union {
    StreamSmem<TR, G, kPcgChunk> st;
    double part[256];
    X lp[4][Packed<kPcgRP>::LDS];
  } u;
  double sc[16];
  int ok;
};

template <class TR, int G, int VM>
__global__ __launch_bounds__(256) void k_pcg_loop(PcgLoopDev a) {
  using X = typename TR::AT;  // dense dtype of the PCG vectors
  __shared__ PcgSmem<TR, G> sm;
  const int tid = threadIdx.x;
  const int64_t nb = gridDim.x;
  unsigned epoch = 0;
  X *x = reinterpret_cast<X *>(a.x), *r = reinterpret_cast<X *>(a.r);
  X *z = reinterpret_cast<X *>(a.z), *p = reinterpret_cast<X *>(a.p);
  X *q = reinterpret_cast<X *>(a.q);
  const int64_t n = a.ntot;
  if (tid < 16) sm.sc[tid] = tid < 10 ? a.sc[tid] : 0.0;
  __syncthreads();
  bool ok = true;

  // Per-pass fields are picked with selects of constant-index loads (a
  // dynamic index into the kernel argument would copy it to scratch).
  auto sel = [](int ps, auto v0, auto v1, auto v2) { return ps == 0 ? v0 : (ps == 1 ? v1 : v2); };
  // the OP_GN pass; then the two OP_MTTKRP passes, chunks numbered consecutively
  auto gn_pass = [&]() {
    for (int64_t c = blockIdx.x; c < a.nchunk[0]; c += nb) {
      stream_chunk<TR, 3, G, VM, OP_GN, kPcgChunk>(a.pass[0], c, sm.u.st);
      __syncthreads();
    }
  };
  auto mttkrp_passes = [&]() {
    const int64_t n1 = a.nchunk[1];
    for (int64_t c = blockIdx.x; c < n1 + a.nchunk[2]; c += nb) {
      if (c < n1)
        stream_chunk<TR, 3, G, VM, OP_MTTKRP, kPcgChunk>(a.pass[1], c, sm.u.st);
      else
        stream_chunk<TR, 3, G, VM, OP_MTTKRP, kPcgChunk>(a.pass[2], c - n1, sm.u.st);
      __syncthreads();
    }
  };
  // heavy-row reductions of passes first..last: segment partials, then rows
  auto nseg_of = [&](int ps) -> int64_t {
    return sel(ps, a.nheavy[0], a.nheavy[1], a.nheavy[2]) > 0
               ? sel(ps, a.nseg[0], a.nseg[1], a.nseg[2])
               : (int64_t)0;
  };
  auto nheavy_of = [&](int ps) -> int64_t { return sel(ps, a.nheavy[0], a.nheavy[1], a.nheavy[2]); };
  auto carries = [&](int first, int last) -> bool {
    int64_t ns = 0, nh = 0;
    for (int ps = first; ps <= last; ++ps) {
      ns += nseg_of(ps);
      nh += nheavy_of(ps);
    }
    if (nh == 0) return true;
    for (int64_t c = blockIdx.x; c < ns; c += nb) {
      int ps = first;
      int64_t k = c;
      while (k >= nseg_of(ps)) k -= nseg_of(ps++);
      carry_partial_seg(sel(ps, a.seg[0], a.seg[1], a.seg[2]),
                        sel(ps, a.pass[0].carry, a.pass[1].carry, a.pass[2].carry), a.srp,
                        sel(ps, a.partial[0], a.partial[1], a.partial[2]), (int)k, sm.u.part);
      __syncthreads();
    }
    if (!grid_sync(a.bar, epoch, &sm.ok)) return false;
    for (int64_t c = blockIdx.x; c < nh; c += nb) {
      int ps = first;
      int64_t k = c;
      while (k >= nheavy_of(ps)) k -= nheavy_of(ps++);
      heavy_fixup_row<X>(sel(ps, a.hrow[0], a.hrow[1], a.hrow[2]),
                         sel(ps, a.hseg[0], a.hseg[1], a.hseg[2]),
                         sel(ps, a.partial[0], a.partial[1], a.partial[2]), a.srp, a.R,
                         sel(ps, a.pass[0].out, a.pass[1].out, a.pass[2].out), 1, (int)k,
                         sm.u.part);
      __syncthreads();
    }
    return grid_sync(a.bar, epoch, &sm.ok);
  };
  // every workgroup sums the same partials in the same order
  auto reduce = [&](const double *parts, int slot, int stage) {
    const double s = sum_parts_block(parts, a.np);
    if (tid == 0) {
      sm.sc[slot] = s;
      pcg_stage(sm.sc, stage, a.tol);
    }
    __syncthreads();
  };
  double *parts0 = a.parts, *parts1 = a.parts + a.np, *parts2 = a.parts + 2 * a.np;

  // q = lambda2 p (the first product's diagonal term)
  for (int64_t i = blockIdx.x * 256 + tid; i < n; i += nb * 256)
    q[i] = scaled<X>(a.lambda2, (double)p[i]);
  ok = grid_sync(a.bar, epoch, &sm.ok);

  for (int it = 0; ok && it < a.kmax && sm.sc[SC_DONE] == 0.0; ++it) {
    // q += (J^T W J) p: the GN pass, then the other modes' MTTKRP passes
    gn_pass();
    if (!(ok = grid_sync(a.bar, epoch, &sm.ok) && carries(0, 0))) break;
    mttkrp_passes();
    if (!(ok = grid_sync(a.bar, epoch, &sm.ok) && carries(1, 2))) break;
    // alpha = r.z / p.q
    for (int64_t vb = blockIdx.x; vb < a.np; vb += nb) {
      const double s = dot_part_block(p, q, n, vb, a.np);
      if (tid == 0) parts0[vb] = s;
    }
    if (!(ok = grid_sync(a.bar, epoch, &sm.ok))) break;
    reduce(parts0, SC_PHP, 1);
    // x += alpha p; r -= alpha q; partials of r.r over the dot partition
    {
      const double al = sm.sc[SC_ALPHA];
      for (int64_t vb = blockIdx.x; vb < a.np; vb += nb) {
        double v = 0.0;
        for (int64_t i = vb * VT_THREADS + tid; i < n; i += a.np * VT_THREADS) {
          axpy2_at(x, p, r, q, i, al);
          v += (double)r[i] * (double)r[i];
        }
        const double s = block_sum_d(v);
        if (tid == 0) parts1[vb] = s;
      }
    }
    if (!(ok = grid_sync(a.bar, epoch, &sm.ok))) break;
    reduce(parts1, SC_RR, 2);
    if (sm.sc[SC_DONE] != 0.0) break;
    // z = P^{-1} r, one wave per row
    {
      const int64_t nrow = a.rowoff[3];
      const int w = tid >> 6;
      for (int64_t gr = blockIdx.x * 4 + w; gr < nrow; gr += nb * 4) {
        const int d = gr < a.rowoff[1] ? 0 : (gr < a.rowoff[2] ? 1 : 2);
        const int64_t r0 = sel(d, a.rowoff[0], a.rowoff[1], a.rowoff[2]);
        const int64_t off = r0 * a.R;
        apply_row<X, kPcgRP>(reinterpret_cast<const X *>(sel(d, a.L[0], a.L[1], a.L[2])),
                             r + off, z + off, a.R, gr - r0, sm.u.lp[w]);
      }
    }
    if (!(ok = grid_sync(a.bar, epoch, &sm.ok))) break;
    // beta = r.z_new / r.z
    for (int64_t vb = blockIdx.x; vb < a.np; vb += nb) {
      const double s = dot_part_block(r, z, n, vb, a.np);
      if (tid == 0) parts2[vb] = s;
    }
    if (!(ok = grid_sync(a.bar, epoch, &sm.ok))) break;
    reduce(parts2, SC_RZNEW, 3);
    // p = z + beta p; q = lambda2 p (the next product's diagonal term)
    {
      const double be = sm.sc[SC_BETA];
      for (int64_t i = blockIdx.x * 256 + tid; i < n; i += nb * 256) {
        const X pi = xpby_at(p, z, i, be);
        p[i] = pi;
        q[i] = scaled<X>(a.lambda2, (double)pi);
      }
    }
    if (!(ok = grid_sync(a.bar, epoch, &sm.ok))) break;
  }
  if (blockIdx.x == 0 && tid == 0) {
    // any workgroup that gave up left its share of the later phases undone
    ok = ok && __hip_atomic_load(&a.bar[kBarAbort], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT) == 0u;
    if (!ok) {
      sm.sc[SC_ITERS] = -1.0;
      sm.sc[SC_REL] = __builtin_nan("");
      sm.sc[SC_DONE] = 1.0;
    }
    for (int i = 0; i < 10; ++i) a.sc[i] = sm.sc[i];
    a.sc[kPcgAbortSlot] = ok ? 0.0 : 1.0;
  }
}

// Workgroups of one launch: wgs per compute unit, capped by the number of
// workgroups that can be resident at once (so that every barrier wait
// ends) and by the largest phase's work.
// Workgroups of k_pcg_loop<TR, G, VM> resident per compute unit (queried
// once per instantiation, on the device of the first call), or -1.
template <class TR, int G, int VM>
int pcg_loop_occupancy_t() {
  static int occ = -1;
  if (occ < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_pcg_loop<TR, G, VM>), 256, 0) != hipSuccess)
      return -1;
    occ = nb;
  }
  return occ;
}

template <class TR, int G, int VM>
hipError_t launch_pcg_loop_t(const PcgLoopDev &a, int wgs_per_cu, int cu_count,
                             hipStream_t s) {
  const int occ = pcg_loop_occupancy_t<TR, G, VM>();
  if (occ < 1) return hipErrorInvalidConfiguration;
  int64_t work = std::max<int64_t>(a.np, (a.rowoff[3] + 3) / 4);
  work = std::max<int64_t>(work, a.nchunk[0]);
  work = std::max<int64_t>(work, a.nchunk[1] + a.nchunk[2]);
  const int64_t grid = std::max<int64_t>(
      1, std::min<int64_t>(std::min<int64_t>(std::min(wgs_per_cu, occ) * (int64_t)cu_count,
                                             kPcgMaxGrid),
                           work));
  k_pcg_loop<TR, G, VM><<<(unsigned)grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

template <class TR, int G>
hipError_t launch_pcg_loop_g(const PcgLoopDev &a, int vm, int wgs_per_cu, int cu_count,
                             hipStream_t s) {
  if (vm == 2) return launch_pcg_loop_t<TR, G, 2>(a, wgs_per_cu, cu_count, s);
  if (vm == 1) return launch_pcg_loop_t<TR, G, 1>(a, wgs_per_cu, cu_count, s);
  return launch_pcg_loop_t<TR, G, 0>(a, wgs_per_cu, cu_count, s);
}

template <class TR, int G>
int pcg_loop_occupancy_g(int vm) {
  if (vm == 2) return pcg_loop_occupancy_t<TR, G, 2>();
  if (vm == 1) return pcg_loop_occupancy_t<TR, G, 1>();
  return pcg_loop_occupancy_t<TR, G, 0>();
}

}  // namespace tt
