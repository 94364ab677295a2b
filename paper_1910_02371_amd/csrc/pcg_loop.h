// Arguments of the persistent conjugate-gradient loop (pcg_loop_impl.h)
// and its per-dtype launchers.
#pragma once
#include <hip/hip_runtime.h>

#include "stream_impl.h"

namespace tt {

constexpr int kPcgChunk = 2048;           // LDS capacity of the streaming phases
constexpr int kPcgRP = 16;                // preconditioner blocks: R <= 16
constexpr unsigned kPcgSpinLimit = 1u << 22;
// grid barrier words (unsigned): generation, abort flag, top-level
// arrivals, then one counter per group of kBarGroup workgroups
constexpr int kBarGen = 0, kBarAbort = 1, kBarTop = 32, kBarFirstGroup = 64, kBarStride = 32;
constexpr int kBarGroup = 16;
#ifndef TT_PCG_MAX_GRID
#define TT_PCG_MAX_GRID 4096
#endif
constexpr int kPcgMaxGrid = TT_PCG_MAX_GRID;  // workgroups of one loop, at most
constexpr int kBarWords = kBarFirstGroup + kBarStride * (kPcgMaxGrid / kBarGroup);

struct PcgLoopDev {
  StreamDev pass[3];            // 0: OP_GN in zmode order; 1, 2: OP_MTTKRP
  int64_t nchunk[3];
  // heavy-row carries of each pass (nheavy = 0: none)
  const int32_t *seg[3];
  const int32_t *hrow[3];
  const int32_t *hseg[3];
  int64_t nseg[3], nheavy[3];
  double *partial[3];
  int srp;                      // carry slot stride (lane group x fragment)
  // preconditioner: row-packed factors per mode, rows of the modes
  const void *L[3];
  int64_t rowoff[4];
  // PCG vectors (dense dtype, all modes' blocks, R per row)
  void *x, *r, *z, *p, *q;
  int64_t ntot;
  int R;
  double lambda2;
  double *parts;                // 3 x np first-level partials
  int64_t np;
  double *sc;                   // scalar slots (in: after stage 0; out: final)
  double tol;
  int kmax;
  unsigned *bar;                // kBarWords barrier words
};

hipError_t launch_pcg_loop_f32(const PcgLoopDev &a, int G, int vm, int wgs_per_cu,
                               int cu_count, hipStream_t s);
hipError_t launch_pcg_loop_bf16(const PcgLoopDev &a, int G, int vm, int wgs_per_cu,
                                int cu_count, hipStream_t s);
hipError_t launch_pcg_loop_f64(const PcgLoopDev &a, int G, int vm, int wgs_per_cu,
                               int cu_count, hipStream_t s);
// resident workgroups per compute unit of the instantiation, or -1
int pcg_loop_occupancy_f32(int G, int vm);
int pcg_loop_occupancy_bf16(int G, int vm);
int pcg_loop_occupancy_f64(int G, int vm);

}  // namespace tt
