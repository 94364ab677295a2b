// Index construction: per-mode stable counting sort of the nonzeros
// (Section 3.4 sorts by the mode-n index with a counting sort; ties keep
// COO order), row pointers, nonzero rows (Section 3.1 compressed rows) and
// the work partitions of the streaming and Gram kernels.
//
// The sort is an LSD radix sort with 4-bit digits: per pass a block digit
// histogram, an exclusive scan of the digit-major (digit, block) counts, and
// a stable scatter whose in-block ranks follow (thread, item) order, so every
// pass is stable and the result equals a stable argsort, bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "common.h"
#include "internal.h"

namespace tt {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;  // 2048 keys per block
constexpr int RS_BITS = 4;
constexpr int RS_BINS = 1 << RS_BITS;

// ---------------------------------------------------------------------------
__global__ void k_range_check(const int32_t *__restrict__ idx, int64_t m,
                              int64_t I, int *flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0;
  for (; i < m; i += stride) {
    int32_t v = idx[i];
    bad |= (v < 0) | ((int64_t)v >= I);
  }
  if (bad) atomicOr(flag, 1);
}

// Digit histogram of one tile per block, written digit-major:
// hist[d * nblocks + b].
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(
    const uint32_t *__restrict__ keys, int64_t m, int shift, int64_t nblocks,
    uint32_t *__restrict__ hist) {
  __shared__ uint32_t cnt[RS_BINS];
  if (threadIdx.x < RS_BINS) cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int j = 0; j < RS_ITEMS; ++j) {
    int64_t e = base + (int64_t)j * RS_THREADS + threadIdx.x;
    if (e < m) atomicAdd(&cnt[(keys[e] >> shift) & (RS_BINS - 1)], 1u);
  }
  __syncthreads();
  if (threadIdx.x < RS_BINS)
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Block-wide exclusive scan of one value per thread (256 threads); returns
// the exclusive prefix and writes the block total to *total.
__device__ uint32_t block_exscan_u32(uint32_t v, uint32_t *total) {
  __shared__ uint32_t wsum[RS_THREADS / 64];
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < RS_THREADS / 64; ++k) {
    uint32_t s = wsum[k];
    if (k < w) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

// Stable scatter of one tile: thread t owns items [t*ITEMS, (t+1)*ITEMS) of
// the tile (blocked arrangement), so (thread, item) order is input order.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    uint32_t *__restrict__ kout, uint32_t *__restrict__ vout, int64_t m,
    int shift, int64_t nblocks, const uint32_t *__restrict__ offs, int first) {
  __shared__ uint32_t cnt[RS_BINS * RS_THREADS];  // [digit][thread]
  __shared__ uint32_t dstart[RS_BINS];
  const int t = threadIdx.x;
  for (int d = 0; d < RS_BINS; ++d) cnt[d * RS_THREADS + t] = 0;
  int64_t base = (int64_t)blockIdx.x * RS_TILE + (int64_t)t * RS_ITEMS;
  uint32_t k[RS_ITEMS], v[RS_ITEMS];
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    int64_t e = base + j;
    if (e < m) {
      k[j] = kin[e];
      v[j] = first ? (uint32_t)e : vin[e];
      cnt[((k[j] >> shift) & (RS_BINS - 1)) * RS_THREADS + t] += 1;
    }
  }
  __syncthreads();
  // exclusive scan of cnt flattened digit-major; thread t owns 16
  // consecutive counters
  uint32_t loc[RS_BINS];
  uint32_t run = 0;
#pragma unroll
  for (int j = 0; j < RS_BINS; ++j) {
    loc[j] = cnt[t * RS_BINS + j];
    run += loc[j];
  }
  uint32_t tot;
  uint32_t pre = block_exscan_u32(run, &tot);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RS_BINS; ++j) {
    cnt[t * RS_BINS + j] = pre;
    pre += loc[j];
  }
  __syncthreads();
  if (t < RS_BINS) dstart[t] = cnt[t * RS_THREADS];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RS_ITEMS; ++j) {
    int64_t e = base + j;
    if (e < m) {
      int d = (k[j] >> shift) & (RS_BINS - 1);
      uint32_t r = cnt[d * RS_THREADS + t]++;
      uint64_t pos = (uint64_t)offs[(int64_t)d * nblocks + blockIdx.x] + (r - dstart[d]);
      if (pos < (uint64_t)m) {
        kout[pos] = k[j];
        vout[pos] = v[j];
      }
    }
  }
}

// Generic exclusive scan of uint32 (reduce-then-scan, recursive).
constexpr int SC_THREADS = 256, SC_ITEMS = 16, SC_TILE = SC_THREADS * SC_ITEMS;

__global__ __launch_bounds__(SC_THREADS) void k_scan_reduce(
    const uint32_t *__restrict__ in, int64_t n, uint32_t *__restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * SC_TILE;
  uint32_t s = 0;
  for (int j = 0; j < SC_ITEMS; ++j) {
    int64_t e = base + (int64_t)j * SC_THREADS + threadIdx.x;
    if (e < n) s += in[e];
  }
  uint32_t tot;
  block_exscan_u32(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SC_THREADS) void k_scan_down(
    const uint32_t *__restrict__ in, int64_t n, const uint32_t *__restrict__ offs,
    uint32_t *__restrict__ out) {
  int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
  uint32_t loc[SC_ITEMS];
  uint32_t run = 0;
#pragma unroll
  for (int j = 0; j < SC_ITEMS; ++j) {
    int64_t e = base + j;
    loc[j] = e < n ? in[e] : 0u;
    run += loc[j];
  }
  uint32_t tot;
  uint32_t pre = block_exscan_u32(run, &tot) + (offs ? offs[blockIdx.x] : 0u);
#pragma unroll
  for (int j = 0; j < SC_ITEMS; ++j) {
    int64_t e = base + j;
    if (e < n) out[e] = pre;
    pre += loc[j];
  }
}

static int64_t scan_tmp_words(int64_t n) {
  int64_t w = 0;
  while (n > SC_TILE) {
    n = (n + SC_TILE - 1) / SC_TILE;
    w += n + 1;
  }
  return w + 1;
}

static hipError_t exscan_u32(const uint32_t *in, uint32_t *out, int64_t n,
                             uint32_t *tmp, hipStream_t s) {
  int64_t nb = (n + SC_TILE - 1) / SC_TILE;
  if (nb <= 1) {
    k_scan_down<<<1, SC_THREADS, 0, s>>>(in, n, nullptr, out);
    return hipGetLastError();
  }
  uint32_t *sums = tmp;
  uint32_t *sums_scan = tmp + nb;  // scanned in place into sums_scan region
  k_scan_reduce<<<nb, SC_THREADS, 0, s>>>(in, n, sums);
  hipError_t e = exscan_u32(sums, sums, nb, sums_scan, s);
  if (e != hipSuccess) return e;
  k_scan_down<<<nb, SC_THREADS, 0, s>>>(in, n, sums, out);
  return hipGetLastError();
}

// ptr[i] = first sorted position whose key >= i, for i in [0, I].
__global__ void k_row_ptr(const uint32_t *__restrict__ key, int64_t m, int64_t I,
                          int64_t *__restrict__ ptr) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > I) return;
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((int64_t)key[mid] < i) lo = mid + 1; else hi = mid;
  }
  ptr[i] = lo;
}

__global__ void k_gather_i32(const int32_t *__restrict__ src,
                             const uint32_t *__restrict__ perm, int64_t m,
                             int32_t *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < m; i += stride) {
    const uint32_t q = perm[i];
    dst[i] = q < (uint64_t)m ? src[q] : 0;
  }
}

template <class X>
__global__ void k_gather_val(const X *__restrict__ src, const uint32_t *__restrict__ perm,
                             int64_t m, X *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < m; i += stride) {
    const uint32_t q = perm[i];
    dst[i] = q < (uint64_t)m ? src[q] : X(0);
  }
}

__global__ void k_copy_u32(const int32_t *__restrict__ src, int64_t m,
                           uint32_t *__restrict__ dst) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < m; i += stride) dst[i] = (uint32_t)src[i];
}

__global__ void k_iota_u32(uint32_t *__restrict__ dst, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < m; i += stride) dst[i] = (uint32_t)i;
}

// inv[perm[q]] = q: the inverse of a sorted-position -> COO-position map
__global__ void k_inv_perm(const int32_t *__restrict__ perm, int64_t m,
                           int32_t *__restrict__ inv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < m; i += stride) {
    const uint32_t q = (uint32_t)perm[i];
    if (q < (uint64_t)m) inv[q] = (int32_t)i;
  }
}

// ---------------------------------------------------------------------------
static int grid_for(int64_t n, int threads, int cap = 65536);

// Stable LSD radix sort of the m keys in kA (all below `range`) with their
// input positions: on return *kout / *vout point at the sorted keys and the
// input position of each (each is one of kA/kB, vA/vB; all four hold m
// words).  hist and offs hold ceil(m / RS_TILE) * RS_BINS words, tmp
// scan_tmp_words of that.
static hipError_t radix_sort_positions(uint32_t *kA, uint32_t *kB, uint32_t *vA, uint32_t *vB,
                                       int64_t m, int64_t range, uint32_t *hist,
                                       uint32_t *offs, uint32_t *tmp, hipStream_t s,
                                       uint32_t **kout, uint32_t **vout) {
  const int64_t nblocks = std::max<int64_t>(1, (m + RS_TILE - 1) / RS_TILE);
  const int64_t hn = nblocks * RS_BINS;
  int bits = 0;
  while (bits < 31 && ((int64_t)1 << bits) < range) ++bits;
  const int passes = (bits + RS_BITS - 1) / RS_BITS;
  uint32_t *kc = kA, *vc = vA, *kn = kB, *vn = vB;
  hipError_t he = hipSuccess;
  if (passes == 0) k_iota_u32<<<grid_for(m, 256), 256, 0, s>>>(vc, m);
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RS_BITS;
    k_rs_hist<<<nblocks, RS_THREADS, 0, s>>>(kc, m, shift, nblocks, hist);
    if ((he = exscan_u32(hist, offs, hn, tmp, s)) != hipSuccess) return he;
    k_rs_scatter<<<nblocks, RS_THREADS, 0, s>>>(kc, vc, kn, vn, m, shift, nblocks, offs,
                                                p == 0);
    std::swap(kc, kn);
    std::swap(vc, vn);
  }
  *kout = kc;
  *vout = vc;
  return hipGetLastError();
}

static int grid_for(int64_t n, int threads, int cap) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

template <class X>
static tt_status dev_alloc(tt_index *ix, X **p, size_t count) {
  void *q = nullptr;
  size_t bytes = std::max<size_t>(count, 1) * sizeof(X);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return TT_ERR_OOM;
  }
  ix->owned.push_back(q);
  *p = (X *)q;
  return TT_OK;
}

#define TT_ST(x)                          \
  do {                                    \
    tt_status _s = (x);                   \
    if (_s != TT_OK) return _s;           \
  } while (0)

// Device copy of a host vector, recorded in `list` (freed by the caller).
template <class X>
static tt_status upload(std::vector<void *> &list, X **p, const std::vector<X> &h,
                        hipStream_t s) {
  const size_t n = std::max<size_t>(h.size(), 1);
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(X));
  if (e != hipSuccess) {
    set_error("hipMalloc of %zu bytes failed: %s", n * sizeof(X), hipGetErrorString(e));
    return TT_ERR_OOM;
  }
  list.push_back(q);
  *p = (X *)q;
  if (!h.empty())
    TT_HIP(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(X), hipMemcpyHostToDevice, s));
  return TT_OK;
}

// Device array of `count` elements recorded in `list` (freed by the caller).
template <class X>
static tt_status dev_alloc_list(std::vector<void *> &list, X **p, int64_t count) {
  void *q = nullptr;
  const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(X);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    return TT_ERR_OOM;
  }
  list.push_back(q);
  *p = (X *)q;
  return TT_OK;
}

static void partitions(const std::vector<int64_t> &ptr, ModeIndex &md, int64_t kChunk,
                       int64_t kGramPiece, std::vector<int64_t> &chunk,
                       std::vector<int32_t> &slot, std::vector<int32_t> &heavy_row,
                       std::vector<int32_t> &heavy_slot, std::vector<int32_t> &rows,
                       std::vector<int64_t> &task, std::vector<int32_t> &row_task);

// (Re)build the streaming chunks, carry segments, Gram tasks and their
// heavy/multi-task lists of mode n from its host row pointers and the
// index's tuning; frees the previous partition arrays first.
tt_status build_partitions(tt_index *ix, int n, hipStream_t s) {
  ModeIndex &md = ix->mode[n];
  hipError_t he;
  if (!md.part.empty()) {
    TT_HIP(hipStreamSynchronize(s));
    for (void *q : md.part) hipFree(q);
    md.part.clear();
  }
  md.ccd = CcdLayout{};  // its arrays were in `part`; rebuilt on next use
  std::vector<int64_t> chunk, task;
  std::vector<int32_t> slot, hrow, hslot, rows, row_task;
  partitions(md.h_ptr, md, ix->tune.chunk, ix->tune.gram_piece, chunk, slot, hrow, hslot, rows,
             task, row_task);
  std::vector<void *> &L = md.part;
  TT_ST(upload(L, &md.d_chunk, chunk, s));
  TT_ST(upload(L, &md.d_chunk_slot, slot, s));
  TT_ST(upload(L, &md.d_heavy_row, hrow, s));
  TT_ST(upload(L, &md.d_heavy_slot, hslot, s));
  // carry segments: each heavy row's slots split into runs of kSegSlots
  std::vector<int32_t> seg(1, 0), hseg(1, 0);
  for (size_t h = 0; h + 1 < hslot.size(); ++h) {
    for (int32_t a = hslot[h]; a < hslot[h + 1]; a += kSegSlots)
      seg.push_back(std::min<int32_t>(hslot[h + 1], a + kSegSlots));
    hseg.push_back((int32_t)seg.size() - 1);
  }
  md.nseg = (int64_t)seg.size() - 1;
  TT_ST(upload(L, &md.d_seg, seg, s));
  TT_ST(upload(L, &md.d_heavy_seg, hseg, s));
  TT_ST(upload(L, &md.d_rows, rows, s));
  TT_ST(upload(L, &md.d_task, task, s));
  TT_ST(upload(L, &md.d_row_task, row_task, s));
  md.h_row_task = row_task;
  md.h_task = task;
  md.h_multi_row.clear();
  for (int64_t i = 0; i < md.I; ++i)
    if (row_task[i + 1] - row_task[i] > kReduceMin) md.h_multi_row.push_back((int32_t)i);
  // rows by their tasks: one light task (solo), one heavy task (heavy
  // solo), the others (several tasks, or none); the heavy and the light
  // tasks of the rows with several tasks
  const int64_t light = ix->tune.gram_light;
  md.h_solo_row.clear();
  md.h_hsolo_row.clear();
  md.h_rest_row.clear();
  md.h_light_task.clear();
  md.h_heavy_task.clear();
  md.h_solo_nnz.assign(1, 0);
  md.h_hsolo_nnz.assign(1, 0);
  md.h_heavy_nnz.assign(1, 0);
  md.h_heavy_task_all.clear();
  md.h_heavy_nnz_all.assign(1, 0);
  md.h_rest_row_all.clear();
  for (int64_t i = 0; i < md.I; ++i) {
    const int32_t a = row_task[i], b = row_task[i + 1];
    for (int32_t q = a; q < b; ++q) {
      const int64_t nz = task[q + 1] - task[q];
      if (nz > light) {
        md.h_heavy_task_all.push_back(q);
        md.h_heavy_nnz_all.push_back(md.h_heavy_nnz_all.back() + nz);
      }
    }
    if (b - a == 1) {
      const int64_t nz = task[a + 1] - task[a];
      if (nz <= light) {
        md.h_solo_row.push_back((int32_t)i);
        md.h_solo_nnz.push_back(md.h_solo_nnz.back() + nz);
      } else {
        md.h_hsolo_row.push_back((int32_t)i);
        md.h_rest_row_all.push_back((int32_t)i);
        md.h_hsolo_nnz.push_back(md.h_hsolo_nnz.back() + nz);
      }
      continue;
    }
    md.h_rest_row.push_back((int32_t)i);
    md.h_rest_row_all.push_back((int32_t)i);
    for (int32_t q = a; q < b; ++q) {
      const int64_t nz = task[q + 1] - task[q];
      if (nz <= light) {
        md.h_light_task.push_back(q);
      } else {
        md.h_heavy_task.push_back(q);
        md.h_heavy_nnz.push_back(md.h_heavy_nnz.back() + nz);
      }
    }
  }
  TT_ST(upload(L, &md.d_heavy_task, md.h_heavy_task, s));
  TT_ST(upload(L, &md.d_multi_row, md.h_multi_row, s));
  TT_ST(upload(L, &md.d_solo_row, md.h_solo_row, s));
  TT_ST(upload(L, &md.d_hsolo_row, md.h_hsolo_row, s));
  TT_ST(upload(L, &md.d_rest_row, md.h_rest_row, s));
  TT_ST(upload(L, &md.d_light_task, md.h_light_task, s));
  TT_ST(upload(L, &md.d_heavy_task_all, md.h_heavy_task_all, s));
  TT_ST(upload(L, &md.d_rest_row_all, md.h_rest_row_all, s));
  // uploads are asynchronous from pageable vectors: wait before they go
  if ((he = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(he, "upload");
  ix->max_nchunk = ix->max_nslot = ix->max_nseg = 0;
  for (int d = 0; d < ix->N; ++d) {
    ix->max_nchunk = std::max(ix->max_nchunk, ix->mode[d].nchunk);
    ix->max_nslot = std::max(ix->max_nslot, ix->mode[d].nslot);
    ix->max_nseg = std::max(ix->max_nseg, ix->mode[d].nseg);
  }
  return TT_OK;
}


// Host-side partitions from the row pointers of one mode.
static void partitions(const std::vector<int64_t> &ptr, ModeIndex &md, int64_t kChunk,
                       int64_t kGramPiece, std::vector<int64_t> &chunk,
                       std::vector<int32_t> &slot, std::vector<int32_t> &heavy_row,
                       std::vector<int32_t> &heavy_slot, std::vector<int32_t> &rows,
                       std::vector<int64_t> &task, std::vector<int32_t> &row_task) {
  const int64_t I = md.I;
  chunk.clear(); slot.clear(); heavy_row.clear(); heavy_slot.clear();
  rows.clear(); task.clear(); row_task.assign(I + 1, 0);
  int64_t cur_begin = 0, cur_count = 0, nslot = 0;
  chunk.push_back(0);
  task.push_back(0);
  int32_t max_tpr = 0;
  for (int64_t i = 0; i < I; ++i) {
    int64_t b = ptr[i], e = ptr[i + 1], c = e - b;
    row_task[i] = (int32_t)(task.size() - 1);
    if (c == 0) continue;
    rows.push_back((int32_t)i);
    // Gram tasks
    int32_t nt = 0;
    for (int64_t p = b; p < e; p += kGramPiece) {
      task.push_back(std::min<int64_t>(e, p + kGramPiece));
      ++nt;
    }
    max_tpr = std::max(max_tpr, nt);
    // streaming chunks
    if (c > kChunk) {
      if (cur_count > 0) {
        chunk.push_back(b);
        slot.push_back(-1);
      }
      heavy_row.push_back((int32_t)i);
      heavy_slot.push_back((int32_t)nslot);
      for (int64_t p = b; p < e; p += kChunk) {
        chunk.push_back(std::min<int64_t>(e, p + kChunk));
        slot.push_back((int32_t)nslot++);
      }
      cur_begin = e;
      cur_count = 0;
    } else {
      if (cur_count + c > kChunk) {
        chunk.push_back(b);
        slot.push_back(-1);
        cur_begin = b;
        cur_count = 0;
      }
      cur_count += c;
    }
  }
  if (cur_count > 0) {
    chunk.push_back(ptr[I]);
    slot.push_back(-1);
  }
  (void)cur_begin;
  row_task[I] = (int32_t)(task.size() - 1);
  heavy_slot.push_back((int32_t)nslot);
  md.nchunk = (int64_t)slot.size();
  md.nslot = nslot;
  md.nheavy = (int64_t)heavy_row.size();
  md.nrows = (int64_t)rows.size();
  md.ntask = (int64_t)task.size() - 1;
  md.max_task_per_row = max_tpr;
  md.mean_row = md.nrows ? (double)ptr[I] / (double)md.nrows : 0.0;
}

tt_status build_index_impl(int N, const int64_t *dims, int64_t m,
                           const int32_t *const *d_idx, const void *d_t,
                           tt_dtype vdt, hipStream_t s, tt_index *ix) {
  ix->N = N;
  ix->m = m;
  ix->vdt = vdt;
  ix->has_t = d_t != nullptr || m == 0;  // an empty value set is always available
  for (int n = 0; n < N; ++n) ix->dims[n] = dims[n];
  const size_t vsz = vdt == TT_F64 ? 8 : 4;
  {
    int dev = 0;
    TT_HIP(hipGetDevice(&dev));
    TT_HIP(hipDeviceGetAttribute(&ix->cu_count, hipDeviceAttributeMultiprocessorCount, dev));
  }

  // range check
  int *d_flag = nullptr;
  TT_HIP(hipMalloc(&d_flag, sizeof(int)));
  TT_HIP(hipMemsetAsync(d_flag, 0, sizeof(int), s));
  for (int n = 0; n < N; ++n)
    if (m > 0)
      k_range_check<<<grid_for(m, 256, 4096), 256, 0, s>>>(d_idx[n], m, dims[n], d_flag);
  int h_flag = 0;
  TT_HIP(hipMemcpyAsync(&h_flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  TT_HIP(hipStreamSynchronize(s));
  TT_HIP(hipFree(d_flag));
  if (h_flag) {
    set_error("tt_build_index: an index lies outside its dimension");
    return TT_ERR_INDEX_RANGE;
  }

  // sort temporaries
  const int64_t nblocks = std::max<int64_t>(1, (m + RS_TILE - 1) / RS_TILE);
  const int64_t hn = nblocks * RS_BINS;
  uint32_t *kA = nullptr, *kB = nullptr, *vA = nullptr, *vB = nullptr, *hist = nullptr,
           *offs = nullptr, *tmp = nullptr;
  const size_t mm = (size_t)std::max<int64_t>(m, 1);
  hipError_t he = hipSuccess;
  auto alloc_tmp = [&](uint32_t **p, size_t n) -> bool {
    he = hipMalloc((void **)p, n * sizeof(uint32_t));
    return he == hipSuccess;
  };
  bool ok = alloc_tmp(&kA, mm) && alloc_tmp(&kB, mm) && alloc_tmp(&vA, mm) &&
            alloc_tmp(&vB, mm) && alloc_tmp(&hist, hn) && alloc_tmp(&offs, hn) &&
            alloc_tmp(&tmp, scan_tmp_words(hn));
  auto free_tmp = [&]() {
    hipFree(kA); hipFree(kB); hipFree(vA); hipFree(vB);
    hipFree(hist); hipFree(offs); hipFree(tmp);
  };
  if (!ok) {
    free_tmp();
    set_error("tt_build_index: temporary allocation failed: %s", hipGetErrorString(he));
    return TT_ERR_OOM;
  }

  tt_status st = TT_OK;
  std::vector<int64_t> h_ptr;
  for (int n = 0; n < N && st == TT_OK; ++n) {
    ModeIndex &md = ix->mode[n];
    md.I = dims[n];
    uint32_t *kc = kA, *vc = vA;
    if (m > 0) {
      k_copy_u32<<<grid_for(m, 256), 256, 0, s>>>(d_idx[n], m, kA);
      he = radix_sort_positions(kA, kB, vA, vB, m, dims[n], hist, offs, tmp, s, &kc, &vc);
      if (he != hipSuccess) { st = hip_fail(he, "radix sort"); break; }
    }
    // persistent per-mode arrays
    if ((st = dev_alloc(ix, &md.d_perm, mm)) != TT_OK) break;
    if ((st = dev_alloc(ix, &md.d_key, mm)) != TT_OK) break;
    if ((st = dev_alloc(ix, &md.d_ptr, (size_t)dims[n] + 1)) != TT_OK) break;
    if (m > 0) {
      hipMemcpyAsync(md.d_perm, vc, m * 4, hipMemcpyDeviceToDevice, s);
      hipMemcpyAsync(md.d_key, kc, m * 4, hipMemcpyDeviceToDevice, s);
    }
    k_row_ptr<<<grid_for(dims[n] + 1, 256, 1 << 30), 256, 0, s>>>(kc, m, dims[n], md.d_ptr);
    for (int p = 0; p < N; ++p) {
      if (p == n) continue;
      if ((st = dev_alloc(ix, &md.d_oidx[p], mm)) != TT_OK) break;
      if (m > 0)
        k_gather_i32<<<grid_for(m, 256), 256, 0, s>>>(d_idx[p], vc, m, md.d_oidx[p]);
    }
    if (st != TT_OK) break;
    if (d_t) {
      void *q = nullptr;
      if ((he = hipMalloc(&q, mm * vsz)) != hipSuccess) { st = TT_ERR_OOM; break; }
      ix->owned.push_back(q);
      md.d_t = q;
      if (m > 0) {
        if (vdt == TT_F64)
          k_gather_val<double><<<grid_for(m, 256), 256, 0, s>>>((const double *)d_t, vc, m,
                                                                  (double *)q);
        else
          k_gather_val<float><<<grid_for(m, 256), 256, 0, s>>>((const float *)d_t, vc, m,
                                                                 (float *)q);
      }
    }
    // host partitions
    h_ptr.assign(dims[n] + 1, 0);
    if ((he = hipMemcpyAsync(h_ptr.data(), md.d_ptr, (dims[n] + 1) * 8,
                             hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (he = hipStreamSynchronize(s)) != hipSuccess) {
      st = hip_fail(he, "row pointers");
      break;
    }
    bool mono = h_ptr[0] == 0 && h_ptr[dims[n]] == m;
    for (int64_t i = 0; mono && i < dims[n]; ++i) mono = h_ptr[i] <= h_ptr[i + 1];
    if (!mono) {
      set_error("tt_build_index: internal error, row pointers of mode %d are inconsistent", n);
      st = TT_ERR_HIP;
      break;
    }
    md.h_ptr = h_ptr;
    if ((st = build_partitions(ix, n, s)) != TT_OK) break;
    ix->max_I = std::max(ix->max_I, md.I);
    ix->sum_I += md.I;
  }
  hipStreamSynchronize(s);
  free_tmp();
  if (st == TT_OK) {
    he = hipGetLastError();
    if (he != hipSuccess) st = hip_fail(he, "tt_build_index");
  }
  return st;
}

}  // namespace tt

namespace tt {

int gn_zmode(const tt_index *ix) {
  int b = 0;
  for (int n = 1; n < ix->N; ++n)
    if (ix->mode[n].I > ix->mode[b].I) b = n;
  return b;
}

// Composite sort key of the CCD++ layout: row * kCcdBuckets + the bucket of
// the nonzero's index in the bucketed mode (bucket b holds rows
// [b[b], b[b + 1])).
struct CcdBounds {
  int32_t b[kCcdBuckets + 1];
};
__global__ void k_ccd_composite(const int32_t *__restrict__ key, const int32_t *__restrict__ big,
                                int64_t m, CcdBounds bnd, uint32_t *__restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < m; i += stride) {
    const int32_t v = big[i];
    uint32_t b = 0;
#pragma unroll
    for (int q = 1; q < kCcdBuckets; ++q) b += v >= bnd.b[q] ? 1u : 0u;
    out[i] = (uint32_t)key[i] * kCcdBuckets + b;
  }
}

tt_status ccd_layout_get(tt_index *ix, int n, size_t vsz, hipStream_t s,
                         const CcdLayout **out) {
  *out = nullptr;
  ModeIndex &md = ix->mode[n];
  int big = -1;
  for (int p = 0; p < ix->N; ++p)
    if (p != n && (big < 0 || ix->mode[p].I > ix->mode[big].I)) big = p;
  const int mode = ix->tune.ccd_xcd;
  const int64_t IB = big < 0 ? 0 : ix->mode[big].I;
  const bool want = mode == 1 ? IB >= kCcdBuckets
                              : (mode < 0 && (double)IB * 4.0 * (double)vsz > 2.0 * (1 << 20));
  if (!want || ix->m <= 0 || (double)md.I * kCcdBuckets >= 2147483647.0) return TT_OK;
  if (md.ccd.built) {
    *out = &md.ccd;
    return TT_OK;
  }
  const int64_t m = ix->m;
  // bucket boundaries: row ranges of mode `big` with balanced nonzero counts
  CcdLayout L;
  L.big = big;
  {
    const std::vector<int64_t> &hp = ix->mode[big].h_ptr;
    L.bnd[0] = 0;
    int64_t r = 0;
    for (int b = 1; b < kCcdBuckets; ++b) {
      const int64_t target = m * b / kCcdBuckets;
      while (r < IB && hp[r] < target) ++r;
      L.bnd[b] = (int32_t)r;
    }
    L.bnd[kCcdBuckets] = (int32_t)IB;
  }
  CcdBounds cb;
  for (int b = 0; b <= kCcdBuckets; ++b) cb.b[b] = L.bnd[b];
  // stable sort of the sorted stream by (row, bucket)
  const int64_t nblocks = std::max<int64_t>(1, (m + RS_TILE - 1) / RS_TILE);
  const int64_t hn = nblocks * RS_BINS;
  const int64_t nseg = md.I * kCcdBuckets;
  uint32_t *kA = nullptr, *kB = nullptr, *vA = nullptr, *vB = nullptr, *hist = nullptr,
           *offs = nullptr, *tmp = nullptr;
  int64_t *segptr = nullptr;
  hipError_t he = hipSuccess;
  auto alloc_tmp = [&](void **p, size_t bytes) -> bool {
    he = hipMalloc(p, bytes);
    return he == hipSuccess;
  };
  auto free_tmp = [&]() {
    hipFree(kA); hipFree(kB); hipFree(vA); hipFree(vB);
    hipFree(hist); hipFree(offs); hipFree(tmp); hipFree(segptr);
  };
  if (!(alloc_tmp((void **)&kA, m * 4) && alloc_tmp((void **)&kB, m * 4) &&
        alloc_tmp((void **)&vA, m * 4) && alloc_tmp((void **)&vB, m * 4) &&
        alloc_tmp((void **)&hist, hn * 4) && alloc_tmp((void **)&offs, hn * 4) &&
        alloc_tmp((void **)&tmp, scan_tmp_words(hn) * 4) &&
        alloc_tmp((void **)&segptr, (nseg + 1) * 8))) {
    free_tmp();
    set_error("CCD++ layout: temporary allocation failed: %s", hipGetErrorString(he));
    return TT_ERR_OOM;
  }
  uint32_t *kc = nullptr, *vc = nullptr;
  k_ccd_composite<<<grid_for(m, 256), 256, 0, s>>>(md.d_key, md.d_oidx[big], m, cb, kA);
  he = radix_sort_positions(kA, kB, vA, vB, m, nseg, hist, offs, tmp, s, &kc, &vc);
  if (he == hipSuccess) {
    k_row_ptr<<<grid_for(nseg + 1, 256, 1 << 30), 256, 0, s>>>(kc, m, nseg, segptr);
    he = hipGetLastError();
  }
  std::vector<int64_t> hseg(nseg + 1);
  if (he == hipSuccess)
    he = hipMemcpyAsync(hseg.data(), segptr, (nseg + 1) * 8, hipMemcpyDeviceToHost, s);
  tt_status st = he == hipSuccess ? TT_OK : hip_fail(he, "CCD++ layout sort");
  // the streams in the new order (vc: new position -> sorted position)
  std::vector<void *> &P = md.part;
  if (st == TT_OK) st = dev_alloc_list(P, &L.d_key, m);
  if (st == TT_OK) st = dev_alloc_list(P, &L.d_inv, m);
  for (int p = 0; p < ix->N && st == TT_OK; ++p)
    if (p != n) st = dev_alloc_list(P, &L.d_oidx[p], m);
  if (st == TT_OK) {
    k_gather_i32<<<grid_for(m, 256), 256, 0, s>>>(md.d_key, vc, m, L.d_key);
    for (int p = 0; p < ix->N; ++p)
      if (p != n)
        k_gather_i32<<<grid_for(m, 256), 256, 0, s>>>(md.d_oidx[p], vc, m, L.d_oidx[p]);
    k_inv_perm<<<grid_for(m, 256), 256, 0, s>>>(reinterpret_cast<const int32_t *>(vc), m,
                                                 L.d_inv);
    he = hipGetLastError();
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) st = hip_fail(he, "CCD++ layout streams");
  }
  if (st != TT_OK) hipStreamSynchronize(s);
  free_tmp();
  if (st != TT_OK) return st;
  // tasks: every (row, bucket) segment cut into pieces of <= gram_piece;
  // bucket b's tasks go to workgroups b, b + kCcdBuckets, ... (4 each)
  const int64_t piece = ix->tune.gram_piece;
  std::vector<int64_t> task{0};
  std::vector<int32_t> row_task(md.I + 1, 0);
  std::vector<std::vector<int32_t>> per(kCcdBuckets);
  for (int64_t r = 0; r < md.I; ++r) {
    row_task[r] = (int32_t)(task.size() - 1);
    for (int b = 0; b < kCcdBuckets; ++b) {
      const int64_t lo = hseg[r * kCcdBuckets + b], hi = hseg[r * kCcdBuckets + b + 1];
      for (int64_t e = lo; e < hi; e += piece) {
        per[b].push_back((int32_t)(task.size() - 1));
        task.push_back(std::min(hi, e + piece));
      }
    }
  }
  row_task[md.I] = (int32_t)(task.size() - 1);
  size_t rounds = 0;
  for (auto &v : per) rounds = std::max(rounds, (v.size() + 3) / 4);
  std::vector<int32_t> sched(rounds * kCcdBuckets * 4, -1);
  for (int b = 0; b < kCcdBuckets; ++b)
    for (size_t j = 0; j < per[b].size(); ++j)
      sched[((j / 4) * kCcdBuckets + b) * 4 + (j % 4)] = per[b][j];
  L.ntask = (int64_t)task.size() - 1;
  L.nsched = (int64_t)rounds * kCcdBuckets;
  TT_ST(upload(P, &L.d_task, task, s));
  TT_ST(upload(P, &L.d_row_task, row_task, s));
  TT_ST(upload(P, &L.d_sched, sched, s));
  TT_HIP(hipStreamSynchronize(s));
  L.built = true;
  md.ccd = L;
  *out = &md.ccd;
  return TT_OK;
}

tt_status zmap_get(tt_index *ix, hipStream_t s, const int32_t **out) {
  if (ix->d_zmap == nullptr) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s != nullptr && hipStreamIsCapturing(s, &cs) == hipSuccess &&
        cs != hipStreamCaptureStatusNone) {
      set_error("the Gauss-Newton position map is built on first use: reserve it with "
                "tt_index_reserve(..., TT_RESERVE_GN) before capturing");
      return TT_ERR_INVALID_ARG;
    }
    const int64_t m = ix->m;
    const int zm = gn_zmode(ix);
    int32_t *map = nullptr;
    tt_status st = dev_alloc(ix, &map, (size_t)ix->N * (size_t)m);
    if (st != TT_OK) return st;
    if (m > 0) {
      // slot zm: inverse of the mode-zm permutation; slot n: mode-n sorted
      // position -> mode-zm sorted position
      int32_t *inv = map + (int64_t)zm * m;
      k_inv_perm<<<grid_for(m, 256), 256, 0, s>>>(ix->mode[zm].d_perm, m, inv);
      for (int n = 0; n < ix->N; ++n)
        if (n != zm)
          k_gather_i32<<<grid_for(m, 256), 256, 0, s>>>(
              inv, reinterpret_cast<const uint32_t *>(ix->mode[n].d_perm), m,
              map + (int64_t)n * m);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "position map");
    ix->d_zmap = map;
  }
  *out = ix->d_zmap;
  return TT_OK;
}

}  // namespace tt
