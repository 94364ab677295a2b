// Host dispatch of the streaming kernels: picks the lane-group width G from
// R and the storage dtype, decides whether the 16-byte vector path applies,
// and runs the heavy-row carry reduction after segmented operations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "pcg_loop.h"
#include "stream_impl.h"

namespace tt {

hipError_t launch_stream_f32(StreamOp op, const StreamDev &d, int64_t nchunk, int G,
                             int vm, int chunk, hipStream_t s);
hipError_t launch_stream_bf16(StreamOp op, const StreamDev &d, int64_t nchunk, int G,
                              int vm, int chunk, hipStream_t s);
hipError_t launch_stream_f64(StreamOp op, const StreamDev &d, int64_t nchunk, int G,
                             int vm, int chunk, hipStream_t s);

static int frag_elems(tt_dtype fdt) { return fdt == TT_F64 ? 2 : 4; }

int stream_group_width(tt_dtype fdt, int R) {
  const int V = frag_elems(fdt);
  int need = (R + V - 1) / V;
  int G = 2;
  while (G < need) G <<= 1;
  return G;
}

int stream_rp(tt_dtype fdt, int R) { return stream_group_width(fdt, R) * frag_elems(fdt); }

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Factor rows are read as whole fragments (V elements: 16 bytes, 8 for
// BF16) when the bases are fragment-aligned and the leading dimension is a
// multiple of V that holds R rounded up to V (the last fragment then stays
// inside the row even when R is not a multiple of V).
static bool frag_aligned(const void *p, tt_dtype fdt) {
  return ((uintptr_t)p & (fdt == TT_BF16 ? 7u : 15u)) == 0;
}

StreamDev stream_dev(StreamOp op, const StreamCall &c, int *vm_out) {
  const tt_index *ix = c.ix;
  const ModeIndex &md = ix->mode[c.mode];
  const int V = frag_elems(c.fdt);
  StreamDev d = {};
  d.chunk = md.d_chunk;
  d.chunk_slot = md.d_chunk_slot;
  d.key = md.d_key;
  // factor rows as fragments (va), dense blocks (row stride R) as
  // fragments too (vd)
  const int64_t Rv = (c.R + V - 1) / V * V;
  bool va = (c.ldA % V == 0) && c.ldA >= Rv;
  bool vd = va && (c.R % V == 0);
  int q = 0;
  for (int p = 0; p < ix->N; ++p) {
    if (p == c.mode) continue;
    d.oidx[q] = md.d_oidx[p];
    d.A_oth[q] = c.A[p];
    d.X_oth[q] = c.X[p];
    if (c.A[p] && !frag_aligned(c.A[p], c.fdt)) va = false;
    if (c.X[p] && !aligned16(c.X[p])) vd = false;
    ++q;
  }
  d.A_own = c.A[c.mode];
  d.X_own = c.X[c.mode];
  if (d.A_own && !frag_aligned(d.A_own, c.fdt)) va = false;
  if (d.X_own && !aligned16(d.X_own)) vd = false;
  if (op != OP_TTTP && !aligned16(c.out)) vd = false;
  const int vm = !va ? 0 : (vd ? 2 : 1);
  d.s = c.s;
  d.s_perm = c.s_perm;
  d.w_const = c.w_const;
  d.R = c.R;
  d.ldA = c.ldA;
  d.epi = c.epi;
  d.loss = c.loss;
  d.out = c.out;
  d.out_perm = c.out_perm;
  d.accumulate = c.accumulate;
  d.sum_parts = c.sum_parts;
  d.carry = c.carry;
  d.skip = c.skip;
  d.zout = (op == OP_GN || op == OP_GRAD) ? c.zout : nullptr;
  *vm_out = vm;
  return d;
}

hipError_t launch_stream(StreamOp op, const StreamCall &c, hipStream_t s) {
  const tt_index *ix = c.ix;
  const ModeIndex &md = ix->mode[c.mode];
  const int V = frag_elems(c.fdt);
  const int G = stream_group_width(c.fdt, c.R);
  int vm = 0;
  const StreamDev d = stream_dev(op, c, &vm);
  hipError_t e;
  {
    // algorithmic work of this launch (per-nonzero byte model: index
    // streams, values, factor-row gathers at storage precision)
    const double m = (double)ix->m, R = c.R, N = ix->N;
    const double b = c.fdt == TT_F64 ? 8 : (c.fdt == TT_F32 ? 4 : 2);
    const double v = c.fdt == TT_F64 ? 8 : 4, xs = v, I = (double)md.I;
    double bytes = 0, flops = 0;
    const char *name = "tttp";
    if (op == OP_TTTP) {
      // the pass runs in this mode's sorted order: the own factor row is
      // read once per nonzero row (segment), the others once per nonzero
      int given = 0;
      for (int p = 0; p < ix->N; ++p) given += c.A[p] != nullptr;
      const bool own = c.A[c.mode] != nullptr;
      bytes = m * (4 * N + (c.s ? v : 0) + (c.out ? v : 0) + (given - own) * R * b) +
              (own ? (double)md.nrows * R * b : 0.0);
      flops = m * R * given;
    } else if (op == OP_MTTKRP) {
      name = "mttkrp";
      bytes = m * (4 * (N - 1) + (c.s ? v : 0) + (c.s_perm ? 4 : 0) + (N - 1) * R * b) +
              I * R * xs * (c.accumulate ? 2 : 1);
      flops = m * R * N;
    } else if (op == OP_GRAD) {
      name = "gradient";
      bytes = m * (4 * (N - 1) + v + (c.zout ? v : 0) + (N - 1) * R * b) +
              I * R * (b + 2 * xs);
      flops = m * R * (N + 3);
    } else if (op == OP_NEWTON) {
      name = "newton_terms";
      bytes = m * (4 * (N - 1) + v + (c.s_perm ? 4 : 0) + (N - 1) * R * (b + xs)) +
              I * R * xs * 2;
      flops = m * R * (2 * (N - 1) + 2);
    } else {
      name = "gn_matvec";
      bytes = m * (4 * (N - 1) + (c.s ? v : 0) + (c.s_perm ? 4 : 0) + (c.zout ? v : 0) +
                   (N - 1) * R * (b + xs)) +
              I * R * (b + 3 * xs);
      flops = m * R * 10;
    }
    if (c.prof_name) name = c.prof_name;
    ProfScope ps(name, s, bytes, flops);
    if (c.fdt == TT_F32)
      e = launch_stream_f32(op, d, md.nchunk, G, vm, ix->tune.chunk, s);
    else if (c.fdt == TT_BF16)
      e = launch_stream_bf16(op, d, md.nchunk, G, vm, ix->tune.chunk, s);
    else
      e = launch_stream_f64(op, d, md.nchunk, G, vm, ix->tune.chunk, s);
  }
  if (e != hipSuccess) return e;
  if (op != OP_TTTP && md.nheavy > 0) {
    const int RP = G * V;
    double *partial = c.carry_partial ? c.carry_partial
                                      : c.carry + (int64_t)ix->max_nslot * 64;  // after the slots
    ProfScope ps("heavy_fixup", s,
                 (double)md.nslot * RP * 8 + (double)md.nseg * RP * 16 +
                     (double)md.nheavy * c.R * 4,
                 (double)md.nslot * RP);
    k_carry_partial<<<(unsigned)md.nseg, 256, 0, s>>>(md.d_seg, c.carry, RP, partial, c.skip);
    if (c.fdt == TT_F64)
      k_heavy_fixup<double><<<(unsigned)md.nheavy, 256, 0, s>>>(
          md.d_heavy_row, md.d_heavy_seg, partial, RP, c.R, c.out, c.accumulate, c.skip);
    else
      k_heavy_fixup<float><<<(unsigned)md.nheavy, 256, 0, s>>>(
          md.d_heavy_row, md.d_heavy_seg, partial, RP, c.R, c.out, c.accumulate, c.skip);
    e = hipGetLastError();
  }
  return e;
}

// Carry slots and heavy-row partials of the three passes side by side (the
// two MTTKRP passes run in the same phase).
int64_t pcg_loop_carry_doubles(const tt_index *ix) {
  int64_t n = 0;
  for (int d = 0; d < ix->N; ++d) n += (ix->mode[d].nslot + ix->mode[d].nseg) * 64;
  return std::max<int64_t>(n, 64);
}

int pcg_loop_bar_words() { return kBarWords; }

// A barrier counter reaches (barriers so far) x (its group size or group
// count, at most kPcgMaxGrid / kBarGroup): at most 1 + 11 barriers per
// iteration, kept below 2^31.
int64_t pcg_loop_max_iters(const tt_index *ix, int wgs_per_cu) {
  (void)ix;
  (void)wgs_per_cu;
  return ((int64_t)1 << 31) / (12 * (kPcgMaxGrid / kBarGroup)) - 1;
}

// Load mode of the loop: the most general one any of the three passes
// needs (the loads differ between load modes, the arithmetic does not).
static int pcg_loop_vm(const PcgLoopCall &c, StreamDev *dev) {
  int vm = 2;
  for (int i = 0; i < 3; ++i) {
    int v = 0;
    const StreamDev d = stream_dev(i == 0 ? OP_GN : OP_MTTKRP, c.pass[i], &v);
    if (dev) dev[i] = d;
    vm = std::min(vm, v);
  }
  return vm;
}

static int pcg_loop_occupancy(const PcgLoopCall &c, int vm) {
  const tt_dtype fdt = c.pass[0].fdt;
  const int G = stream_group_width(fdt, c.pass[0].R);
  if (fdt == TT_F32) return pcg_loop_occupancy_f32(G, vm);
  if (fdt == TT_BF16) return pcg_loop_occupancy_bf16(G, vm);
  return pcg_loop_occupancy_f64(G, vm);
}

bool pcg_loop_fits(const PcgLoopCall &c) {
  const tt_index *ix = c.pass[0].ix;
  if (ix->N != 3 || c.pass[0].R > kPcgMaxRank) return false;
  const int occ = pcg_loop_occupancy(c, pcg_loop_vm(c, nullptr));
  if (occ < 1) return false;
  const int64_t grid = (int64_t)std::min(occ, 2) * ix->cu_count;
  const int64_t gn = ix->mode[c.pass[0].mode].nchunk;
  const int64_t mt = ix->mode[c.pass[1].mode].nchunk + ix->mode[c.pass[2].mode].nchunk;
  return gn <= grid && mt <= grid;
}

hipError_t launch_pcg_loop(const PcgLoopCall &c, hipStream_t s) {
  const tt_index *ix = c.pass[0].ix;
  const tt_dtype fdt = c.pass[0].fdt;
  const int R = c.pass[0].R;
  if (ix->N != 3 || R > kPcgMaxRank || c.wgs_per_cu < 1) return hipErrorInvalidValue;
  PcgLoopDev a = {};
  const int vm = pcg_loop_vm(c, a.pass);
  double *cb = c.carry;
  for (int i = 0; i < 3; ++i) {
    a.pass[i].skip = nullptr;
    const ModeIndex &md = ix->mode[c.pass[i].mode];
    a.nchunk[i] = md.nchunk;
    a.pass[i].carry = cb;
    cb += md.nslot * 64;
    a.partial[i] = cb;
    cb += md.nseg * 64;
    a.seg[i] = md.d_seg;
    a.hrow[i] = md.d_heavy_row;
    a.hseg[i] = md.d_heavy_seg;
    a.nseg[i] = md.nseg;
    a.nheavy[i] = md.nheavy;
  }
  a.srp = stream_rp(fdt, R);
  a.rowoff[0] = 0;
  for (int d = 0; d < 3; ++d) {
    a.L[d] = c.L[d];
    a.rowoff[d + 1] = a.rowoff[d] + ix->mode[d].I;
  }
  a.x = c.x;
  a.r = c.r;
  a.z = c.z;
  a.p = c.p;
  a.q = c.q;
  a.ntot = a.rowoff[3] * R;
  a.R = R;
  a.lambda2 = c.lambda2;
  a.parts = c.parts;
  a.np = dot_parts_needed(a.ntot);
  a.sc = c.sc;
  a.tol = c.tol;
  a.kmax = c.kmax;
  a.bar = c.bar;
  if (c.kmax > pcg_loop_max_iters(ix, c.wgs_per_cu)) return hipErrorInvalidValue;
  hipError_t e = launch_fill(c.bar, kBarWords, TT_F32, 0.0, s);  // zero words
  if (e != hipSuccess) return e;
  const int G = stream_group_width(fdt, R);
  ProfScope ps("pcg_loop", s, 0.0, 0.0);
  if (fdt == TT_F32) return launch_pcg_loop_f32(a, G, vm, c.wgs_per_cu, ix->cu_count, s);
  if (fdt == TT_BF16) return launch_pcg_loop_bf16(a, G, vm, c.wgs_per_cu, ix->cu_count, s);
  return launch_pcg_loop_f64(a, G, vm, c.wgs_per_cu, ix->cu_count, s);
}

}  // namespace tt
