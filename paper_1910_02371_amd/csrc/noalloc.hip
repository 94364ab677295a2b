// Allocation-free MTTKRP: the same kernels as `mttkrp`, with the FP64 carry
// slots of rows longer than one work chunk (and their first-level partials)
// in a fixed device array of this translation unit instead of the index's
// workspace, so the call never allocates device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace tt {

// 32 MiB per device, held from the first call on that device until the
// process ends.
constexpr int64_t kScratchDoubles = (32ll << 20) / 8;

static __device__ __align__(256) double scratch[kScratchDoubles];

// Device address of `scratch` on each device (the host-side name is only a
// stand-in, never a device address).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kMaxDevices] = {};

static tt_status scratch_on_current_device(double **out) {
  int dev = -1;
  TT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d outside the %d devices the scratch table covers", dev, kMaxDevices);
    return TT_ERR_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[dev] == nullptr) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch symbol address");
    g_scratch_dev[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_dev[dev];
  return TT_OK;
}

}  // namespace tt

using namespace tt;

extern "C" {

tt_status mttkrp_noalloc(const tt_index *cix, const void *d_s, int s_order,
                         const void *const *d_A, int R, int64_t ldA, tt_dtype fdt, int mode,
                         void *d_out, int accumulate, hipStream_t stream) {
  tt::set_error("");
  TT_CHECK(cix != nullptr, "index is NULL");
  TT_CHECK(mode >= 0 && mode < cix->N, "bad mode %d", mode);
  TT_CHECK(R >= 1 && R <= TT_MAX_RANK, "rank %d outside [1, %d]", R, TT_MAX_RANK);
  TT_CHECK(fdt == TT_F64 || fdt == TT_F32 || fdt == TT_BF16, "bad factor dtype %d", (int)fdt);
  const ModeIndex &md = cix->mode[mode];
  const int64_t need = (md.nslot + md.nseg) * (int64_t)stream_rp(fdt, R);
  if (need > kScratchDoubles) {
    set_error("mttkrp_noalloc: mode %d needs %lld bytes of carry scratch (%lld pieces of rows "
              "longer than one work chunk at rank %d); the fixed scratch holds %lld bytes",
              mode, (long long)(need * 8), (long long)md.nslot, R,
              (long long)(kScratchDoubles * 8));
    return TT_ERR_UNSUPPORTED;
  }
  double *carry = nullptr;
  tt_status st = scratch_on_current_device(&carry);
  if (st != TT_OK) return st;
  return mttkrp_checked(const_cast<tt_index *>(cix), d_s, s_order, d_A, R, ldA, fdt, mode, d_out,
                        accumulate, stream, carry);
}

}  // extern "C"
