// Persistent conjugate-gradient loop instantiated for f32 factor storage
// (see pcg_loop_impl.h); ranks up to 16.
#include "pcg_loop_impl.h"

namespace tt {

hipError_t launch_pcg_loop_f32(const PcgLoopDev &a, int G, int vm, int wgs_per_cu,
                               int cu_count, hipStream_t s) {
  switch (G) {
    case 2: return launch_pcg_loop_g<TrF32, 2>(a, vm, wgs_per_cu, cu_count, s);
    case 4: return launch_pcg_loop_g<TrF32, 4>(a, vm, wgs_per_cu, cu_count, s);
    default: return hipErrorInvalidValue;
  }
}

int pcg_loop_occupancy_f32(int G, int vm) {
  switch (G) {
    case 2: return pcg_loop_occupancy_g<TrF32, 2>(vm);
    case 4: return pcg_loop_occupancy_g<TrF32, 4>(vm);
    default: return -1;
  }
}

}  // namespace tt
