// Fused Gram + solve kernels of Solve Factor instantiated for bf16 factor
// storage (see solve_impl.h).
#include "solve_impl.h"

namespace tt {

hipError_t launch_fused_rows_bf16(int RP, const GramDev &d, const SolveDev &sd,
                                 const GramLists &gl, hipStream_t s) {
  return launch_fused_rows<TrBF16>(RP, d, sd, gl, s);
}

}  // namespace tt
