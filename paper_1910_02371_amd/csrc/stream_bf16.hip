// Streaming kernels instantiated for bf16 factor storage (see stream_impl.h).
#include "stream_impl.h"

namespace tt {

hipError_t launch_stream_bf16(StreamOp op, const StreamDev &d, int64_t nchunk, int G,
                             int vm, int chunk, hipStream_t s) {
  switch (G) {
    case 2: return launch_stream_g<TrBF16, 2>(op, d, nchunk, vm, chunk, s);
    case 4: return launch_stream_g<TrBF16, 4>(op, d, nchunk, vm, chunk, s);
    case 8: return launch_stream_g<TrBF16, 8>(op, d, nchunk, vm, chunk, s);
    case 16: return launch_stream_g<TrBF16, 16>(op, d, nchunk, vm, chunk, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tt
