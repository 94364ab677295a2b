// Streaming kernels instantiated for f32 factor storage (see stream_impl.h).
#include "stream_impl.h"

namespace tt {

hipError_t launch_stream_f32(StreamOp op, const StreamDev &d, int64_t nchunk, int G,
                             int vm, int chunk, hipStream_t s) {
  switch (G) {
    case 2: return launch_stream_g<TrF32, 2>(op, d, nchunk, vm, chunk, s);
    case 4: return launch_stream_g<TrF32, 4>(op, d, nchunk, vm, chunk, s);
    case 8: return launch_stream_g<TrF32, 8>(op, d, nchunk, vm, chunk, s);
    case 16: return launch_stream_g<TrF32, 16>(op, d, nchunk, vm, chunk, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tt
