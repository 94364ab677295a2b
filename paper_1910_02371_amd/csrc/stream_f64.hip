// Streaming kernels instantiated for f64 factor storage (see stream_impl.h).
#include "stream_impl.h"

namespace tt {

hipError_t launch_stream_f64(StreamOp op, const StreamDev &d, int64_t nchunk, int G,
                             int vm, int chunk, hipStream_t s) {
  switch (G) {
    case 2: return launch_stream_g<TrF64, 2>(op, d, nchunk, vm, chunk, s);
    case 4: return launch_stream_g<TrF64, 4>(op, d, nchunk, vm, chunk, s);
    case 8: return launch_stream_g<TrF64, 8>(op, d, nchunk, vm, chunk, s);
    case 16: return launch_stream_g<TrF64, 16>(op, d, nchunk, vm, chunk, s);
    case 32: return launch_stream_g<TrF64, 32>(op, d, nchunk, vm, chunk, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tt
