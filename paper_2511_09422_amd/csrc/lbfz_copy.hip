// lbfz_copy.hip -- the streaming-copy reference of the step: a device copy
// that reads and writes every byte once, as one time step reads and writes
// the whole solver state once.  Its bandwidth is what this memory system
// gives a pure streaming kernel, the practical ceiling of the step.
//
// Form (chosen by timing 1007 MB copies on MI355X): 16-byte loads and stores,
// one in flight per lane, a grid-stride loop over 4 blocks of 256 threads
// per compute unit -- 5.83 TB/s, against 5.34 TB/s for the runtime's
// device-to-device copy and 5.0-5.7 TB/s for more blocks, more loads in
// flight per lane, non-temporal stores or one contiguous span per block.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbfz.h"

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const f4* __restrict__ src,
                                                     f4* __restrict__ dst, long n4) {
  const long stride = (long)gridDim.x * 256;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" int lbfz_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
    return LBFZ_EINVAL;
  if (bytes == 0) return LBFZ_OK;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return LBFZ_EHIP;
  const long n4 = (long)(bytes / 16);
  const long want = 4L * (cus > 0 ? cus : 256);
  const int grid = (int)(want < (n4 + 255) / 256 ? want : (n4 + 255) / 256);
  hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, (hipStream_t)stream,
                     static_cast<const f4*>(src), static_cast<f4*>(dst), n4);
  return hipGetLastError() == hipSuccess ? LBFZ_OK : LBFZ_EHIP;
}
