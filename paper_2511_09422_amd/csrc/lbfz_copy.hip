// lbfz_copy.hip -- the streaming references of the step: a device copy that
// reads and writes every byte once, as one time step reads and writes the
// whole solver state once, and the step's own plane pattern without its
// arithmetic.  Their bandwidths are what this memory system gives a pure
// streaming kernel and the step's access pattern, its practical ceilings.
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

// The memory pattern of the 2D FP32 step without its arithmetic: each node
// reads the 30 planes of a node update (24 populations, 6 previous-level
// fields) at its own position and writes them one row down, in place or one
// row up (y periodic) in turn, as the step's pushed populations land on the
// rows of their targets (the step's planes are shifted along x, so a push
// lands on the target row at the writer's own column).  All loads of a lane
// are issued before its first store; loads and stores carry the
// non-temporal hint.
constexpr int kPatternPlanes = 30;
__global__ __launch_bounds__(256) void k_stream_planes(const float* __restrict__ src,
                                                       float* __restrict__ dst, int nx, int ny,
                                                       long ps) {
  const long n = (long)blockIdx.x * 256 + threadIdx.x;
  if (n >= (long)nx * ny) return;
  const int y = (int)(n / nx), x = (int)(n - (long)y * nx);
  float v[kPatternPlanes];
#pragma unroll
  for (int k = 0; k < kPatternPlanes; ++k) v[k] = __builtin_nontemporal_load(src + k * ps + n);
  const long rows[3] = {(long)(y == 0 ? ny - 1 : y - 1) * nx + x, (long)y * nx + x,
                        (long)(y == ny - 1 ? 0 : y + 1) * nx + x};
#pragma unroll
  for (int k = 0; k < kPatternPlanes; ++k)
    __builtin_nontemporal_store(v[k], dst + k * ps + rows[k % 3]);
}

// The memory pattern of one launch of the 3D FP32 step without its
// arithmetic: each node reads nread planes at its own position and writes
// nwrite planes, plane k < 38 displaced by D3Q19 direction k mod 19 (the
// step pushes its 38 moving and rest populations to the nodes they stream
// to; x, y, z periodic here), the others in place.  Default cache policy,
// as the 3D step uses.  The closure launch moves 22 planes in (f, h, l and
// the previous velocity) and 5 out; the collision launch about 50 in and 42
// out.
constexpr int CX19[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
constexpr int CY19[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
constexpr int CZ19[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
// NR, NW compile-time: every load of a lane is issued before its first store,
// with no branch between them.  The planes read but not written are summed
// into a store guarded by `never` (NaN from the host, so it is never taken)
// that keeps their loads in the kernel.
template <int NR, int NW>
__global__ __launch_bounds__(256) void k_stream_planes3d(const float* __restrict__ src,
                                                         float* __restrict__ dst, int nx, int ny,
                                                         int nz, long ps, float never) {
  static_assert(NW <= NR, "each written plane is a read one");
  const long N = (long)nx * ny * nz;
  const long n = (long)blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  const int x = (int)(n % nx);
  const long r = n / nx;
  const int y = (int)(r % ny), z = (int)(r / ny);
  float v[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) v[k] = src[k * ps + n];
  const long xs[3] = {x == 0 ? nx - 1 : x - 1, x, x == nx - 1 ? 0 : x + 1};
  const long ys[3] = {y == 0 ? ny - 1 : y - 1, y, y == ny - 1 ? 0 : y + 1};
  const long zs[3] = {z == 0 ? nz - 1 : z - 1, z, z == nz - 1 ? 0 : z + 1};
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    long o = n;
    if (k < 38) {
      const int d = k % 19;
      o = (zs[CZ19[d] + 1] * ny + ys[CY19[d] + 1]) * nx + xs[CX19[d] + 1];
    }
    dst[k * ps + o] = v[k];
  }
  float rest = 0.0f;
#pragma unroll
  for (int k = NW; k < NR; ++k) rest += v[k];
  if (rest == never) dst[n] = rest;
}

}  // namespace

extern "C" int lbfz_stream_planes3d(float* dst, const float* src, int nx, int ny, int nz,
                                    long plane_stride, int nread, int nwrite, void* stream) {
  const bool closure = nread == 22 && nwrite == 5, collision = nread == 50 && nwrite == 42;
  if (!dst || !src || nx < 1 || ny < 1 || nz < 1 || !(closure || collision) ||
      plane_stride < (long)nx * ny * nz)
    return LBFZ_EINVAL;
  const long n = (long)nx * ny * nz;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (closure)
    hipLaunchKernelGGL((k_stream_planes3d<22, 5>), grid, dim3(256), 0, (hipStream_t)stream, src,
                       dst, nx, ny, nz, plane_stride, __builtin_nanf(""));
  else
    hipLaunchKernelGGL((k_stream_planes3d<50, 42>), grid, dim3(256), 0, (hipStream_t)stream, src,
                       dst, nx, ny, nz, plane_stride, __builtin_nanf(""));
  return hipGetLastError() == hipSuccess ? LBFZ_OK : LBFZ_EHIP;
}

extern "C" int lbfz_stream_planes(float* dst, const float* src, int nx, int ny, long plane_stride,
                                  void* stream) {
  if (!dst || !src || nx < 1 || ny < 1 || plane_stride < (long)nx * ny) return LBFZ_EINVAL;
  const long n = (long)nx * ny;
  hipLaunchKernelGGL(k_stream_planes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, src, dst, nx, ny, plane_stride);
  return hipGetLastError() == hipSuccess ? LBFZ_OK : LBFZ_EHIP;
}

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
