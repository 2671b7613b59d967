// Precision conversion between the FP64 boundary state and the FP32 copy the
// FP32-bulk propagator advances (same tiled layout, elementwise), and the
// plain FP64 copy a sweep with an odd number of stages ends with (a kernel,
// so that a captured sweep holds kernel nodes only).

#include <hip/hip_runtime.h>

#include "wadg_internal.h"

namespace wadg {
namespace {

template <typename A, typename B>
__global__ __launch_bounds__(256) void convert_kernel(const A* __restrict__ in, B* __restrict__ out,
                                                     size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = static_cast<B>(in[i]);
}

template <typename A, typename B>
int launch(const A* in, B* out, size_t n, void* stream) {
  if (n == 0) return 0;
  const size_t want = (n + 255) / 256;
  const unsigned blocks = (unsigned)(want < 16384 ? want : 16384);
  hipLaunchKernelGGL((convert_kernel<A, B>), dim3(blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), in, out, n);
  return (int)hipGetLastError();
}

}  // namespace

int launch_to_fp32(const double* in, float* out, size_t n, void* stream) {
  return launch(in, out, n, stream);
}
int launch_to_fp64(const float* in, double* out, size_t n, void* stream) {
  return launch(in, out, n, stream);
}
int launch_copy(const double* in, double* out, size_t n, void* stream) {
  return launch(in, out, n, stream);
}

}  // namespace wadg
