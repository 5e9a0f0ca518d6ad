// FP64 -> FP32 conversion of the adjoint's weights in the FP32 mode.
//
// The FP32 products round each FP64 weight to FP32 as they load it; doing
// that once per call in a streaming pass (round to nearest, as the loaders
// do) gives the products the same values at half the bytes, and lets them
// run their FP32-operand instantiations.
#include "qmk_internal.h"

namespace qmk {
namespace {

__global__ __launch_bounds__(256) void f64_to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst,
                                                         int64_t n, int vec) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * 4;
  if (vec && i + 4 <= n) {
    const double4 v = *reinterpret_cast<const double4*>(src + i);
    *reinterpret_cast<float4*>(dst + i) =
        make_float4(static_cast<float>(v.x), static_cast<float>(v.y), static_cast<float>(v.z), static_cast<float>(v.w));
  } else {
    for (int64_t k = i; k < min(i + 4, n); ++k) dst[k] = static_cast<float>(src[k]);
  }
}

}  // namespace

hipError_t launch_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 1023) / 1024;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  // vector loads and stores need 32-byte / 16-byte aligned pointers
  const int vec = reinterpret_cast<uintptr_t>(src) % 32 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, src, dst, n, vec);
  return hipGetLastError();
}

}  // namespace qmk
