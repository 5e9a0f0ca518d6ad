// Conversions of the adjoint's weights W: FP64 -> FP32 in the FP32 mode, and
// the split into bf16 hi / lo planes in the BF16x3 mode.
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

// W[p][c][n] -> hi, lo planes [Pp][5][Nw]: hi = bf16(x), lo = bf16(x - hi) of
// the FP32-rounded weight x (round to nearest even); zeros beyond P and N.
// One thread per eight consecutive n of one (p, c) row: idx < Pp * 5 * Nw / 8,
// which the launchers keep below 2^32 (32-bit index arithmetic).
template <typename T>
__device__ __forceinline__ void split_w8(const T* __restrict__ w, int64_t P, int64_t N, int64_t Nw, int vec,
                                         const int32_t* __restrict__ perm, __bf16* __restrict__ hi,
                                         __bf16* __restrict__ lo, uint32_t idx) {
  typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
  const uint32_t cpr = static_cast<uint32_t>(Nw / 8);
  const uint32_t row32 = idx / cpr;
  const int64_t row = row32, n0 = static_cast<int64_t>(idx - row32 * cpr) * 8;
  // source row: point perm[p] (or p), same component
  const int64_t p = row32 / 5u;
  const int64_t srow = (perm && p < P) ? static_cast<int64_t>(perm[p]) * 5 + (row - p * 5) : row;
  float x[8];
  if (row < P * 5 && vec && n0 + 8 <= N) {
    const T* src = w + srow * N + n0;
    if constexpr (sizeof(T) == 8) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 v = *reinterpret_cast<const double2*>(src + 2 * q);
        x[2 * q] = static_cast<float>(v.x);
        x[2 * q + 1] = static_cast<float>(v.y);
      }
    } else {
      const float4 a = *reinterpret_cast<const float4*>(src);
      const float4 b = *reinterpret_cast<const float4*>(src + 4);
      x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
      x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      x[e] = (row < P * 5 && n0 + e < N) ? static_cast<float>(w[srow * N + n0 + e]) : 0.0f;
  }
  bf16x8 h, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    // hi is the bf16 rounding of the FP32 value: without this barrier the
    // two conversions of an FP64 weight would be merged into one rounding
    asm volatile("" : "+v"(x[e]));
    const __bf16 hh = static_cast<__bf16>(x[e]);
    h[e] = hh;
    l[e] = static_cast<__bf16>(x[e] - static_cast<float>(hh));
  }
  *reinterpret_cast<bf16x8*>(hi + row * Nw + n0) = h;
  *reinterpret_cast<bf16x8*>(lo + row * Nw + n0) = l;
}

template <typename T>
__global__ __launch_bounds__(256) void split_w_kernel(const T* __restrict__ w, int64_t P, int64_t N, int64_t Pp,
                                                      int64_t Nw, int vec, const int32_t* __restrict__ perm,
                                                      __bf16* __restrict__ hi, __bf16* __restrict__ lo) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= static_cast<uint64_t>(Pp * 5 * (Nw / 8))) return;
  split_w8(w, P, N, Nw, vec, perm, hi, lo, idx);
}

template <typename T>
__global__ __launch_bounds__(256) void split_w_batch_kernel(const SplitJob* __restrict__ jobs,
                                                            const int64_t* __restrict__ prefix, int n_jobs,
                                                            int64_t total) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int jb = find_job(prefix, n_jobs, e);
  const SplitJob& j = jobs[jb];
  split_w8(static_cast<const T*>(j.w), j.P, j.N, j.Nw, j.vec, static_cast<const int32_t*>(nullptr),
           static_cast<__bf16*>(j.hi), static_cast<__bf16*>(j.lo), static_cast<uint32_t>(e - prefix[jb]));
}

}  // namespace

hipError_t launch_split_w(const void* w, int w_is_f32, int64_t P, int64_t N, int64_t Pp, int64_t Nw,
                          const int32_t* perm, void* hi, void* lo, hipStream_t s) {
  if (Pp <= 0 || Nw <= 0) return hipSuccess;
  if (Nw % 8 != 0 || Pp < P || Nw < N) return hipErrorInvalidValue;
  const int64_t n = Pp * 5 * (Nw / 8);
  if (n > 0xffffffffLL - 255) return hipErrorInvalidValue;
  const int64_t blocks = (n + 255) / 256;
  const size_t esz = w_is_f32 ? 4 : 8;
  // vector loads need every group of eight weights to start 16-byte aligned
  const int vec = reinterpret_cast<uintptr_t>(w) % 16 == 0 && (N * esz) % 16 == 0;
  if (w_is_f32)
    hipLaunchKernelGGL(split_w_kernel<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<const float*>(w), P, N, Pp, Nw, vec, perm, static_cast<__bf16*>(hi),
                       static_cast<__bf16*>(lo));
  else
    hipLaunchKernelGGL(split_w_kernel<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<const double*>(w), P, N, Pp, Nw, vec, perm, static_cast<__bf16*>(hi),
                       static_cast<__bf16*>(lo));
  return hipGetLastError();
}

hipError_t launch_split_w_batch(const SplitJob* jobs, const int64_t* prefix, int n_jobs, int64_t total,
                                int w_is_f32, hipStream_t s) {
  if (total <= 0 || n_jobs <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (w_is_f32)
    hipLaunchKernelGGL(split_w_batch_kernel<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, jobs,
                       prefix, n_jobs, total);
  else
    hipLaunchKernelGGL(split_w_batch_kernel<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, jobs,
                       prefix, n_jobs, total);
  return hipGetLastError();
}

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
