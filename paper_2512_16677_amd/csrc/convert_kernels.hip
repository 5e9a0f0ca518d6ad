// Conversions of the adjoint's weights W: FP64 -> FP32 in the FP32 mode, and
// the split into bf16 hi / lo planes in the BF16x3 mode.
//
// The FP32 products round each FP64 weight to FP32 as they load it; doing
// that once per call in a streaming pass (round to nearest, as the loaders
// do) gives the products the same values at half the bytes, and lets them
// run their FP32-operand instantiations.  The copy pads its rows to a
// multiple of four weights, so that both products can load it in 16-byte
// pieces; the same padded copy (without conversion) serves weights whose row
// length does not allow that.
#include "qmk_internal.h"

namespace qmk {
namespace {

// rows of n source values -> rows of ldd destination values (ldd a multiple
// of 4, zeros from n on; FP64 -> FP32 rounds to nearest); output quad q of
// the copy (four values of one row)
template <typename TS, typename TD>
__device__ __forceinline__ void pad_quad(const TS* __restrict__ src, TD* __restrict__ dst, int64_t n, int64_t ldd,
                                         int64_t q) {
  const int64_t qpr = ldd / 4, row = q / qpr, c0 = (q - row * qpr) * 4;
  const TS* sr = src + row * n;
  TD v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = c0 + e < n ? static_cast<TD>(sr[c0 + e]) : TD(0);
  TD* dr = dst + row * ldd + c0;
  if constexpr (sizeof(TD) == 4) {
    *reinterpret_cast<float4*>(dr) = make_float4(v[0], v[1], v[2], v[3]);
  } else {
    reinterpret_cast<double2*>(dr)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2*>(dr)[1] = make_double2(v[2], v[3]);
  }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void pad_rows_kernel(const TS* __restrict__ src, TD* __restrict__ dst,
                                                       int64_t rows, int64_t n, int64_t ldd) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= rows * (ldd / 4)) return;
  pad_quad(src, dst, n, ldd, q);
}

template <typename T>
__global__ __launch_bounds__(256) void pad_rows_batch_kernel(const PadJob* __restrict__ jobs,
                                                             const int64_t* __restrict__ prefix, int n_jobs,
                                                             int64_t total) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int jb = find_job(prefix, n_jobs, e);
  const PadJob& j = jobs[jb];
  pad_quad(static_cast<const T*>(j.src), static_cast<T*>(j.dst), j.n, j.ldd, e - prefix[jb]);
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

hipError_t launch_pad_rows_batch(const PadJob* jobs, const int64_t* prefix, int n_jobs, int64_t total, int f32,
                                 hipStream_t s) {
  if (total <= 0 || n_jobs <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (f32)
    hipLaunchKernelGGL(pad_rows_batch_kernel<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, jobs,
                       prefix, n_jobs, total);
  else
    hipLaunchKernelGGL(pad_rows_batch_kernel<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, jobs,
                       prefix, n_jobs, total);
  return hipGetLastError();
}

hipError_t launch_pad_rows(const void* src, int src_f32, void* dst, int dst_f32, int64_t rows, int64_t n,
                           int64_t ldd, hipStream_t s) {
  if (rows <= 0 || n <= 0) return hipSuccess;
  // the vector stores need 16-byte aligned rows; FP32 -> FP64 is not offered
  if (ldd < n || ldd % 4 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0 || (src_f32 && !dst_f32))
    return hipErrorInvalidValue;
  const int64_t blocks = (rows * (ldd / 4) + 255) / 256;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(blocks));
  if (src_f32)
    hipLaunchKernelGGL((pad_rows_kernel<float, float>), grid, dim3(256), 0, s, static_cast<const float*>(src),
                       static_cast<float*>(dst), rows, n, ldd);
  else if (dst_f32)
    hipLaunchKernelGGL((pad_rows_kernel<double, float>), grid, dim3(256), 0, s, static_cast<const double*>(src),
                       static_cast<float*>(dst), rows, n, ldd);
  else
    hipLaunchKernelGGL((pad_rows_kernel<double, double>), grid, dim3(256), 0, s, static_cast<const double*>(src),
                       static_cast<double*>(dst), rows, n, ldd);
  return hipGetLastError();
}

}  // namespace qmk
