// Point ordering for the screened contraction (QMCkl paper, Section 3.2: the
// sparsity of the AOs reduces the cost of the MO product).  On MFMA tiles the
// sparsity is usable only if the points of a tile are close in space: points
// are sorted by their nearest nucleus, so that a 64-point block sees the AOs
// of one neighbourhood.  The sort is a stable radix sort of (nearest
// nucleus, point index) pairs, so the order -- and with it every sum over
// sorted points -- is the same on every run.
#include <hipcub/hipcub.hpp>

#include "qmk_internal.h"

namespace qmk {
namespace {

__global__ __launch_bounds__(256) void nearest_nucleus_kernel(PointArgs pts, const double* __restrict__ nuc,
                                                              int64_t n_nuc, int32_t* __restrict__ key,
                                                              int32_t* __restrict__ index) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= pts.P) return;
  const double x = pts.coord[p * pts.s_pt], y = pts.coord[p * pts.s_pt + pts.s_ax],
               z = pts.coord[p * pts.s_pt + 2 * pts.s_ax];
  double best = INFINITY;
  int32_t arg = 0;
  for (int64_t a = 0; a < n_nuc; ++a) {
    const double dx = x - nuc[3 * a], dy = y - nuc[3 * a + 1], dz = z - nuc[3 * a + 2];
    const double u = dx * dx + dy * dy + dz * dz;
    if (u < best) {
      best = u;
      arg = static_cast<int32_t>(a);
    }
  }
  key[p] = arg;
  index[p] = static_cast<int32_t>(p);
}

// dst row q = src row perm[q]; rows of `row` elements of `esz` bytes, moved
// as 4-byte words (row * esz is a multiple of 4).
__global__ __launch_bounds__(256) void gather_rows_kernel(const uint32_t* __restrict__ src,
                                                          const int32_t* __restrict__ perm, int64_t rows,
                                                          int64_t words, uint32_t* __restrict__ dst) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rows * words) return;
  const int64_t q = e / words, x = e - q * words;
  dst[e] = src[static_cast<int64_t>(perm[q]) * words + x];
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_gather_rows(const void* src, const int32_t* perm, int64_t rows, int64_t row_bytes, void* dst,
                              hipStream_t s) {
  if (rows <= 0 || row_bytes % 4 != 0) return rows <= 0 ? hipSuccess : hipErrorInvalidValue;
  const int64_t words = row_bytes / 4, n = rows * words;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s,
                     static_cast<const uint32_t*>(src), perm, rows, words, static_cast<uint32_t*>(dst));
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

static int key_bits(int64_t n_nuc) {
  int b = 1;
  while ((int64_t{1} << b) < n_nuc) ++b;
  return b;
}

size_t sort_scratch_bytes(int64_t P, int64_t n_nuc) {
  size_t bytes = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, static_cast<const int32_t*>(nullptr),
                                           static_cast<int32_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                                           static_cast<int32_t*>(nullptr), static_cast<int>(P), 0,
                                           key_bits(n_nuc));
  return bytes;
}

hipError_t launch_sort_points(const PointArgs& pts, const double* nuc_xyz, int64_t n_nuc, int32_t* key,
                              int32_t* key_sorted, int32_t* index, int32_t* perm, void* scratch,
                              size_t scratch_bytes, hipStream_t s) {
  if (pts.P <= 0) return hipSuccess;
  hipLaunchKernelGGL(nearest_nucleus_kernel, dim3(static_cast<unsigned>((pts.P + 255) / 256)), dim3(256), 0, s,
                     pts, nuc_xyz, n_nuc, key, index);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipcub::DeviceRadixSort::SortPairs(scratch, scratch_bytes, key, key_sorted, index, perm,
                                            static_cast<int>(pts.P), 0, key_bits(n_nuc), s);
}

}  // namespace qmk
