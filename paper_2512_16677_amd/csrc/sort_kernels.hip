// Point ordering for the screened contraction (QMCkl paper, Section 3.2: the
// sparsity of the AOs reduces the cost of the MO product).  On MFMA tiles the
// sparsity is usable only if the points of a tile are close in space: points
// are counting-sorted by their nearest nucleus, so that a 64-point block sees
// the AOs of one neighbourhood.  Points of one nucleus keep no particular
// order among themselves (atomic slots); the product does not depend on it.
#include "qmk_internal.h"

namespace qmk {
namespace {

__global__ __launch_bounds__(256) void nearest_nucleus_kernel(PointArgs pts, const double* __restrict__ nuc,
                                                              int64_t n_nuc, int32_t* __restrict__ key,
                                                              int32_t* __restrict__ counts) {
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
  atomicAdd(counts + arg, 1);
}

// Exclusive prefix sum of counts[0..n) in place (one workgroup; the sums of
// 256-entry pieces are carried serially).
__global__ __launch_bounds__(256) void scan_counts_kernel(int32_t* __restrict__ counts, int64_t n) {
  __shared__ int32_t part[256];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 256) {
    const int64_t i = base + threadIdx.x;
    const int32_t v = i < n ? counts[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < n) counts[i] = carry + part[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 255) carry += part[255];
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void scatter_points_kernel(const int32_t* __restrict__ key, int64_t P,
                                                             int32_t* __restrict__ cursor,
                                                             int32_t* __restrict__ perm) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  perm[atomicAdd(cursor + key[p], 1)] = static_cast<int32_t>(p);
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_sort_points(const PointArgs& pts, const double* nuc_xyz, int64_t n_nuc, int32_t* key,
                              int32_t* counts, int32_t* perm, hipStream_t s) {
  if (pts.P <= 0) return hipSuccess;
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(counts), n_nuc, 0u, s);
  if (e != hipSuccess) return e;
  const dim3 grid(static_cast<unsigned>((pts.P + 255) / 256));
  hipLaunchKernelGGL(nearest_nucleus_kernel, grid, dim3(256), 0, s, pts, nuc_xyz, n_nuc, key, counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(scan_counts_kernel, dim3(1), dim3(256), 0, s, counts, n_nuc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_points_kernel, grid, dim3(256), 0, s, key, pts.P, counts, perm);
  return hipGetLastError();
}

}  // namespace qmk
