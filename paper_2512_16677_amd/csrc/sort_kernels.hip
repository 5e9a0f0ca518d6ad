// Point ordering for the screened contraction (QMCkl paper, Section 3.2: the
// sparsity of the AOs reduces the cost of the MO product).  On MFMA tiles the
// sparsity is usable only if the points of a tile are close in space: points
// are sorted by their nearest nucleus, so that a 64-point block sees the AOs
// of one neighbourhood.  The sort is a stable counting sort of the points by
// nearest nucleus (keys 0 .. n_nuc-1), so the order -- and with it every sum
// over sorted points -- is the same on every run:
//   1. nearest nucleus of every point, and per block of kSortBlock points the
//      count of each key (LDS histogram), stored as hist[key][block];
//   2. exclusive scan of hist in (key, block) order: each key's blocks in
//      order, one wave per key, then the keys' totals in order;
//   3. per block, one wave walks its points in order; a point's position is
//      its (key, block) offset plus the number of earlier points of the block
//      with the same key.
#include "qmk_internal.h"

namespace qmk {
namespace {

constexpr int kSortBlock = 1024;                // points per histogram block (4 per thread)
constexpr int kSortMaxKeys = kSortMaxNuclei;  // LDS histogram of one block

__global__ __launch_bounds__(256) void nearest_nucleus_kernel(PointArgs pts, const double* __restrict__ nuc,
                                                              int64_t n_nuc, int64_t n_blocks,
                                                              int32_t* __restrict__ key,
                                                              int32_t* __restrict__ hist) {
  __shared__ int32_t h[kSortMaxKeys];
  for (int64_t i = threadIdx.x; i < n_nuc; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int r = 0; r < kSortBlock / 256; ++r) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * kSortBlock + r * 256 + threadIdx.x;
    if (p >= pts.P) break;
    const double x = pts.coord[p * pts.s_pt], y = pts.coord[p * pts.s_pt + pts.s_ax],
                 z = pts.coord[p * pts.s_pt + 2 * pts.s_ax];
    double best = INFINITY;
    int32_t arg = 0;
    for (int64_t a = 0; a < n_nuc; ++a) {
      const double u = dist2(x - nuc[3 * a], y - nuc[3 * a + 1], z - nuc[3 * a + 2]);
      if (u < best) {
        best = u;
        arg = static_cast<int32_t>(a);
      }
    }
    key[p] = arg;
    atomicAdd(&h[arg], 1);
  }
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n_nuc; i += blockDim.x) hist[i * n_blocks + blockIdx.x] = h[i];
}

// One wave per key: exclusive scan of the key's block counts in place; the
// key's total to tot[key].
__global__ __launch_bounds__(256) void scan_blocks_kernel(int32_t* __restrict__ hist, int64_t n_nuc,
                                                          int64_t n_blocks, int32_t* __restrict__ tot) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= n_nuc) return;
  int32_t* row = hist + k * n_blocks;
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < n_blocks; b0 += 64) {
    const int64_t b = b0 + lane;
    const int32_t v = b < n_blocks ? row[b] : 0;
    int32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    if (b < n_blocks) row[b] = carry + incl - v;
    carry += __shfl(incl, 63, 64);
  }
  if (lane == 0) tot[k] = carry;
}

// One workgroup: exclusive scan of the keys' totals in place.
__global__ __launch_bounds__(1024) void scan_keys_kernel(int32_t* __restrict__ tot, int64_t n_nuc) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t s_carry;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t k0 = 0; k0 < n_nuc; k0 += 1024) {
    const int64_t k = k0 + threadIdx.x;
    const int32_t v = k < n_nuc ? tot[k] : 0;
    int32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t before = s_carry;
    for (int i = 0; i < w; ++i) before += wsum[i];
    if (k < n_nuc) tot[k] = before + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t t = 0;
      for (int i = 0; i < 16; ++i) t += wsum[i];
      s_carry += t;
    }
    __syncthreads();
  }
}

// One wave per block of kSortBlock points, walking them 64 at a time in
// order: stable positions from the per-key running offsets in LDS.
__global__ __launch_bounds__(64) void scatter_kernel(const int32_t* __restrict__ key, int64_t P, int64_t n_nuc,
                                                     int64_t n_blocks, const int32_t* __restrict__ hist,
                                                     const int32_t* __restrict__ tot, int32_t* __restrict__ perm) {
  __shared__ int32_t next[kSortMaxKeys];
  const int lane = threadIdx.x;
  const int64_t blk = blockIdx.x;
  for (int64_t i = lane; i < n_nuc; i += 64) next[i] = tot[i] + hist[i * n_blocks + blk];
  __syncthreads();
  for (int r = 0; r < kSortBlock / 64; ++r) {
    const int64_t p = blk * kSortBlock + r * 64 + lane;
    const bool in = p < P;
    const int32_t k = in ? key[p] : -1;
    // rank among the earlier lanes with the same key
    int32_t rank = 0, last = 1;
    for (int j = 0; j < 64; ++j) {
      const int32_t kj = __shfl(k, j, 64);
      if (kj == k && j < lane) ++rank;
      if (kj == k && j > lane) last = 0;
    }
    if (in) perm[next[k] + rank] = static_cast<int32_t>(p);
    __syncthreads();
    // the last lane of each key advances that key's offset
    if (in && last) next[k] += rank + 1;
    __syncthreads();
  }
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

size_t sort_scratch_bytes(int64_t P, int64_t n_nuc) {
  const int64_t n_blocks = (P + kSortBlock - 1) / kSortBlock;
  return static_cast<size_t>((n_nuc * n_blocks + n_nuc) * 4);
}

hipError_t launch_sort_points(const PointArgs& pts, const double* nuc_xyz, int64_t n_nuc, int32_t* key,
                              int32_t* perm, void* scratch, size_t scratch_bytes, hipStream_t s) {
  if (pts.P <= 0) return hipSuccess;
  if (n_nuc < 1 || n_nuc > kSortMaxKeys || pts.P > 0x7fffffffLL) return hipErrorInvalidValue;
  const int64_t n_blocks = (pts.P + kSortBlock - 1) / kSortBlock;
  if (scratch_bytes < sort_scratch_bytes(pts.P, n_nuc)) return hipErrorInvalidValue;
  int32_t* hist = static_cast<int32_t*>(scratch);
  int32_t* tot = hist + n_nuc * n_blocks;
  hipLaunchKernelGGL(nearest_nucleus_kernel, dim3(static_cast<unsigned>(n_blocks)), dim3(256), 0, s, pts, nuc_xyz,
                     n_nuc, n_blocks, key, hist);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(static_cast<unsigned>((n_nuc + 3) / 4)), dim3(256), 0, s, hist, n_nuc,
                     n_blocks, tot);
  hipLaunchKernelGGL(scan_keys_kernel, dim3(1), dim3(1024), 0, s, tot, n_nuc);
  hipLaunchKernelGGL(scatter_kernel, dim3(static_cast<unsigned>(n_blocks)), dim3(64), 0, s, key, pts.P, n_nuc,
                     n_blocks, hist, tot, perm);
  return hipGetLastError();
}

}  // namespace qmk
