// Three-body (electron-electron-nucleus) Jastrow factor through the
// intermediate matrix P (QMCkl paper, Section 3.5):
//   P^{k,m}_{i a} = sum_{j != i} rt_ij^k Rt_ja^m,
//   J = sum_t sum_a c[t,a] sum_i Rt_ia^((p-k+l)/2) P^{k,(p-k-l)/2}_{i a},
// with rt_ij = exp(-kappa r_ij) and Rt_ia = exp(-kappa |r_i - R_a|).
//
// Grouping the terms by (k, m), J = sum_{k,m} sum_{i,a} w_{k,m,a}(Rt_ia)
// P^{k,m}_{ia} with w_{k,m,a} a polynomial in Rt_ia whose coefficients are
// the c[t,a] of the terms with that (k, m).  Terms with m >= 1 have
// k <= nord - 2 and m <= nord / 2; terms with m = 0 (k >= 1) need only
// P^{k,0}_i = sum_{j != i} rt_ij^k, which does not depend on the nucleus.
// Per walker:
//   een_en      Ra[p][(m-1) nn + a] = Rt_pa^m (m = 1..mh), the left operand of
//               the product, and x[w][a][i] = Rt_ia;
//   een_ee      rt[w][i][j] (diagonal marked), the right operand, plus the
//               m = 0 part of J for electron i;
//   the product (gemm_body, EPI 5) forms P^{k,m} for m >= 1 on MFMA, taking
//               the k-th power of rt as it stages B (split k), and folds the
//               weights into its epilogue, so neither rt^k nor P is stored;
//   een_finish  sums the per-wave partial sums and the m = 0 parts of one
//               walker in a fixed order (deterministic).
#include "qmk_internal.h"

namespace qmk {
namespace {

constexpr int kMaxOrd = 8;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block = (walker, 16 electrons) x 64 nuclei.  Ra is written nucleus-fast
// and x electron-fast (through an LDS transpose), both in full lines.
__global__ __launch_bounds__(256) void een_en_kernel(PointArgs pts, int64_t ne, const double* __restrict__ nuc,
                                                     int64_t nn, double kappa, int mh, double* __restrict__ ra,
                                                     double* __restrict__ xo) {
  __shared__ double xs[16][65];
  const int64_t nblk = (ne + 15) / 16;
  const int64_t w = blockIdx.x / nblk, i0 = (blockIdx.x - w * nblk) * 16, a0 = static_cast<int64_t>(blockIdx.y) * 64;
  const int64_t M = mh * nn;
  for (int idx = threadIdx.x; idx < 16 * 64; idx += 256) {
    const int il = idx >> 6, al = idx & 63;
    const int64_t i = i0 + il, a = a0 + al;
    if (i >= ne || a >= nn) continue;
    const int64_t p = w * ne + i;
    const double dx = pts.coord[p * pts.s_pt] - nuc[3 * a];
    const double dy = pts.coord[p * pts.s_pt + pts.s_ax] - nuc[3 * a + 1];
    const double dz = pts.coord[p * pts.s_pt + 2 * pts.s_ax] - nuc[3 * a + 2];
    const double x = exp(-kappa * sqrt(dx * dx + dy * dy + dz * dz));
    double v = x;
    double* o = ra + p * M + a;
    for (int m = 1; m <= mh; ++m) {
      o[(m - 1) * nn] = v;
      v *= x;
    }
    xs[il][al] = x;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 16 * 64; idx += 256) {
    const int al = idx >> 4, il = idx & 15;
    const int64_t i = i0 + il, a = a0 + al;
    if (i < ne && a < nn) xo[(w * nn + a) * ne + i] = xs[il][al];
  }
}

// Block = (walker w, 16 electrons i); each wave takes 4 of them, its lanes
// run over the electrons j and then over the nuclei, whose coordinates are
// staged in LDS in chunks.  Writes rt[w][i][j] = exp(-kappa r_ij), -1 on the
// diagonal (the product takes powers and maps the diagonal to zero), and
// j0[w][i] = sum_{k=1}^{nord-1} (sum_{j != i} rt_ij^k) sum_a w_{k,0,a}(Rt_ia),
// the polynomial coefficients in q0[k-1][a][0..nord].
constexpr int kEeRows = 4, kEeChunk = 512;
__global__ __launch_bounds__(256) void een_ee_kernel(PointArgs pts, int64_t ne, const double* __restrict__ nuc,
                                                     int64_t nn, double kappa, int nord,
                                                     const double* __restrict__ q0, double* __restrict__ rt,
                                                     double* __restrict__ j0) {
  __shared__ double cs[3][kEeChunk];
  __shared__ double gs[4][kEeRows][kMaxOrd];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nblk = (ne + 4 * kEeRows - 1) / (4 * kEeRows);
  const int64_t w = blockIdx.x / nblk, ib = (blockIdx.x - w * nblk) * 4 * kEeRows + wv * kEeRows;
  double xi[kEeRows], yi[kEeRows], zi[kEeRows];
#pragma unroll
  for (int r = 0; r < kEeRows; ++r) {
    const int64_t p = w * ne + min(ib + r, ne - 1);
    xi[r] = pts.coord[p * pts.s_pt];
    yi[r] = pts.coord[p * pts.s_pt + pts.s_ax];
    zi[r] = pts.coord[p * pts.s_pt + 2 * pts.s_ax];
  }
  // nuclei: G[r][k] = sum_a w_{k,0,a}(Rt_ia), kept in LDS per wave
  {
    double gk[kEeRows][kMaxOrd] = {};
    for (int64_t c0 = 0; c0 < nn; c0 += kEeChunk) {
      const int cn = static_cast<int>(min<int64_t>(kEeChunk, nn - c0));
      __syncthreads();
      for (int t = threadIdx.x; t < 3 * cn; t += blockDim.x) cs[t % 3][t / 3] = nuc[3 * c0 + t];
      __syncthreads();
      for (int t = lane; t < cn; t += 64) {
        const int64_t a = c0 + t;
        double x[kEeRows];
#pragma unroll
        for (int r = 0; r < kEeRows; ++r) {
          const double dx = xi[r] - cs[0][t], dy = yi[r] - cs[1][t], dz = zi[r] - cs[2][t];
          x[r] = exp(-kappa * sqrt(dx * dx + dy * dy + dz * dz));
        }
        for (int k = 1; k < nord; ++k) {
          const double* q = q0 + ((k - 1) * nn + a) * (nord + 1);
          double pw[kEeRows];
#pragma unroll
          for (int r = 0; r < kEeRows; ++r) pw[r] = q[nord];
          for (int e = nord - 1; e >= 0; --e) {
            const double qe = q[e];
#pragma unroll
            for (int r = 0; r < kEeRows; ++r) pw[r] = pw[r] * x[r] + qe;
          }
#pragma unroll
          for (int r = 0; r < kEeRows; ++r)
#pragma unroll
            for (int kk = 1; kk < kMaxOrd; ++kk)
              if (kk == k) gk[r][kk] += pw[r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kEeRows; ++r)
#pragma unroll
      for (int k = 1; k < kMaxOrd; ++k) {
        const double g = wave_sum(gk[r][k]);
        if (lane == 0) gs[wv][r][k] = g;
      }
  }
  // electrons: rt row and S[r][k] = sum_{j != i} rt_ij^k
  double sk[kEeRows][kMaxOrd] = {};
  for (int64_t c0 = 0; c0 < ne; c0 += kEeChunk) {
    const int cn = static_cast<int>(min<int64_t>(kEeChunk, ne - c0));
    __syncthreads();
    for (int t = threadIdx.x; t < cn; t += blockDim.x) {
      const int64_t p = w * ne + c0 + t;
      cs[0][t] = pts.coord[p * pts.s_pt];
      cs[1][t] = pts.coord[p * pts.s_pt + pts.s_ax];
      cs[2][t] = pts.coord[p * pts.s_pt + 2 * pts.s_ax];
    }
    __syncthreads();
    for (int t = lane; t < cn; t += 64) {
      const int64_t j = c0 + t;
      const double xj = cs[0][t], yj = cs[1][t], zj = cs[2][t];
#pragma unroll
      for (int r = 0; r < kEeRows; ++r) {
        const int64_t i = ib + r;
        if (i >= ne) break;
        const double dx = xi[r] - xj, dy = yi[r] - yj, dz = zi[r] - zj;
        const double x = exp(-kappa * sqrt(dx * dx + dy * dy + dz * dz));
        rt[(w * ne + i) * ne + j] = j == i ? -1.0 : x;
        double v = j == i ? 0.0 : x;
#pragma unroll
        for (int k = 1; k < kMaxOrd; ++k) {
          if (k >= nord) break;
          sk[r][k] += v;
          v *= x;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kEeRows; ++r) {
    double acc = 0.0;
#pragma unroll
    for (int k = 1; k < kMaxOrd; ++k) {
      if (k >= nord) break;
      acc += wave_sum(sk[r][k]) * gs[wv][r][k];
    }
    if (lane == 0 && ib + r < ne) j0[w * ne + ib + r] = acc;
  }
}

// One wave per walker: J[w] = sum of the walker's `slots` partial sums and
// of its ne m = 0 parts (fixed lane assignment and tree: deterministic).
__global__ __launch_bounds__(256) void een_finish_kernel(const double* __restrict__ part, int64_t slots,
                                                         const double* __restrict__ j0, int64_t nw, int64_t ne,
                                                         double* __restrict__ J) {
  const int lane = threadIdx.x & 63;
  const int64_t w = static_cast<int64_t>(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (w >= nw) return;
  double v = 0.0;
  for (int64_t t = lane; t < slots; t += 64) v += part[w * slots + t];
  for (int64_t i = lane; i < ne; i += 64) v += j0[w * ne + i];
  v = wave_sum(v);
  if (lane == 0) J[w] = v;
}

}  // namespace

hipError_t launch_een_en(const PointArgs& pts, int64_t ne, const double* nuc, int64_t nn, double kappa, int mh,
                         double* ra, double* x, hipStream_t s) {
  if (pts.P <= 0 || nn <= 0) return hipSuccess;
  const int64_t nw = pts.P / ne, gx = nw * ((ne + 15) / 16), gy = (nn + 63) / 64;
  if (gx > 0x7fffffff || gy > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(een_en_kernel, dim3(static_cast<unsigned>(gx), static_cast<unsigned>(gy)), dim3(256), 0, s, pts,
                     ne, nuc, nn, kappa, mh, ra, x);
  return hipGetLastError();
}

hipError_t launch_een_ee(const PointArgs& pts, int64_t ne, const double* nuc, int64_t nn, double kappa, int nord,
                         const double* q0, double* rt, double* j0, hipStream_t s) {
  if (pts.P <= 0) return hipSuccess;
  if (nord < 2 || nord > kMaxOrd) return hipErrorInvalidValue;
  const int64_t nw = pts.P / ne, g = nw * ((ne + 4 * kEeRows - 1) / (4 * kEeRows));
  if (g > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(een_ee_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, pts, ne, nuc, nn, kappa, nord,
                     q0, rt, j0);
  return hipGetLastError();
}

hipError_t launch_een_finish(const double* part, int64_t slots, const double* j0, int64_t nw, int64_t ne,
                             double* J, hipStream_t s) {
  if (nw <= 0) return hipSuccess;
  hipLaunchKernelGGL(een_finish_kernel, dim3(static_cast<unsigned>((nw + 3) / 4)), dim3(256), 0, s, part, slots, j0,
                     nw, ne, J);
  return hipGetLastError();
}

}  // namespace qmk
