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
//   een_g0      the nucleus sums of the m = 0 weights per electron;
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

// One thread per point p = (walker w, electron i):
//   g0[p][k-1] = sum_a w_{k,0,a}(x[w][a][i]),  k = 1..NORD-1,
// with the polynomial coefficients q0[k-1][a][0..NORD] staged in LDS for 64
// nuclei at a time.
constexpr int kG0Chunk = 64;
template <int NORD>
__global__ __launch_bounds__(256) void een_g0_kernel(const double* __restrict__ x, int64_t P, int64_t ne, int64_t nn,
                                                     const double* __restrict__ q0, double* __restrict__ g0) {
  constexpr int NQ = (NORD - 1) * (NORD + 1);
  __shared__ double qs[kG0Chunk * NQ];
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool valid = p < P;
  const int64_t w = valid ? p / ne : 0, i = valid ? p - w * ne : 0;
  double g[NORD - 1] = {};
  for (int64_t a0 = 0; a0 < nn; a0 += kG0Chunk) {
    const int an = static_cast<int>(min<int64_t>(kG0Chunk, nn - a0));
    __syncthreads();
    for (int t = threadIdx.x; t < an * NQ; t += blockDim.x) {
      const int al = t / NQ, r = t - al * NQ;  // r = (k-1) (NORD+1) + e
      const int k1 = r / (NORD + 1), e = r - k1 * (NORD + 1);
      qs[t] = q0[(k1 * nn + a0 + al) * (NORD + 1) + e];
    }
    __syncthreads();
    for (int al = 0; al < an; ++al) {
      const double xv = valid ? x[(w * nn + a0 + al) * ne + i] : 0.0;
      const double* q = qs + al * NQ;
#pragma unroll
      for (int k1 = 0; k1 < NORD - 1; ++k1) {
        double pw = q[k1 * (NORD + 1) + NORD];
#pragma unroll
        for (int e = NORD - 1; e >= 0; --e) pw = pw * xv + q[k1 * (NORD + 1) + e];
        g[k1] += pw;
      }
    }
  }
  if (!valid) return;
#pragma unroll
  for (int k1 = 0; k1 < kMaxOrd - 1; ++k1) g0[p * (kMaxOrd - 1) + k1] = k1 < NORD - 1 ? g[k1] : 0.0;
}

// Block = (walker w, 16 electrons i); each wave takes 4 of them and its
// lanes run over the electrons j, whose coordinates are staged in LDS in
// chunks.  Writes rt[w][i][j] = exp(-kappa r_ij), -1 on the diagonal (the
// product takes powers and maps the diagonal to zero), and
//   j0[w][i] = sum_{k=1}^{nord-1} (sum_{j != i} rt_ij^k) g0[w][i][k-1]
// (g0 from een_g0_kernel).
constexpr int kEeRows = 2, kEeChunk = 512;
template <int NORD>
__global__ __launch_bounds__(256) void een_ee_kernel(PointArgs pts, int64_t ne, double kappa,
                                                     const double* __restrict__ g0, double* __restrict__ rt,
                                                     double* __restrict__ j0) {
  __shared__ double cs[3][kEeChunk];
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
  double sk[kEeRows][NORD] = {};  // [row][k]: sum_j rt_ij^k, k = 1 .. NORD-1
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
      // the rows are independent chains: no branch between them
      double x[kEeRows];
#pragma unroll
      for (int r = 0; r < kEeRows; ++r) {
        const double dx = xi[r] - xj, dy = yi[r] - yj, dz = zi[r] - zj;
        x[r] = exp(-kappa * sqrt(dx * dx + dy * dy + dz * dz));
      }
#pragma unroll
      for (int r = 0; r < kEeRows; ++r) {
        const int64_t i = ib + r;
        const bool diag = j == i;
        if (i < ne) rt[(w * ne + i) * ne + j] = diag ? -1.0 : x[r];
        double v = diag ? 0.0 : x[r];
#pragma unroll
        for (int k = 1; k < NORD; ++k) {
          sk[r][k] += v;
          v *= x[r];
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kEeRows; ++r) {
    const int64_t i = min(ib + r, ne - 1);
    const double* g = g0 + (w * ne + i) * (kMaxOrd - 1);
    double acc = 0.0;
#pragma unroll
    for (int k = 1; k < NORD; ++k) acc += wave_sum(sk[r][k]) * g[k - 1];
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

hipError_t launch_een_ee(const PointArgs& pts, int64_t ne, int64_t nn, double kappa, int nord, const double* x,
                         const double* q0, double* g0, double* rt, double* j0, hipStream_t s) {
  if (pts.P <= 0) return hipSuccess;
  if (nord < 2 || nord > kMaxOrd) return hipErrorInvalidValue;
  const dim3 gg(static_cast<unsigned>((pts.P + 255) / 256));
  const int64_t nw = pts.P / ne, g = nw * ((ne + 4 * kEeRows - 1) / (4 * kEeRows));
  if (g > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 ge(static_cast<unsigned>(g));
  switch (nord) {
#define QMK_EEN(n)                                                                                \
  case n:                                                                                         \
    hipLaunchKernelGGL(een_g0_kernel<n>, gg, dim3(256), 0, s, x, pts.P, ne, nn, q0, g0);          \
    if (hipPeekAtLastError() != hipSuccess) break;                                                \
    hipLaunchKernelGGL(een_ee_kernel<n>, ge, dim3(256), 0, s, pts, ne, kappa, g0, rt, j0);        \
    break;
    QMK_EEN(2) QMK_EEN(3) QMK_EEN(4) QMK_EEN(5) QMK_EEN(6) QMK_EEN(7) QMK_EEN(8)
#undef QMK_EEN
  }
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
