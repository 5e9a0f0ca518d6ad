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
//   een_ee      rt^k[w][k][i][j] (k = 0..nord-2, zero diagonal), the right
//               operand, plus the m = 0 part of J for electron i;
//   the product (gemm_body, EPI 5) forms P^{k,m} for m >= 1 on MFMA and folds
//               the weights into its epilogue, so P is never stored;
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

// One thread per (point p, nucleus a).
__global__ __launch_bounds__(256) void een_en_kernel(PointArgs pts, int64_t ne, const double* __restrict__ nuc,
                                                     int64_t nn, double kappa, int mh, double* __restrict__ ra,
                                                     double* __restrict__ xo) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= pts.P * nn) return;
  const int64_t p = e / nn, a = e - p * nn;
  const double dx = pts.coord[p * pts.s_pt] - nuc[3 * a];
  const double dy = pts.coord[p * pts.s_pt + pts.s_ax] - nuc[3 * a + 1];
  const double dz = pts.coord[p * pts.s_pt + 2 * pts.s_ax] - nuc[3 * a + 2];
  const double x = exp(-kappa * sqrt(dx * dx + dy * dy + dz * dz));
  double v = x;
  double* o = ra + p * mh * nn + a;
  for (int m = 1; m <= mh; ++m) {
    o[(m - 1) * nn] = v;
    v *= x;
  }
  const int64_t w = p / ne, i = p - w * ne;
  xo[(w * nn + a) * ne + i] = x;
}

// One wave per (walker w, electron i); lanes run over the electrons j and
// then over the nuclei.  Writes rt[w][k][i][j] for k < nsplit and
// j0[w][i] = sum_{k=1}^{nord-1} (sum_{j != i} rt_ij^k) sum_a w_{k,0,a}(x_ia),
// the polynomial coefficients in q0[k-1][a][0..nord].
__global__ __launch_bounds__(256) void een_ee_kernel(PointArgs pts, int64_t ne, double kappa, int nord, int nsplit,
                                                     const double* __restrict__ xi, const double* __restrict__ q0,
                                                     int64_t nn, double* __restrict__ rt, double* __restrict__ j0) {
  const int lane = threadIdx.x & 63;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= pts.P) return;
  const int64_t w = row / ne, i = row - w * ne, pi = row;
  const double xi0 = pts.coord[pi * pts.s_pt], yi0 = pts.coord[pi * pts.s_pt + pts.s_ax],
               zi0 = pts.coord[pi * pts.s_pt + 2 * pts.s_ax];
  double sk[kMaxOrd] = {};
  double* const ro = rt + (w * nsplit * ne + i) * ne;
  for (int64_t j = lane; j < ne; j += 64) {
    const int64_t pj = w * ne + j;
    const double dx = xi0 - pts.coord[pj * pts.s_pt];
    const double dy = yi0 - pts.coord[pj * pts.s_pt + pts.s_ax];
    const double dz = zi0 - pts.coord[pj * pts.s_pt + 2 * pts.s_ax];
    const double x = exp(-kappa * sqrt(dx * dx + dy * dy + dz * dz));
    const double off = j == i ? 0.0 : 1.0;
    double v = off;
#pragma unroll
    for (int k = 0; k < kMaxOrd; ++k) {
      if (k >= nord) break;
      if (k < nsplit) ro[k * ne * ne + j] = v;
      sk[k] += v;
      v *= x;
    }
  }
  double gk[kMaxOrd] = {};
  for (int64_t a = lane; a < nn; a += 64) {
    const double x = xi[(w * nn + a) * ne + i];
#pragma unroll
    for (int k = 1; k < kMaxOrd; ++k) {
      if (k >= nord) break;
      const double* q = q0 + ((k - 1) * nn + a) * (nord + 1);
      double pw = q[nord];
      for (int e = nord - 1; e >= 0; --e) pw = pw * x + q[e];
      gk[k] += pw;
    }
  }
  double acc = 0.0;
#pragma unroll
  for (int k = 1; k < kMaxOrd; ++k) {
    if (k >= nord) break;
    acc += wave_sum(sk[k]) * wave_sum(gk[k]);
  }
  if (lane == 0) j0[row] = acc;
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
  const int64_t n = pts.P * nn;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(een_en_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, pts, ne, nuc,
                     nn, kappa, mh, ra, x);
  return hipGetLastError();
}

hipError_t launch_een_ee(const PointArgs& pts, int64_t ne, double kappa, int nord, int nsplit, const double* x,
                         const double* q0, int64_t nn, double* rt, double* j0, hipStream_t s) {
  if (pts.P <= 0) return hipSuccess;
  if (nord < 2 || nord > kMaxOrd) return hipErrorInvalidValue;
  hipLaunchKernelGGL(een_ee_kernel, dim3(static_cast<unsigned>((pts.P + 3) / 4)), dim3(256), 0, s, pts, ne, kappa,
                     nord, nsplit, x, q0, nn, rt, j0);
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
