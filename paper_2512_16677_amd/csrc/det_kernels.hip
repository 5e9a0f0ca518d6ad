// Determinant and adjugate of batches of small matrices (QMCkl paper,
// Section 3.4: the inverse is adj(A) / det(A); returning det and adj(A)
// together serves the gradients of Slater determinants, and for n < 5 the
// explicit cofactor form beats an LU factorisation).
//
// n <= 4: one lane per matrix (staged through LDS for coalesced loads and
// stores); the n*n entries live in registers and every
// cofactor is an unrolled signed minor determinant (Laplace expansion along
// the first row, compile-time n), so the result is exact also for singular
// matrices.  5 <= n <= 32: one wavefront per matrix, LU with partial
// pivoting in LDS (lanes over rows), det = sign * prod(U_kk), and
// adj = det * A^{-1} from substitutions (lanes over columns of A^{-1}).
#include "qmk_internal.h"

namespace qmk {
namespace {

// Determinant of the m x m matrix made of rows r[0..m) and columns c[0..m)
// of the n x n row-major matrix a (Laplace expansion along the first row).
template <int N, int M>
struct Minor {
  static __device__ __forceinline__ double det(const double (&a)[N * N], const int (&r)[M],
                                               const int (&c)[M]) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j) {
      int rr[M - 1], cc[M - 1];
#pragma unroll
      for (int k = 0; k < M - 1; ++k) {
        rr[k] = r[k + 1];
        cc[k] = c[k < j ? k : k + 1];
      }
      const double t = a[r[0] * N + c[j]] * Minor<N, M - 1>::det(a, rr, cc);
      s += (j & 1) ? -t : t;
    }
    return s;
  }
};
template <int N>
struct Minor<N, 1> {
  static __device__ __forceinline__ double det(const double (&a)[N * N], const int (&r)[1],
                                               const int (&c)[1]) {
    return a[r[0] * N + c[0]];
  }
};

// The 256 matrices of a workgroup pass through LDS (rows padded by one
// element against bank conflicts), so that the global loads and stores of the
// workgroup cover one contiguous range, coalesced across lanes.
template <int N>
__global__ __launch_bounds__(256) void det_adj_small_kernel(const double* __restrict__ A, int64_t batch,
                                                            double* __restrict__ det,
                                                            double* __restrict__ adj) {
  constexpr int E = N * N, LD = E + 1;
  __shared__ double s_m[256 * LD];
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * 256;
  const int64_t nb = min<int64_t>(256, batch - b0);
  const double* src = A + b0 * E;
  for (int64_t e = threadIdx.x; e < nb * E; e += 256) s_m[(e / E) * LD + e % E] = src[e];
  __syncthreads();
  const int t = threadIdx.x;
  double a[E];
  if (t < nb) {
#pragma unroll
    for (int i = 0; i < E; ++i) a[i] = s_m[t * LD + i];
  }
  __syncthreads();  // s_m is reused for the adjugates
  if (t < nb) {
    if constexpr (N == 1) {
      det[b0 + t] = a[0];
      s_m[t * LD] = 1.0;
    } else {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) {
          // cofactor C_ij = (-1)^(i+j) det(A without row i, column j); adj = C^T
          int r[N - 1], c[N - 1];
#pragma unroll
          for (int k = 0; k < N - 1; ++k) {
            r[k] = k < i ? k : k + 1;
            c[k] = k < j ? k : k + 1;
          }
          const double m = Minor<N, N - 1>::det(a, r, c);
          const double cij = ((i + j) & 1) ? -m : m;
          s_m[t * LD + j * N + i] = cij;
          if (i == 0) d += a[j] * cij;
        }
      det[b0 + t] = d;
    }
  }
  __syncthreads();
  double* dst = adj + b0 * E;
  for (int64_t e = threadIdx.x; e < nb * E; e += 256) dst[e] = s_m[(e / E) * LD + e % E];
}

// One wavefront per matrix, 4 per workgroup; n <= 32.
__global__ __launch_bounds__(256) void det_adj_lu_kernel(const double* __restrict__ A, int n, int64_t batch,
                                                         double* __restrict__ det,
                                                         double* __restrict__ adj) {
  __shared__ double s_lu[4][32][33];
  __shared__ int s_piv[4][32];
  __shared__ double s_a[4][32], s_r[4][32];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t b = static_cast<int64_t>(blockIdx.x) * 4 + w;
  if (b >= batch) return;  // whole waves leave together; no workgroup barrier below
  double(*lu)[33] = s_lu[w];
  const double* src = A + b * n * n;
  for (int e = lane; e < n * n; e += 64) lu[e / n][e % n] = src[e];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  double sign = 1.0, d = 1.0;
  for (int k = 0; k < n; ++k) {
    // pivot: largest |a_ik|, i >= k (ties to the lowest row)
    double v = lane >= k && lane < n ? fabs(lu[lane][k]) : -1.0;
    int idx = lane;
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(v, off, 64);
      const int oi = __shfl_xor(idx, off, 64);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
    const int p = idx;
    if (lane == 0) s_piv[w][k] = p;
    if (p != k) {
      if (lane < n) {
        const double t = lu[k][lane];
        lu[k][lane] = lu[p][lane];
        lu[p][lane] = t;
      }
      sign = -sign;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double piv = lu[k][k];
    d *= piv;
    if (lane > k && lane < n) {
      // a zero pivot leaves only zeros below it: nothing to eliminate
      const double l = piv != 0.0 ? lu[lane][k] / piv : 0.0;
      lu[lane][k] = l;
      for (int j = k + 1; j < n; ++j) lu[lane][j] -= l * lu[k][j];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  d *= sign;
  if (lane == 0) det[b] = d;
  // Exactly zero pivots make d A^{-1} undefined; the adjugate is still the
  // transposed cofactor matrix.  With PA = LU, adj(A) = adj(U) L^{-1} sign P.
  // Two or more zero pivots (rank <= n - 2): adj(A) = 0.  One, at k0 (rank
  // n - 1): adj(U) = c a b^T with c = prod_{m != k0} u_mm (the (k0, k0)
  // cofactor), U a = 0, a_k0 = 1, a_m = 0 past k0, and b^T U = 0, b_k0 = 1,
  // b_m = 0 before k0; so adj(A) = sign c a r^T with r = P^T L^{-T} b.
  int nzero = 0, k0 = -1;
  for (int m = 0; m < n; ++m)
    if (lu[m][m] == 0.0) {
      ++nzero;
      k0 = m;
    }
  if (nzero > 0) {
    double* dst = adj + b * n * n;
    if (nzero >= 2) {
      for (int e = lane; e < n * n; e += 64) dst[e] = 0.0;
      return;
    }
    if (lane == 0) {
      double c = sign;
      for (int m = 0; m < n; ++m)
        if (m != k0) c *= lu[m][m];
      double* a = s_a[w];
      double* r = s_r[w];
      for (int m = n - 1; m >= 0; --m) {
        if (m >= k0) {
          a[m] = m == k0 ? 1.0 : 0.0;
        } else {
          double t = 0.0;
          for (int q = m + 1; q <= k0; ++q) t += lu[m][q] * a[q];
          a[m] = -t / lu[m][m];
        }
      }
      // b into r, then z = L^{-T} b in place (L unit lower, below the diagonal of lu)
      for (int j = 0; j < n; ++j) {
        if (j <= k0) {
          r[j] = j == k0 ? 1.0 : 0.0;
        } else {
          double t = 0.0;
          for (int q = k0; q < j; ++q) t += r[q] * lu[q][j];
          r[j] = -t / lu[j][j];
        }
      }
      for (int i = n - 1; i >= 0; --i)
        for (int j = i + 1; j < n; ++j) r[i] -= lu[j][i] * r[j];
      // r = P^T z: the row swaps undone in reverse order
      for (int k = n - 1; k >= 0; --k) {
        const int p = s_piv[w][k];
        const double t = r[k];
        r[k] = r[p];
        r[p] = t;
      }
      for (int m = 0; m < n; ++m) a[m] *= c;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < n)
      for (int i = 0; i < n; ++i) dst[i * n + lane] = s_a[w][i] * s_r[w][lane];
    return;
  }
  // column `lane` of A^{-1}: solve L U x = P e_lane
  if (lane < n) {
    double x[32];
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    // P e_lane: the row permutation applied to the identity
    int col = lane;
    for (int k = 0; k < n; ++k) {
      const int p = s_piv[w][k];
      if (col == k) col = p;
      else if (col == p) col = k;
    }
    x[col] = 1.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) x[i] -= lu[i][j] * x[j];
    for (int i = n - 1; i >= 0; --i) {
      for (int j = i + 1; j < n; ++j) x[i] -= lu[i][j] * x[j];
      x[i] /= lu[i][i];
    }
    double* dst = adj + b * n * n;
    for (int i = 0; i < n; ++i) dst[i * n + lane] = d * x[i];
  }
}

}  // namespace

hipError_t launch_det_adj(int n, int64_t batch, const double* A, double* det, double* adj, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  const dim3 blk(256);
  const dim3 g_small(static_cast<unsigned>((batch + 255) / 256));
  switch (n) {
    case 1: hipLaunchKernelGGL(det_adj_small_kernel<1>, g_small, blk, 0, s, A, batch, det, adj); break;
    case 2: hipLaunchKernelGGL(det_adj_small_kernel<2>, g_small, blk, 0, s, A, batch, det, adj); break;
    case 3: hipLaunchKernelGGL(det_adj_small_kernel<3>, g_small, blk, 0, s, A, batch, det, adj); break;
    case 4: hipLaunchKernelGGL(det_adj_small_kernel<4>, g_small, blk, 0, s, A, batch, det, adj); break;
    default:
      if (n < 1 || n > 32) return hipErrorInvalidValue;
      hipLaunchKernelGGL(det_adj_lu_kernel, dim3(static_cast<unsigned>((batch + 3) / 4)), blk, 0, s, A, n,
                         batch, det, adj);
  }
  return hipGetLastError();
}

}  // namespace qmk
