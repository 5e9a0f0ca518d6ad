// AO -> MO contraction and adjoint GEMMs on MFMA (QMCkl paper, Section 3.2:
// the MO values, gradients and Laplacians are one matrix product of the
// concatenated AO array with the coefficient matrix).
//
// One strided, batched kernel serves the three products of the path:
//   forward   mo[p][c][n]   = sum_k ao[k][c][p] Ct[k][n]        (batch c)
//   Gbar      Gb[k][c][p]   = sum_n W[p][c][n]  C[n][k]         (batch c)
//   dC        ws[c,s][n][k] = sum_{p in split s} W[p][c][n] ao[k][c][p]
// (see GemmArgs for the index algebra).  Tiles are 128 x 128 with a K step
// of 16, four wavefronts in a 2 x 2 arrangement, each owning a 64 x 64
// sub-tile as 4 x 4 MFMA 16x16x4 blocks (FP64 or FP32).  Operand tiles go
// global -> registers -> LDS with one tile of prefetch (double-buffered
// LDS, one barrier per K step).  Tile order is XCD-aware: the eight
// consecutive workgroup ids land on the eight XCDs, so ids are remapped so
// that all N tiles of one M tile run on the same XCD back to back and the
// M-tile of A is fetched from HBM once per XCD L2.
#include "qmk_internal.h"

namespace qmk {
namespace {

template <typename T>
struct Mfma;

// Accumulator element r of lane l sits in column l % 16 and in row
//   FP64 16x16x4:  l / 16 + 4 r
//   FP32 16x16x4:  4 (l / 16) + r
// (measured lane layouts on gfx950).
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Tile coordinates of this workgroup; false if it has no tile.
__device__ __forceinline__ bool tile_of_block(int nM, int nN, int& mt, int& nt) {
  const int bid = blockIdx.x;
  if (nM >= 8) {
    const int x = bid & 7, j = bid >> 3;
    mt = (j / nN) * 8 + x;
    nt = j % nN;
    return mt < nM;
  }
  mt = bid / nN;
  nt = bid % nN;
  return mt < nM;
}

template <typename T, typename TA, typename TB, typename TD, int BM, int BN, int BK, bool A_I,
          bool B_J>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g, int nM, int nN) {
  constexpr int PAD = 16 / sizeof(T);
  constexpr int EA = BM * BK / 256, EB = BK * BN / 256;
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  typedef typename Mfma<T>::v4 v4;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  int mt, nt;
  if (!tile_of_block(nM, nN, mt, nt)) return;
  const int z = blockIdx.y;
  const int c = z / g.nsplit, s = z - c * g.nsplit;
  const TA* __restrict__ Ap = static_cast<const TA*>(g.A) + c * g.oAc + s * g.oAs;
  const TB* __restrict__ Bp = static_cast<const TB*>(g.B) + c * g.oBc + s * g.oBs;
  TD* __restrict__ Dp = static_cast<TD*>(g.D) + z * g.oDz;
  const int64_t Ls = min(g.Lchunk, g.L - s * g.Lchunk);
  const int64_t i0 = static_cast<int64_t>(mt) * BM, j0 = static_cast<int64_t>(nt) * BN;
  const int tid = threadIdx.x;

  T ra[EA], rb[EB];
  auto load = [&](int64_t l0) {
#pragma unroll
    for (int r = 0; r < EA; ++r) {
      const int e = tid + 256 * r;
      const int i = A_I ? e % BM : e / BK;
      const int l = A_I ? e / BM : e % BK;
      const int64_t gi = i0 + i, gl = l0 + l;
      ra[r] = (gi < g.M && gl < Ls) ? static_cast<T>(Ap[gi * g.sAi + gl * g.sAl]) : T(0);
    }
#pragma unroll
    for (int r = 0; r < EB; ++r) {
      const int e = tid + 256 * r;
      const int j = B_J ? e % BN : e / BK;
      const int l = B_J ? e / BN : e % BK;
      const int64_t gj = j0 + j, gl = l0 + l;
      rb[r] = (gj < g.N && gl < Ls) ? static_cast<T>(Bp[gl * g.sBl + gj * g.sBj]) : T(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < EA; ++r) {
      const int e = tid + 256 * r;
      const int i = A_I ? e % BM : e / BK;
      const int l = A_I ? e / BM : e % BK;
      As[buf][l][i] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < EB; ++r) {
      const int e = tid + 256 * r;
      const int j = B_J ? e % BN : e / BK;
      const int l = B_J ? e / BN : e % BK;
      Bs[buf][l][j] = rb[r];
    }
  };

  const int lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  v4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = v4{0, 0, 0, 0};

  const int64_t nk = (Ls + BK - 1) / BK;
  if (nk > 0) {
    load(0);
    stash(0);
  }
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = static_cast<int>(kt & 1);
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4), ci = lane & 15;
      T fa[TM], fb[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) fa[a] = As[buf][kr][wm * WM + a * 16 + ci];
#pragma unroll
      for (int b = 0; b < TN; ++b) fb[b] = Bs[buf][kr][wn * WN + b * 16 + ci];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<T>::op(fa[a], fb[b], acc[a][b]);
    }
    if (kt + 1 < nk) stash(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + wm * WM + a * 16 + Mfma<T>::row(lane, r);
        const int64_t gj = j0 + wn * WN + b * 16 + (lane & 15);
        if (gi < g.M && gj < g.N) Dp[gi * g.sDi + gj * g.sDj] = static_cast<TD>(acc[a][b][r]);
      }
}

__global__ void reduce_splits_kernel(const double* __restrict__ ws, int64_t nz, int64_t rows,
                                     int64_t cols, int64_t ld_ws, int64_t z_stride,
                                     double* __restrict__ out, int64_t ld_out) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols, c = e - r * cols;
  double acc = 0.0;
  for (int64_t z = 0; z < nz; ++z) acc += ws[z * z_stride + r * ld_ws + c];
  out[r * ld_out + c] = acc;
}

template <typename T, typename TA, typename TB, typename TD, bool A_I, bool B_J>
hipError_t run(const GemmArgs& g, hipStream_t s) {
  constexpr int BM = 128, BN = 128, BK = 16;
  const int nM = static_cast<int>((g.M + BM - 1) / BM), nN = static_cast<int>((g.N + BN - 1) / BN);
  if (nM <= 0 || nN <= 0) return hipSuccess;
  const int gx = nM >= 8 ? 8 * nN * ((nM + 7) / 8) : nM * nN;
  dim3 grid(gx, g.nbatch * g.nsplit);
  hipLaunchKernelGGL((gemm_kernel<T, TA, TB, TD, BM, BN, BK, A_I, B_J>), grid, dim3(256), 0, s, g,
                     nM, nN);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_typed(GemmKind kind, Prec prec, const GemmArgs& g, int w_is_f32,
                             int out_is_f32, hipStream_t s) {
  if (prec == Prec::kF64) {
    switch (kind) {
      case GemmKind::kForward:
        return out_is_f32 ? run<double, double, double, float, true, true>(g, s)
                          : run<double, double, double, double, true, true>(g, s);
      case GemmKind::kGbar:
        return w_is_f32 ? run<double, float, double, double, false, true>(g, s)
                        : run<double, double, double, double, false, true>(g, s);
      case GemmKind::kDcoef:
        return w_is_f32 ? run<double, float, double, double, true, false>(g, s)
                        : run<double, double, double, double, true, false>(g, s);
    }
  } else {
    switch (kind) {
      case GemmKind::kForward:
        return out_is_f32 ? run<float, float, float, float, true, true>(g, s)
                          : run<float, float, float, double, true, true>(g, s);
      case GemmKind::kGbar:
        return w_is_f32 ? run<float, float, float, float, false, true>(g, s)
                        : run<float, double, float, float, false, true>(g, s);
      case GemmKind::kDcoef:
        return w_is_f32 ? run<float, float, float, double, true, false>(g, s)
                        : run<float, double, float, double, true, false>(g, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_splits(const double* ws, int64_t nz, int64_t rows, int64_t cols,
                                int64_t ld_ws, int64_t z_stride, double* out, int64_t ld_out,
                                hipStream_t s) {
  const int64_t n = rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_splits_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256),
                     0, s, ws, nz, rows, cols, ld_ws, z_stride, out, ld_out);
  return hipGetLastError();
}

}  // namespace qmk
