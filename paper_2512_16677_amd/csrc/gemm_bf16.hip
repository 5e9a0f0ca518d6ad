// Three-product BF16-split contraction on MFMA (mixed precision mode).
//
// Every operand value x is split into bf16 parts hi = bf16(x) and
// lo = bf16(x - hi), and a product is formed from three BF16 MFMAs,
//   a b  ~  a_hi b_hi + a_hi b_lo + a_lo b_hi,
// accumulated in FP32 (the dropped a_lo b_lo term is ~2^-18 |a b|).  The
// two cross products are the correction of the leading BF16 product.
// The product indices follow the FP64/FP32 kernel (GemmArgs); the MFMA is
// v_mfma_f32_16x16x32_bf16, whose lanes hold eight consecutive reduction
// indices of one row of A and one column of B.  Operand tiles are staged in
// LDS k-contiguous per row ([row][k], hi and lo planes):
//   * an operand whose reduction index is contiguous in memory (W in the
//     W C product, the AO array in the W^T ao product, the pre-split C and
//     C^T) is read in runs of eight along k;
//   * an operand whose rows are contiguous (the AO array in the forward
//     product, W^T in the W^T ao product) is read as 2-row x 8-k
//     micro-tiles (coalesced along the rows) and transposed in registers
//     before the LDS store.
// Splitting happens on the way into LDS, so FP32 AOs and FP64/FP32 weights
// need no extra pass over HBM.
#include <type_traits>

#include "qmk_internal.h"

namespace qmk {

struct BfPersist {
  const GemmArgs* jobs;
  const WorkItem* items;
  int n_items, grid;
  int* occupancy;
};

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void split1(float x, __bf16& h, __bf16& l) {
  h = static_cast<__bf16>(x);
  l = static_cast<__bf16>(x - static_cast<float>(h));
}
// FP64 values are rounded to FP32 first (relative error 2^-24, far below
// the 2^-18 of the split), so the residual is an FP32 subtraction.
__device__ __forceinline__ void split1(double x, __bf16& h, __bf16& l) {
  split1(static_cast<float>(x), h, l);
}

// Source marker: values already split, hi plane at the operand pointer and
// lo plane at the second pointer (same layout).
struct PreSplit {};

// Eight consecutive reduction-index values of one row, split.
template <typename TS>
struct RunLoader;

template <>
struct RunLoader<float> {
  static __device__ __forceinline__ void fast(const float* p, const float*, bf16x8& h, bf16x8& l) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    const float4 b = *reinterpret_cast<const float4*>(p + 4);
    const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 hh, ll;
      split1(v[e], hh, ll);
      h[e] = hh;
      l[e] = ll;
    }
  }
  static __device__ __forceinline__ void one(const float* p, const float*, int64_t off, __bf16& h,
                                             __bf16& l) {
    split1(p[off], h, l);
  }
};

template <>
struct RunLoader<double> {
  static __device__ __forceinline__ void fast(const double* p, const double*, bf16x8& h, bf16x8& l) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double2 v = *reinterpret_cast<const double2*>(p + 2 * q);
      __bf16 hh, ll;
      split1(v.x, hh, ll);
      h[2 * q] = hh;
      l[2 * q] = ll;
      split1(v.y, hh, ll);
      h[2 * q + 1] = hh;
      l[2 * q + 1] = ll;
    }
  }
  static __device__ __forceinline__ void one(const double* p, const double*, int64_t off, __bf16& h,
                                             __bf16& l) {
    split1(p[off], h, l);
  }
};

template <>
struct RunLoader<PreSplit> {
  static __device__ __forceinline__ void fast(const PreSplit* p, const PreSplit* p2, bf16x8& h,
                                              bf16x8& l) {
    h = *reinterpret_cast<const bf16x8*>(p);
    l = *reinterpret_cast<const bf16x8*>(p2);
  }
  static __device__ __forceinline__ void one(const PreSplit* p, const PreSplit* p2, int64_t off,
                                             __bf16& h, __bf16& l) {
    h = reinterpret_cast<const __bf16*>(p)[off];
    l = reinterpret_cast<const __bf16*>(p2)[off];
  }
};

// Pointer arithmetic in elements of the stored type (bf16 for PreSplit).
template <typename TS>
__device__ __forceinline__ const TS* adv(const TS* p, int64_t n) { return p + n; }
template <>
__device__ __forceinline__ const PreSplit* adv(const PreSplit* p, int64_t n) {
  return reinterpret_cast<const PreSplit*>(reinterpret_cast<const __bf16*>(p) + n);
}

template <typename TS>
__device__ __forceinline__ void pair_load(const TS* p, TS& a, TS& b) {
  if constexpr (sizeof(TS) == 4) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    a = v.x;
    b = v.y;
  } else {
    const double2 v = *reinterpret_cast<const double2*>(p);
    a = v.x;
    b = v.y;
  }
}

// Loads one operand tile of ROWS rows x 32 reduction indices into
// registers (raw values; the loads stay in flight during the MFMAs of the
// current tile) and later splits them into hi/lo and writes them to LDS as
// [row][k].
//   KC: reduction index contiguous (runs of 8 along k), else rows
//   contiguous (2-row x 8-k micro-tiles, transposed in registers).
// Element (row, l) of the operand is at base[row * s_row + l * s_l].
template <typename TS, bool KC, int ROWS, int NT, int BK>
struct TileLoader {
  static constexpr int LDK = BK + 8;
  static constexpr int UNITS = KC ? ROWS * (BK / 8) : (ROWS / 2) * (BK / 8);
  static constexpr int PER = (UNITS + NT - 1) / NT;
  static constexpr bool PRE = std::is_same<TS, PreSplit>::value;
  typedef typename std::conditional<PRE, float, TS>::type Raw;  // unused for PRE
  static constexpr int NRAW = PRE ? 1 : (KC ? 8 : 16);
  Raw raw[PER][NRAW];
  bf16x8 ph[PER], pl[PER];  // PRE only

  __device__ __forceinline__ void load(const TS* base, const TS* base2, int64_t s_row, int64_t s_l,
                                       int64_t rows_left, int64_t l_left, bool fast, int tid) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = tid + NT * u;
      if (UNITS % NT != 0 && q >= UNITS) continue;
      if constexpr (KC) {
        const int row = q / (BK / 8), kg = q % (BK / 8);
        if constexpr (PRE) {
          if (fast) {
            const int64_t off = row * s_row + kg * 8;
            ph[u] = *reinterpret_cast<const bf16x8*>(adv(base, off));
            pl[u] = *reinterpret_cast<const bf16x8*>(adv(base2, off));
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              __bf16 hh = static_cast<__bf16>(0.0f), ll = static_cast<__bf16>(0.0f);
              if (row < rows_left && kg * 8 + e < l_left)
                RunLoader<TS>::one(base, base2, row * s_row + (kg * 8 + e) * s_l, hh, ll);
              ph[u][e] = hh;
              pl[u][e] = ll;
            }
          }
        } else if (fast) {
          const TS* p = base + row * s_row + kg * 8;
          if constexpr (sizeof(TS) == 4) {
            const float4 a = *reinterpret_cast<const float4*>(p);
            const float4 b = *reinterpret_cast<const float4*>(p + 4);
            raw[u][0] = a.x; raw[u][1] = a.y; raw[u][2] = a.z; raw[u][3] = a.w;
            raw[u][4] = b.x; raw[u][5] = b.y; raw[u][6] = b.z; raw[u][7] = b.w;
          } else {
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
              const double2 v = *reinterpret_cast<const double2*>(p + 2 * qq);
              raw[u][2 * qq] = v.x;
              raw[u][2 * qq + 1] = v.y;
            }
          }
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e)
            raw[u][e] = (row < rows_left && kg * 8 + e < l_left)
                            ? base[row * s_row + (kg * 8 + e) * s_l] : TS(0);
        }
      } else {
        const int rp = q % (ROWS / 2), kg = q / (ROWS / 2);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t lidx = kg * 8 + e;
          TS a = TS(0), b = TS(0);
          if (fast) {
            pair_load(base + 2 * rp + lidx * s_l, a, b);
          } else if (lidx < l_left) {
            if (2 * rp < rows_left) a = base[2 * rp + lidx * s_l];
            if (2 * rp + 1 < rows_left) b = base[2 * rp + 1 + lidx * s_l];
          }
          raw[u][e] = a;
          raw[u][8 + e] = b;
        }
      }
    }
  }

  __device__ __forceinline__ void stash(__bf16* hi, __bf16* lo, int tid) const {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int q = tid + NT * u;
      if (UNITS % NT != 0 && q >= UNITS) continue;
      if constexpr (KC) {
        const int row = q / (BK / 8), kg = q % (BK / 8);
        bf16x8 h, l;
        if constexpr (PRE) {
          h = ph[u];
          l = pl[u];
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 hh, ll;
            split1(raw[u][e], hh, ll);
            h[e] = hh;
            l[e] = ll;
          }
        }
        *reinterpret_cast<bf16x8*>(hi + row * LDK + kg * 8) = h;
        *reinterpret_cast<bf16x8*>(lo + row * LDK + kg * 8) = l;
      } else {
        const int rp = q % (ROWS / 2), kg = q / (ROWS / 2);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          bf16x8 h, l;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 hh, ll;
            split1(raw[u][8 * v + e], hh, ll);
            h[e] = hh;
            l[e] = ll;
          }
          *reinterpret_cast<bf16x8*>(hi + (2 * rp + v) * LDK + kg * 8) = h;
          *reinterpret_cast<bf16x8*>(lo + (2 * rp + v) * LDK + kg * 8) = l;
        }
      }
    }
  }
};

template <int BM, int BN, int BK>
struct BfSmem {
  static constexpr int LDK = BK + 8;
  __bf16 A[2][2][BM * LDK];  // [buffer][hi, lo][row * LDK + k]
  __bf16 B[2][2][BN * LDK];
};

template <typename TA, bool A_KC, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK>
__device__ __forceinline__ void bf16x3_body(const GemmArgs& g, int mt, int nt, int z,
                                            BfSmem<16 * WGM * TM, 16 * WGN * TN, BK>& sm) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN, LDK = BK + 8;
  auto& sA = sm.A;
  auto& sB = sm.B;
  const int c = z / g.nsplit, s = z - c * g.nsplit;
  const TA* Ap = adv(static_cast<const TA*>(g.A), c * g.oAc + s * g.oAs);
  const TA* Ap2 = g.A2 ? adv(static_cast<const TA*>(g.A2), c * g.oAc + s * g.oAs) : Ap;
  const TB* Bp = adv(static_cast<const TB*>(g.B), c * g.oBc + s * g.oBs);
  const TB* Bp2 = g.B2 ? adv(static_cast<const TB*>(g.B2), c * g.oBc + s * g.oBs) : Bp;
  TD* __restrict__ Dp = static_cast<TD*>(g.D) + z * g.oDz;
  const int64_t Ls = min(g.Lchunk, g.L - s * g.Lchunk);
  const int64_t i0 = static_cast<int64_t>(mt) * BM, j0 = static_cast<int64_t>(nt) * BN;
  const int tid = threadIdx.x;
  const bool a_vec = (g.vec_ok & 1) != 0, b_vec = (g.vec_ok & 2) != 0;

  // A rows are i (stride sAi), reduction l (stride sAl); B rows are j
  // (stride sBj), reduction l (stride sBl = 1).
  TileLoader<TA, A_KC, BM, NT, BK> la;
  TileLoader<TB, true, BN, NT, BK> lb;
  auto load = [&](int64_t l0) {
    const int64_t rows_a = g.M - i0, rows_b = g.N - j0, lleft = Ls - l0;
    const bool a_fast = a_vec && rows_a >= BM && lleft >= BK;
    const bool b_fast = b_vec && rows_b >= BN && lleft >= BK;
    la.load(adv(Ap, i0 * g.sAi + l0 * g.sAl), adv(Ap2, i0 * g.sAi + l0 * g.sAl), g.sAi, g.sAl,
            rows_a, lleft, a_fast, tid);
    lb.load(adv(Bp, l0 * g.sBl + j0 * g.sBj), adv(Bp2, l0 * g.sBl + j0 * g.sBj), g.sBj, g.sBl,
            rows_b, lleft, b_fast, tid);
  };

  const int lane = tid & 63, w = tid >> 6;
  const int wm = w / WGN, wn = w % WGN;
  f32x4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int64_t nk = (Ls + BK - 1) / BK;
  if (nk > 0) {
    load(0);
    la.stash(sA[0][0], sA[0][1], tid);
    lb.stash(sB[0][0], sB[0][1], tid);
  }
  __syncthreads();
  const int ri = lane & 15, kq = (lane >> 4) * 8;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = static_cast<int>(kt & 1);
    if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 32; ++kk) {
      bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        const int off = ((wm * TM + a) * 16 + ri) * LDK + kk * 32 + kq;
        ah[a] = *reinterpret_cast<const bf16x8*>(&sA[buf][0][off]);
        al[a] = *reinterpret_cast<const bf16x8*>(&sA[buf][1][off]);
      }
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int off = ((wn * TN + b) * 16 + ri) * LDK + kk * 32 + kq;
        bh[b] = *reinterpret_cast<const bf16x8*>(&sB[buf][0][off]);
        bl[b] = *reinterpret_cast<const bf16x8*>(&sB[buf][1][off]);
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) {
      la.stash(sA[buf ^ 1][0], sA[buf ^ 1][1], tid);
      lb.stash(sB[buf ^ 1][0], sB[buf ^ 1][1], tid);
    }
    __syncthreads();
  }

  // accumulator element r of lane l: row 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + (wm * TM + a) * 16 + 4 * (lane >> 4) + r;
        const int64_t gj = j0 + (wn * TN + b) * 16 + (lane & 15);
        if (gi < g.M && gj < g.N) Dp[gi * g.sDi + gj * g.sDj] = static_cast<TD>(acc[a][b][r]);
      }
}

template <typename TA, bool A_KC, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_bf16x3_kernel(GemmArgs g, int nM, int nN) {
  __shared__ __align__(16) BfSmem<16 * WGM * TM, 16 * WGN * TN, BK> sm;
  int mt, nt, z;
  if (!grid_tile(g, nM, nN, blockIdx.x, mt, nt, z)) return;
  bf16x3_body<TA, A_KC, TB, TD, WGM, WGN, TM, TN, BK>(g, mt, nt, z, sm);
}

template <typename TA, bool A_KC, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_bf16x3_persist(
    const GemmArgs* __restrict__ jobs, const WorkItem* __restrict__ items, int n_items) {
  __shared__ __align__(16) BfSmem<16 * WGM * TM, 16 * WGN * TN, BK> sm;
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const WorkItem it = items[i];
    bf16x3_body<TA, A_KC, TB, TD, WGM, WGN, TM, TN, BK>(jobs[it.job], it.a, it.b, it.c, sm);
    __syncthreads();
  }
}

// {WGM, WGN, TM, TN, BK}
#define QMK_BF16_TILE_LIST(X) \
  X(0, 2, 2, 4, 4, 32)        \
  X(1, 4, 1, 4, 5, 32)        \
  X(2, 2, 2, 4, 5, 32)        \
  X(3, 2, 2, 2, 4, 32)        \
  X(4, 1, 2, 5, 5, 32)        \
  X(5, 2, 2, 2, 5, 32)        \
  X(6, 2, 2, 4, 2, 32)        \
  X(7, 2, 2, 4, 3, 32)        \
  X(8, 2, 1, 5, 5, 32)        \
  X(9, 4, 1, 2, 5, 32)        \
  X(10, 2, 2, 4, 4, 64)       \
  X(11, 4, 1, 2, 5, 64)       \
  X(12, 2, 2, 2, 4, 64)       \
  X(13, 2, 1, 4, 5, 64)       \
  X(14, 2, 2, 4, 2, 64)

constexpr TileCfg kBfTiles[] = {
#define QMK_BF_ENTRY(id, wgm, wgn, tm, tn, bk) {wgm, wgn, tm, tn, bk},
    QMK_BF16_TILE_LIST(QMK_BF_ENTRY)
#undef QMK_BF_ENTRY
};

template <typename TA, bool A_KC, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK>
hipError_t run_bf_tile(const GemmArgs& g, hipStream_t s) {
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN;
  const int nM = static_cast<int>((g.M + BM - 1) / BM), nN = static_cast<int>((g.N + BN - 1) / BN);
  if (nM <= 0 || nN <= 0) return hipSuccess;
  const dim3 grid = grid_of(g, nM, nN);
  hipLaunchKernelGGL((gemm_bf16x3_kernel<TA, A_KC, TB, TD, WGM, WGN, TM, TN, BK>), grid,
                     dim3(64 * WGM * WGN), 0, s, g, nM, nN);
  return hipGetLastError();
}

template <typename TA, bool A_KC, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK>
hipError_t run_bf_tile_persist(const BfPersist& pl, hipStream_t s) {
  auto k = gemm_bf16x3_persist<TA, A_KC, TB, TD, WGM, WGN, TM, TN, BK>;
  if (pl.occupancy) {
    int n = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * WGM * WGN, 0);
    *pl.occupancy = (e == hipSuccess && n > 0) ? n : 1;
    return e;
  }
  if (pl.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3(pl.grid), dim3(64 * WGM * WGN), 0, s, pl.jobs, pl.items, pl.n_items);
  return hipGetLastError();
}

template <typename TA, bool A_KC, typename TB, typename TD>
hipError_t run_bf_persist(int cfg, const BfPersist& pl, hipStream_t s) {
  switch (cfg) {
#define QMK_BF_PCASE(id, wgm, wgn, tm, tn, bk) \
  case id:                                     \
    return run_bf_tile_persist<TA, A_KC, TB, TD, wgm, wgn, tm, tn, bk>(pl, s);
    QMK_BF16_TILE_LIST(QMK_BF_PCASE)
#undef QMK_BF_PCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename TA, bool A_KC, typename TB, typename TD>
hipError_t run_bf(int cfg, const GemmArgs& g, hipStream_t s) {
  switch (cfg) {
#define QMK_BF_CASE(id, wgm, wgn, tm, tn, bk) \
  case id:                                    \
    return run_bf_tile<TA, A_KC, TB, TD, wgm, wgn, tm, tn, bk>(g, s);
    QMK_BF16_TILE_LIST(QMK_BF_CASE)
#undef QMK_BF_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

#ifdef QMK_GEMM_UNIT
#if QMK_GEMM_UNIT == 1
hipError_t bf16_unit_fwd(int cfg, const GemmArgs* g, const BfPersist* pl, int w32, int o32,
                          hipStream_t s) {
  const bool alt = o32 != 0;
  if (pl) return alt ? run_bf_persist<float, false, PreSplit, float>(cfg, *pl, s) : run_bf_persist<float, false, PreSplit, double>(cfg, *pl, s);
  return alt ? run_bf<float, false, PreSplit, float>(cfg, *g, s) : run_bf<float, false, PreSplit, double>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 2
hipError_t bf16_unit_gbar(int cfg, const GemmArgs* g, const BfPersist* pl, int w32, int o32,
                          hipStream_t s) {
  const bool alt = w32 != 0;
  if (pl) return alt ? run_bf_persist<PreSplit, true, float, float>(cfg, *pl, s) : run_bf_persist<PreSplit, true, double, float>(cfg, *pl, s);
  return alt ? run_bf<PreSplit, true, float, float>(cfg, *g, s) : run_bf<PreSplit, true, double, float>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 3
hipError_t bf16_unit_dc(int cfg, const GemmArgs* g, const BfPersist* pl, int w32, int o32,
                          hipStream_t s) {
  const bool alt = w32 != 0;
  if (pl) return alt ? run_bf_persist<float, false, float, double>(cfg, *pl, s) : run_bf_persist<double, false, float, double>(cfg, *pl, s);
  return alt ? run_bf<float, false, float, double>(cfg, *g, s) : run_bf<double, false, float, double>(cfg, *g, s);
}
#endif
#else
// The three products are instantiated in their own translation units (this
// file compiled with QMK_GEMM_UNIT = 1..3); the unit without it holds the
// tile table and the dispatch.
hipError_t bf16_unit_fwd(int cfg, const GemmArgs* g, const BfPersist* pl, int w32, int o32,
                          hipStream_t s);
hipError_t bf16_unit_gbar(int cfg, const GemmArgs* g, const BfPersist* pl, int w32, int o32,
                          hipStream_t s);
hipError_t bf16_unit_dc(int cfg, const GemmArgs* g, const BfPersist* pl, int w32, int o32,
                          hipStream_t s);

int gemm_bf16_num_tiles() { return sizeof(kBfTiles) / sizeof(kBfTiles[0]); }
TileCfg gemm_bf16_tile(int cfg) { return kBfTiles[cfg]; }
size_t gemm_bf16_tile_lds_bytes(int cfg) {
  const TileCfg& t = kBfTiles[cfg];
  return 2 * 2 * static_cast<size_t>(16 * t.wgm * t.tm + 16 * t.wgn * t.tn) * (t.bk + 8) * 2;
}

// forward: A = AO array (FP32, rows contiguous), B = C split (k contiguous)
// Gbar:    A = C^T split (k contiguous),         B = W (k contiguous)
// dC:      A = W^T (rows contiguous),            B = AO array (k contiguous)
namespace {
hipError_t bf16_dispatch(GemmKind kind, int cfg, const GemmArgs* g, const BfPersist* pl, int w32,
                         int o32, hipStream_t s) {
  if (cfg < 0 || cfg >= gemm_bf16_num_tiles()) return hipErrorInvalidValue;
  switch (kind) {
    case GemmKind::kForward: return bf16_unit_fwd(cfg, g, pl, w32, o32, s);
    case GemmKind::kGbar: return bf16_unit_gbar(cfg, g, pl, w32, o32, s);
    case GemmKind::kDcoef: return bf16_unit_dc(cfg, g, pl, w32, o32, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_gemm_bf16x3(GemmKind kind, int cfg, const GemmArgs& g, int w_is_f32,
                              int out_is_f32, hipStream_t s) {
  return bf16_dispatch(kind, cfg, &g, nullptr, w_is_f32, out_is_f32, s);
}

hipError_t launch_gemm_bf16x3_persist(GemmKind kind, int cfg, const GemmArgs* jobs,
                                      const WorkItem* items, int n_items, int grid, int w_is_f32,
                                      int out_is_f32, int* occupancy, hipStream_t s) {
  const BfPersist pl{jobs, items, n_items, grid, occupancy};
  return bf16_dispatch(kind, cfg, nullptr, &pl, w_is_f32, out_is_f32, s);
}

#endif  // QMK_GEMM_UNIT

}  // namespace qmk
