// Templates of the FP64 / FP32 MFMA product (shared by the translation units
// that instantiate them; see gemm_kernels.hip).
#pragma once

#include <type_traits>

#include "qmk_internal.h"

namespace qmk {

struct PersistLaunch {
  const GemmArgs* jobs;
  const WorkItem* items;
  int n_items, grid;
  int* occupancy;  // when non-NULL: report resident blocks per CU instead of launching
};

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

// Tile: WGM x WGN wavefronts, each owning TM x TN MFMA blocks of 16 x 16,
// so the workgroup tile is BM = 16 WGM TM rows by BN = 16 WGN TN columns,
// with a reduction step of BK.
template <typename T, int BM, int BN, int BK>
struct alignas(16) GemmSmem {
  static constexpr int PAD = 16 / sizeof(T);
  T A[2][BK][BM + PAD];
  T B[2][BK][BN + PAD];
};

// ---------------------------------------------------------------------------
// K loop with direct global -> LDS loads (FP64 and FP32 operands;
// global_load_lds_dwordx4: 16 bytes per lane, one 1 KB block per wave and
// instruction, written at the wave-uniform LDS address in M0 plus 16 lane).
// The operand tiles never pass through registers, so the register staging of
// the generic loop, its LDS stores and their address arithmetic go away.  Two
// stages: the loads of K step k + 1 run under the products of step k.
//
// Stage layout in LDS (no padding: the loads fill whole 1 KB blocks; E = 2
// doubles or 4 floats per 16 bytes):
//   A, i contiguous:  [BK][BM]  element (l, i) at l BM + (i ^ dma_xr<T, BM>(l))
//   B, j contiguous:  [BK][BN]  element (l, j) at l BN + (j ^ dma_xr<T, BN>(l))
//   B, l contiguous:  [BN][BK]  element (l, j) at j BK + E ((l/E) ^ dma_kx<T, BK>(j)) + l % E
// (BK = 16 or 32).  One fragment read (64 lanes; lane l reads column l % 16
// of row l / 16 of a 16-wide block) is served in two halves of 256 bytes for
// FP64 and in one for FP32.  dma_xr permutes the 16-element blocks of a row
// (by XOR) so that the rows one such half touches fall on different banks;
// dma_kx permutes the 16-byte slots of an l-contiguous row so that the 16 rows
// a fragment read touches spread over all banks.
//
// Rows past the end of the matrix read a copy of the last 16 bytes that hold
// an in-range element (or of the last row); their products land in outputs
// that are never stored.  A partial
// last K step (the K extent not a multiple of BK) is staged through
// registers instead, with zeros beyond the extent.
template <typename T, int R>
__device__ __forceinline__ int dma_xr(int l) {
  if constexpr (sizeof(T) == 8) return R % 32 == 0 ? (l & 1) << 4 : 0;
  return R % 64 == 0 ? (l & 3) << 4 : (R % 64 == 32 ? ((l >> 1) & 1) << 4 : 0);
}

template <typename T, int BK>
__device__ __forceinline__ int dma_kx(int j) {
  if constexpr (sizeof(T) == 8) return BK == 16 ? (j >> 1) & 7 : j & 15;
  return BK == 16 ? (j >> 2) & 3 : (j >> 1) & 7;
}

__device__ __forceinline__ uint32_t dma_lds_address(const void* p) {
  return static_cast<uint32_t>(
      reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) char*)(p)));
}

// Lane l's 16 bytes at g land at LDS byte lds + 16 l.  The compiler does not
// see these LDS writes: dma_sync waits for them.
__device__ __forceinline__ void dma_b128(const void* g, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" : : "s"(lds), "v"(g)
               : "memory", "m0");
}

// Waits for this wave's loads and LDS reads, then joins the workgroup
// barrier; the memory clobber keeps LDS reads from moving across it.
__device__ __forceinline__ void dma_sync() {
  asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" : : : "memory");
}

// Whether this tile may take the direct-load loop: unit stride along i (A)
// and along j or l (B), 16-byte aligned operands, strides that are multiples
// of E = 16 / sizeof(T) (every 16-byte slot starts aligned), and a row (and,
// for j-contiguous B, column) count that is a multiple of E or padded
// (GemmArgs::pad_ok), so that the last slot is in range.
template <typename T, int BK, bool B_J>
__device__ __forceinline__ bool dma_tile_ok(const GemmArgs& g, const void* Ap, const void* Bp) {
  constexpr int64_t E = 16 / sizeof(T);
  if ((BK != 16 && BK != 32) || g.sAi != 1 || g.sAl % E != 0 || (g.M % E != 0 && !(g.pad_ok & 1))) return false;
  if (B_J ? (g.sBj != 1 || g.sBl % E != 0 || (g.N % E != 0 && !(g.pad_ok & 2)))
          : (g.sBl != 1 || g.sBj % E != 0))
    return false;
  return ((reinterpret_cast<uintptr_t>(Ap) | reinterpret_cast<uintptr_t>(Bp)) & 15) == 0;
}

// K loop of one tile: At / Bt point at the tile's first row / column,
// rows_a = M - i0 and rows_b = N - j0 (slots past them are clamped to the
// last slot that holds an in-range element).  The K steps visited are first,
// next(first), next(next(first)), ... up to the first one >= end, in
// increasing order (the caller's next() returns the following step to visit,
// wave-uniform).  Step `part`, when visited, is the last one and holds only
// tail < BK values of l.  The caller synchronises the workgroup before the LDS
// is written again after the loop.
template <typename T, int BK, bool B_J, int WGM, int WGN, int TM, int TN, class Next>
__device__ __forceinline__ void dma_loop(T* stages, const T* At, const T* Bt, int64_t sAl, int64_t sBl,
                                         int64_t sBj, int64_t rows_a, int64_t rows_b, int64_t first,
                                         int64_t end, int64_t part, int tail, Next next,
                                         typename Mfma<T>::v4 (&acc)[TM][TN]) {
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN, NW = WGM * WGN;
  constexpr int E = 16 / sizeof(T), SZ = sizeof(T);
  static_assert(BK == 16 || BK == 32, "K step");
  constexpr int NIA = BM * BK * SZ / 1024, NI = (BM + BN) * BK * SZ / 1024;  // 1 KB blocks per stage (A first)
  static_assert(NIA * 1024 == BM * BK * SZ && NI * 1024 == (BM + BN) * BK * SZ, "whole 1 KB blocks");
  constexpr int IPW = (NI + NW - 1) / NW;
  constexpr int STAGE = (BM + BN) * BK;  // elements
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WGN, wn = w % WGN;
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const uint32_t lds0 = __builtin_amdgcn_readfirstlane(dma_lds_address(stages));

  // per instruction: this lane's source in step 0, whether it loads A (the
  // bytes a K step moves it are stepA, else stepB), and the LDS offset of its
  // block within a stage.  A wave short of blocks repeats one (the same bytes
  // written twice).
  const char* gp[IPW];
  bool isa[IPW];
  uint32_t ldso[IPW];
  const int64_t stepA = static_cast<int64_t>(BK) * sAl * SZ;
  const int64_t stepB = static_cast<int64_t>(BK) * (B_J ? sBl : 1) * SZ;
#pragma unroll
  for (int q = 0; q < IPW; ++q) {
    int ig = wu + NW * q;
    if (NI % NW != 0 && ig >= NI) ig -= NI;
    ldso[q] = static_cast<uint32_t>(ig) * 1024u;
    const T* src;
    if (ig < NIA) {
      const int sl = 64 * ig + lane, l = sl / (BM / E);
      const int i = (E * (sl % (BM / E))) ^ dma_xr<T, BM>(l);
      src = At + (i < rows_a ? i : (rows_a - 1) & ~int64_t(E - 1)) + l * sAl;
    } else if constexpr (B_J) {
      const int sl = 64 * (ig - NIA) + lane, l = sl / (BN / E);
      const int j = (E * (sl % (BN / E))) ^ dma_xr<T, BN>(l);
      src = Bt + (j < rows_b ? j : (rows_b - 1) & ~int64_t(E - 1)) + l * sBl;
    } else {
      const int sl = 64 * (ig - NIA) + lane, j = sl / (BK / E);
      const int l = E * ((sl % (BK / E)) ^ dma_kx<T, BK>(j));
      src = Bt + (j < rows_b ? j : rows_b - 1) * sBj + l;
    }
    gp[q] = reinterpret_cast<const char*>(src);
    isa[q] = ig < NIA;
  }
  auto issue = [&](int slot, int64_t kt) {
    // two wave-uniform offsets per step, one for each operand
    const int64_t t = __builtin_amdgcn_readfirstlane(static_cast<int>(kt));
    int64_t oa = t * stepA, ob = t * stepB;
    // opaque to the compiler, which would otherwise fold the select below into
    // one 64-bit multiply per instruction
    asm("" : "+s"(oa), "+s"(ob));
    const uint32_t sb = lds0 + static_cast<uint32_t>(slot * STAGE * SZ);
#pragma unroll
    for (int q = 0; q < IPW; ++q) dma_b128(gp[q] + (isa[q] ? oa : ob), sb + ldso[q]);
  };
  // fragments of sub-step kk + 1 are read before the products of kk
  auto compute = [&](const T* sa) {
    const T* sb = sa + BM * BK;
    const int ci = lane & 15, kq = lane >> 4;
    T fa[2][TM], fb[2][TN];
    auto rd = [&](int kk, int u) {
      const int k = kk * 4 + kq;
#pragma unroll
      for (int a = 0; a < TM; ++a) fa[u][a] = sa[k * BM + (((wm * TM + a) * 16 + ci) ^ dma_xr<T, BM>(k))];
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        const int j = (wn * TN + b) * 16 + ci;
        fb[u][b] = B_J ? sb[k * BN + (j ^ dma_xr<T, BN>(k))]
                       : sb[j * BK + (((k / E) ^ dma_kx<T, BK>(ci)) * E + k % E)];
      }
    };
    rd(0, 0);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      if (kk + 1 < BK / 4) rd(kk + 1, (kk + 1) & 1);
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<T>::op(fa[kk & 1][a], fb[kk & 1][b], acc[a][b]);
    }
  };

  // the partial last step, through registers with zeros beyond l < tail and
  // beyond the last row / column
  auto stage_tail = [&](T* st, int64_t t) {
    constexpr int NT = 64 * NW;
    const int64_t l0 = t * BK;
    for (int e = tid; e < BM * BK; e += NT) {
      const int l = e / BM, i = e % BM;
      st[l * BM + (i ^ dma_xr<T, BM>(l))] = l < tail && i < rows_a ? At[i + (l0 + l) * sAl] : T(0);
    }
    T* sb = st + BM * BK;
    for (int e = tid; e < BN * BK; e += NT) {
      if constexpr (B_J) {
        const int l = e / BN, j = e % BN;
        sb[l * BN + (j ^ dma_xr<T, BN>(l))] = l < tail && j < rows_b ? Bt[j + (l0 + l) * sBl] : T(0);
      } else {
        const int j = e / BK, l = e % BK;
        sb[j * BK + (((l / E) ^ dma_kx<T, BK>(j)) * E + l % E)] = l < tail && j < rows_b ? Bt[j * sBj + l0 + l] : T(0);
      }
    }
  };

  int64_t cur = first;
  if (cur >= end) return;
  // nxt: the step after cur, found one step ahead of its use
  int64_t nxt = cur == part ? end : next(cur);
  int slot = 0;
  if (cur != part) issue(0, cur);
  while (cur < end && cur != part) {
    // step cur has landed; the stage read in the step before it is free
    dma_sync();
    int64_t after = end;
    if (nxt < end && nxt != part) {
      issue(slot ^ 1, nxt);
      after = next(nxt);
    }
    compute(stages + slot * STAGE);
    cur = nxt;
    nxt = after;
    slot ^= 1;
  }
  if (cur < end) {
    // the partial step, into the stage last read two steps earlier (before
    // every wave passed the barrier of the step in between)
    T* st = stages + slot * STAGE;
    stage_tail(st, cur);
    __syncthreads();
    compute(st);
  }
}

// One output tile (mt, nt) of batch index z.  EPI = 0 stores D; EPI = 1 is
// the density epilogue: each wave reduces occ[j] * D(i, j)^2 over its own
// columns and stores the partial sum of row i in slot nt * WGN + wn, at
// D[i*sDi + slot*sDj] (FP64).
// EPI = 2 is the screened forward product: the K loop visits only the
// stages listed in stage_list (the rest of A is zero for every row of the
// tile), and row i of D is stored at row perm[i].
// EPI = 3 is the screened G-bar product (rows: AOs, columns: sorted points;
// W already in sorted point order): a tile whose AO chunks are inactive for
// all of its point blocks is stored as zeros without running the K loop.
// EPI = 5 is the three-body Jastrow product (FP64, batch z = (walker, k)):
// B holds rescaled distances and split s = k stages their k-th power; there
// is no output matrix: each wave weighs its outputs by the row's polynomial
// in x (GemmArgs::jx, jq), sums them and stores the sum in slot
// (mt WGM + wm) nNw + nt WGN + wn of batch z, nNw = (N tiles) WGN.
// EPI = 4 is the screened dC product (K runs over sorted points): the K
// stages whose 64-point block has no active chunk among the tile's N
// columns are skipped.
template <typename T, typename TA, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK, bool A_I, bool B_J, int EPI = 0>
__device__ __forceinline__ void gemm_body(const GemmArgs& g, int mt, int nt, int z,
                                          GemmSmem<T, 16 * WGM * TM, 16 * WGN * TN, BK>& sm,
                                          const int16_t* stage_list = nullptr, int n_stages = 0) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN;
  constexpr int EA = (BM * BK + NT - 1) / NT, EB = (BK * BN + NT - 1) / NT;
  // FP64 / FP32 products with i-contiguous A and unconverted operands may
  // take the direct-load K loop
  constexpr bool kDirect = (std::is_same<T, double>::value || std::is_same<T, float>::value) &&
                           std::is_same<TA, T>::value && std::is_same<TB, T>::value && (BK == 16 || BK == 32) &&
                           A_I && EPI != 5;
  typedef typename Mfma<T>::v4 v4;
  auto& As = sm.A;
  auto& Bs = sm.B;
  const int c = z / g.nsplit, s = z - c * g.nsplit;
  const TA* __restrict__ Ap = static_cast<const TA*>(g.A) + c * g.oAc + s * g.oAs;
  const TB* __restrict__ Bp = static_cast<const TB*>(g.B) + c * g.oBc + s * g.oBs;
  TD* __restrict__ Dp = static_cast<TD*>(g.D) + z * g.oDz;
  const int64_t Ls = min(g.Lchunk, g.L - s * g.Lchunk);
  const int64_t i0 = static_cast<int64_t>(mt) * BM, j0 = static_cast<int64_t>(nt) * BN;
  const int tid = threadIdx.x;

  T ra[EA], rb[EB];
  // Operand tiles fully inside the matrices take an unguarded path (uniform
  // branch per K step); only edge tiles test every element.
  const bool a_rows_in = i0 + BM <= g.M, b_cols_in = j0 + BN <= g.N;
  // In the instantiations that also hold the direct-load loop, this loop
  // recomputes its per-thread element indices at every K step (the thread
  // index is opaque to the compiler here), so that they are not kept in
  // registers across the whole kernel.
  auto load = [&](int64_t l0) {
    int tid = threadIdx.x;
    if constexpr (kDirect) asm volatile("" : "+v"(tid));
    const bool l_in = l0 + BK <= Ls;
    if (a_rows_in && l_in && BM * BK % NT == 0) {
      const TA* base = Ap + i0 * g.sAi + l0 * g.sAl;
#pragma unroll
      for (int r = 0; r < EA; ++r) {
        const int e = tid + NT * r;
        const int i = A_I ? e % BM : e / BK;
        const int l = A_I ? e / BM : e % BK;
        ra[r] = static_cast<T>(base[i * g.sAi + l * g.sAl]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < EA; ++r) {
        const int e = tid + NT * r;
        const int i = A_I ? e % BM : e / BK;
        const int l = A_I ? e / BM : e % BK;
        const int64_t gi = i0 + i, gl = l0 + l;
        const bool in = (BM * BK % NT == 0 || e < BM * BK) && gi < g.M && gl < Ls;
        ra[r] = in ? static_cast<T>(Ap[gi * g.sAi + gl * g.sAl]) : T(0);
      }
    }
    if (b_cols_in && l_in && BK * BN % NT == 0) {
      const TB* base = Bp + l0 * g.sBl + j0 * g.sBj;
#pragma unroll
      for (int r = 0; r < EB; ++r) {
        const int e = tid + NT * r;
        const int j = B_J ? e % BN : e / BK;
        const int l = B_J ? e / BN : e % BK;
        rb[r] = static_cast<T>(base[l * g.sBl + j * g.sBj]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < EB; ++r) {
        const int e = tid + NT * r;
        const int j = B_J ? e % BN : e / BK;
        const int l = B_J ? e / BN : e % BK;
        const int64_t gj = j0 + j, gl = l0 + l;
        const bool in = (BK * BN % NT == 0 || e < BK * BN) && gj < g.N && gl < Ls;
        rb[r] = in ? static_cast<T>(Bp[gl * g.sBl + gj * g.sBj]) : T(0);
      }
    }
  };
  auto stash = [&](int buf) {
    int tid = threadIdx.x;
    if constexpr (kDirect) asm volatile("" : "+v"(tid));
#pragma unroll
    for (int r = 0; r < EA; ++r) {
      const int e = tid + NT * r;
      if (BM * BK % NT != 0 && e >= BM * BK) continue;
      const int i = A_I ? e % BM : e / BK;
      const int l = A_I ? e / BM : e % BK;
      As[buf][l][i] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < EB; ++r) {
      const int e = tid + NT * r;
      if (BK * BN % NT != 0 && e >= BK * BN) continue;
      const int j = B_J ? e % BN : e / BK;
      const int l = B_J ? e / BN : e % BK;
      T val = rb[r];
      if constexpr (EPI == 5) {
        // Jastrow: B holds the rescaled e-e distances (diagonal < 0); split
        // s takes their s-th power, zero on the diagonal
        T pw = val < T(0) ? T(0) : T(1);
        for (int t = 0; t < s; ++t) pw *= val;
        val = pw;
      }
      Bs[buf][l][j] = val;
    }
  };

  const int lane = tid & 63, w = tid >> 6;
  const int wm = w / WGN, wn = w % WGN;
  v4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = v4{0, 0, 0, 0};

  auto mma = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4), ci = lane & 15;
      T fa[TM], fb[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) fa[a] = As[buf][kr][(wm * TM + a) * 16 + ci];
#pragma unroll
      for (int b = 0; b < TN; ++b) fb[b] = Bs[buf][kr][(wn * TN + b) * 16 + ci];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<T>::op(fa[a], fb[b], acc[a][b]);
    }
  };
  if constexpr (EPI == 4) {
    // K stages of sorted points: a stage is active if its 64-point block has
    // an active chunk among the AO columns [j0, j0 + BN) of this tile
    const int64_t nk = (Ls + BK - 1) / BK;
    const int64_t c0 = j0 / kSparseChunk, c1 = (min(j0 + BN, g.N) - 1) / kSparseChunk;
    const int64_t w0 = c0 >> 5, w1 = c1 >> 5;
    const uint32_t m0 = (~0u << (c0 & 31)) & (w1 == w0 ? (~0u >> (31 - (c1 & 31))) : ~0u);
    const uint32_t m1 = w1 == w0 ? 0u : (~0u >> (31 - (c1 & 31)));
    const int64_t p0 = static_cast<int64_t>(s) * g.Lchunk;
    auto next = [&](int64_t t) -> int64_t {
      for (; t < nk; ++t) {
        const uint32_t* w = g.act + ((p0 + t * BK) >> 6) * g.act_words;
        if ((w[w0] & m0) | (w1 != w0 ? (w[w1] & m1) : 0u)) break;
      }
      return t;
    };
    bool direct = false;
    if constexpr (kDirect) {
      if (dma_tile_ok<T, BK, B_J>(g, Ap, Bp)) {
        direct = true;
        dma_loop<T, BK, B_J, WGM, WGN, TM, TN>(
            reinterpret_cast<T*>(&sm), Ap + i0, Bp + (B_J ? j0 : j0 * g.sBj), g.sAl, g.sBl, g.sBj,
            g.M - i0, g.N - j0, next(0), nk, Ls % BK != 0 ? nk - 1 : -1, static_cast<int>(Ls % BK),
            [&](int64_t t) { return next(t + 1); }, acc);
      }
    }
    if (!direct) {
      int64_t cur = next(0);
      int buf = 0;
      if (cur < nk) {
        load(cur * BK);
        stash(0);
      }
      __syncthreads();
      while (cur < nk) {
        const int64_t nxt = next(cur + 1);
        if (nxt < nk) load(nxt * BK);
        mma(buf);
        if (nxt < nk) stash(buf ^ 1);
        __syncthreads();
        cur = nxt;
        buf ^= 1;
      }
    }
  } else {
    int64_t nk = EPI == 2 ? n_stages : (Ls + BK - 1) / BK;
    if constexpr (EPI == 3) {
      // output tile (AO rows [i0, i0 + BM), sorted points [j0, j0 + BN)):
      // skip the product if no point block of it has an active chunk there
      const int64_t c0 = i0 / kSparseChunk, c1 = (min(i0 + BM, g.M) - 1) / kSparseChunk;
      const int64_t b0 = j0 >> 6, b1 = (min(j0 + BN, g.N) - 1) >> 6;
      bool on = false;
      for (int64_t b = b0; b <= b1 && !on; ++b)
        for (int64_t c = c0; c <= c1 && !on; ++c) on = (g.act[b * g.act_words + (c >> 5)] >> (c & 31)) & 1u;
      if (!on) nk = 0;
    }
    auto l0_of = [&](int64_t t) -> int64_t {
      return (EPI == 2 ? static_cast<int64_t>(stage_list[t]) : t) * BK;
    };
    bool direct = false;
    if constexpr (kDirect) {
      if (dma_tile_ok<T, BK, B_J>(g, Ap, Bp)) {
        direct = true;
        // steps 0 .. nk-1, or the listed ones; the last step of the extent is
        // partial when Ls is not a multiple of BK
        const int64_t end = (Ls + BK - 1) / BK, part = Ls % BK != 0 ? end - 1 : -1;
        T* const stages = reinterpret_cast<T*>(&sm);
        const T* const At = Ap + i0;
        const T* const Bt = Bp + (B_J ? j0 : j0 * g.sBj);
        if constexpr (EPI == 2) {
          int pos = 0;
          dma_loop<T, BK, B_J, WGM, WGN, TM, TN>(
              stages, At, Bt, g.sAl, g.sBl, g.sBj, g.M - i0, g.N - j0, nk > 0 ? stage_list[0] : end, end, part,
              static_cast<int>(Ls % BK), [&](int64_t) -> int64_t { return ++pos < nk ? stage_list[pos] : end; },
              acc);
        } else {
          dma_loop<T, BK, B_J, WGM, WGN, TM, TN>(stages, At, Bt, g.sAl, g.sBl, g.sBj, g.M - i0, g.N - j0, 0,
                                                       nk, part, static_cast<int>(Ls % BK),
                                                       [](int64_t t) { return t + 1; }, acc);
        }
      }
    }
    if (!direct) {
      if (nk > 0) {
        load(l0_of(0));
        stash(0);
      }
      __syncthreads();
      for (int64_t kt = 0; kt < nk; ++kt) {
        const int buf = static_cast<int>(kt & 1);
        if (kt + 1 < nk) load(l0_of(kt + 1));
        mma(buf);
        if (kt + 1 < nk) stash(buf ^ 1);
        __syncthreads();
      }
    }
  }

  if constexpr (EPI == 1) {
    // the 16 lanes sharing lane / 16 hold the 16 columns of one row: sum
    // them with butterfly shuffles inside each 16-lane group
    double* const part = reinterpret_cast<double*>(g.D) + z * g.oDz +
                         static_cast<int64_t>(nt * WGN + wn) * g.sDj;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      // one block row at a time keeps the accumulators in place
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int64_t gj = j0 + (wn * TN + b) * 16 + (lane & 15);
          const double x = static_cast<double>(acc[a][b][r]);
          v += (gj < g.N ? g.occ[gj] : 0.0) * x * x;
        }
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        const int64_t gi = i0 + (wm * TM + a) * 16 + Mfma<T>::row(lane, r);
        if ((lane & 15) == 0 && gi < g.M) part[gi * g.sDi] = v;
      }
    }
  } else if constexpr (EPI == 5) {
    // Jastrow: weight output (i, j) by the polynomial of row i in x[a][j],
    // sum over the wave and store the sum in the wave's slot of batch z.
    // The coefficients of the tile's rows are staged in LDS (the operand
    // buffers are free after the last K step's barrier); x comes from L2,
    // one batch of loads per block row.
    const int64_t c_b = z / g.nsplit, s_k = z - c_b * g.nsplit;
    const double* const xw = g.jx + c_b * g.j_nn * g.N;
    const int nn = static_cast<int>(g.j_nn);
    static_assert(sizeof(sm.A) >= sizeof(double) * BM * kJasCoef, "coefficient stage does not fit");
    double* const qs = reinterpret_cast<double*>(&sm.A[0][0][0]);
    for (int e = tid; e < BM * kJasCoef; e += NT) {
      const int lr = e / kJasCoef, d = e - lr * kJasCoef;
      const int gi = static_cast<int>(i0) + lr;
      double q = 0.0;
      if (gi < g.M) {
        const int m1 = gi / nn, na = gi - m1 * nn;
        q = g.jq[((s_k * g.j_mh + m1) * g.j_nn + na) * kJasCoef + d];
      }
      qs[e] = q;
    }
    __syncthreads();
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      __builtin_amdgcn_sched_barrier(0);
      double xv[4][TN];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = static_cast<int>(i0) + (wm * TM + a) * 16 + Mfma<T>::row(lane, r);
        const bool row_in = gi < g.M;
        const int na = row_in ? gi % nn : 0;
        const double* const xr = xw + static_cast<int64_t>(na) * g.N;
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int64_t gj = j0 + (wn * TN + b) * 16 + (lane & 15);
          xv[r][b] = row_in && gj < g.N ? xr[gj] : 0.0;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double* const q = qs + ((wm * TM + a) * 16 + Mfma<T>::row(lane, r)) * kJasCoef;
        double qr[kJasCoef];
#pragma unroll
        for (int d = 0; d < kJasCoef; ++d) qr[d] = q[d];
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          // padded columns hold products with the k = 0 padding: masked
          const int64_t gj = j0 + (wn * TN + b) * 16 + (lane & 15);
          const double x = xv[r][b];
          double pw = qr[kJasCoef - 1];
#pragma unroll
          for (int d = kJasCoef - 2; d >= 0; --d) pw = pw * x + qr[d];
          v += gj < g.N ? pw * static_cast<double>(acc[a][b][r]) : 0.0;
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int64_t nNw = (g.N + BN - 1) / BN * WGN;
    if (lane == 0) Dp[(static_cast<int64_t>(mt) * WGM + wm) * nNw + static_cast<int64_t>(nt) * WGN + wn] = v;
  } else if constexpr (EPI == 2) {
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + (wm * TM + a) * 16 + Mfma<T>::row(lane, r);
        if (gi >= g.M) continue;
        TD* const row = Dp + static_cast<int64_t>(g.perm[gi]) * g.sDi;
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          const int64_t gj = j0 + (wn * TN + b) * 16 + (lane & 15);
          if (gj < g.N) row[gj * g.sDj] = static_cast<TD>(acc[a][b][r]);
        }
      }
    }
  } else {
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gi = i0 + (wm * TM + a) * 16 + Mfma<T>::row(lane, r);
          const int64_t gj = j0 + (wn * TN + b) * 16 + (lane & 15);
          if (gi < g.M && gj < g.N) Dp[gi * g.sDi + gj * g.sDj] = static_cast<TD>(acc[a][b][r]);
        }
  }
}

// Screened forward product (A = the AO array in sorted point order, i
// contiguous; B = C^T, j contiguous).  Wave 0 lists the K stages for which
// any 64-point block of this M tile has an active 16-AO chunk (g.act bitmap
// written by the AO kernel); the tile then runs over those stages only.
// Skipped stages hold exact zeros of A for every row of the tile, so each
// row's result is the dense product's, bit for bit.
template <typename T, typename TA, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_sparse_kernel(GemmArgs g, int nM, int nN) {
  constexpr int BM = 16 * WGM * TM;
  __shared__ GemmSmem<T, BM, 16 * WGN * TN, BK> sm;
  __shared__ int16_t s_list[kSparseMaxStages];
  __shared__ int s_n;
  int mt, nt, z;
  if (!grid_tile(g, nM, nN, blockIdx.x, mt, nt, z)) return;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int64_t i0 = static_cast<int64_t>(mt) * BM;
    const int64_t wb0 = i0 / 64, wb1 = (min(i0 + BM, g.M) - 1) / 64;
    const int64_t nk = (g.L + BK - 1) / BK, nchunk = (g.L + kSparseChunk - 1) / kSparseChunk;
    int count = 0;
    for (int64_t base = 0; base < nk; base += 64) {
      const int64_t t = base + lane;
      bool on = false;
      if (t < nk) {
        const int64_t c1 = min((t + 1) * BK / kSparseChunk, nchunk);
        for (int64_t c = t * BK / kSparseChunk; c < c1 && !on; ++c)
          for (int64_t wb = wb0; wb <= wb1 && !on; ++wb)
            on = (g.act[wb * g.act_words + (c >> 5)] >> (c & 31)) & 1u;
      }
      const uint64_t mask = __ballot(on);
      if (on) s_list[count + __popcll(mask & ((1ull << lane) - 1))] = static_cast<int16_t>(t);
      count += __popcll(mask);
    }
    if (lane == 0) s_n = count;
  }
  __syncthreads();
  gemm_body<T, TA, TB, TD, WGM, WGN, TM, TN, BK, true, true, 2>(g, mt, nt, z, sm, s_list, s_n);
}

// Density product: partial sums over columns of occ[j] (sum_l A(i,l) B(l,j))^2
// (see gemm_body, EPI = 1).
template <typename T, int WGM, int WGN, int TM, int TN, int BK>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_density_kernel(GemmArgs g, int nM, int nN) {
  __shared__ GemmSmem<T, 16 * WGM * TM, 16 * WGN * TN, BK> sm;
  int mt, nt, z;
  if (!grid_tile(g, nM, nN, blockIdx.x, mt, nt, z)) return;
  gemm_body<T, T, T, double, WGM, WGN, TM, TN, BK, true, true, 1>(g, mt, nt, z, sm);
}

template <typename T, typename TA, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK, bool A_I, bool B_J, int EPI = 0>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_kernel(GemmArgs g, int nM, int nN) {
  __shared__ GemmSmem<T, 16 * WGM * TM, 16 * WGN * TN, BK> sm;
  int mt, nt, z;
  if (!grid_tile(g, nM, nN, blockIdx.x, mt, nt, z)) return;
  gemm_body<T, TA, TB, TD, WGM, WGN, TM, TN, BK, A_I, B_J, EPI>(g, mt, nt, z, sm);
}

// Persistent form: the grid walks a list of (job, M tile, N tile, z).
template <typename T, typename TA, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK, bool A_I, bool B_J>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_persist(const GemmArgs* __restrict__ jobs,
                                                               const WorkItem* __restrict__ items,
                                                               int n_items) {
  __shared__ GemmSmem<T, 16 * WGM * TM, 16 * WGN * TN, BK> sm;
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const WorkItem it = items[i];
    gemm_body<T, TA, TB, TD, WGM, WGN, TM, TN, BK, A_I, B_J>(jobs[it.job], it.a, it.b, it.c, sm);
    __syncthreads();
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

// Tile configurations offered to the autotuner: {WGM, WGN, TM, TN, BK}.
#define QMK_TILE_LIST(X) \
  X(0, 2, 2, 4, 4, 16)   \
  X(1, 4, 1, 4, 5, 16)   \
  X(2, 2, 2, 4, 5, 16)   \
  X(3, 2, 2, 5, 4, 16)   \
  X(4, 1, 2, 5, 5, 16)   \
  X(5, 2, 2, 2, 5, 16)   \
  X(6, 2, 2, 4, 4, 32)   \
  X(7, 2, 2, 4, 3, 16)   \
  X(8, 2, 1, 5, 5, 16)   \
  X(9, 4, 1, 2, 5, 32)   \
  X(10, 2, 2, 5, 5, 16)  \
  X(11, 4, 1, 5, 5, 16)

constexpr TileCfg kTiles[] = {
#define QMK_TILE_ENTRY(id, wgm, wgn, tm, tn, bk) {wgm, wgn, tm, tn, bk},
    QMK_TILE_LIST(QMK_TILE_ENTRY)
#undef QMK_TILE_ENTRY
};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

template <typename T, typename TA, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK, bool A_I, bool B_J, int EPI = 0>
hipError_t run_tile(const GemmArgs& g, hipStream_t s) {
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN;
  const int nM = static_cast<int>((g.M + BM - 1) / BM), nN = static_cast<int>((g.N + BN - 1) / BN);
  if (nM <= 0 || nN <= 0) return hipSuccess;
  const dim3 grid = grid_of(g, nM, nN);
  hipLaunchKernelGGL((gemm_kernel<T, TA, TB, TD, WGM, WGN, TM, TN, BK, A_I, B_J, EPI>), grid,
                     dim3(64 * WGM * WGN), 0, s, g, nM, nN);
  return hipGetLastError();
}

template <typename T, typename TA, typename TB, typename TD, int WGM, int WGN, int TM, int TN,
          int BK, bool A_I, bool B_J>
hipError_t run_tile_persist(const PersistLaunch& pl, hipStream_t s) {
  auto k = gemm_persist<T, TA, TB, TD, WGM, WGN, TM, TN, BK, A_I, B_J>;
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

template <typename T, typename TA, typename TB, typename TD, bool A_I, bool B_J>
hipError_t run_persist(int cfg, const PersistLaunch& pl, hipStream_t s) {
  switch (cfg) {
#define QMK_TILE_PCASE(id, wgm, wgn, tm, tn, bk) \
  case id:                                       \
    return run_tile_persist<T, TA, TB, TD, wgm, wgn, tm, tn, bk, A_I, B_J>(pl, s);
    QMK_TILE_LIST(QMK_TILE_PCASE)
#undef QMK_TILE_PCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, typename TA, typename TB, typename TD, bool A_I, bool B_J, int EPI = 0>
hipError_t run(int cfg, const GemmArgs& g, hipStream_t s) {
  switch (cfg) {
#define QMK_TILE_CASE(id, wgm, wgn, tm, tn, bk) \
  case id:                                      \
    return run_tile<T, TA, TB, TD, wgm, wgn, tm, tn, bk, A_I, B_J, EPI>(g, s);
    QMK_TILE_LIST(QMK_TILE_CASE)
#undef QMK_TILE_CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T, int WGM, int WGN, int TM, int TN, int BK>
hipError_t run_density_tile(const GemmArgs& g, hipStream_t s) {
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN;
  const int nM = static_cast<int>((g.M + BM - 1) / BM), nN = static_cast<int>((g.N + BN - 1) / BN);
  if (nM <= 0 || nN <= 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_density_kernel<T, WGM, WGN, TM, TN, BK>), grid_of(g, nM, nN),
                     dim3(64 * WGM * WGN), 0, s, g, nM, nN);
  return hipGetLastError();
}

template <typename T, typename TD, int WGM, int WGN, int TM, int TN, int BK>
hipError_t run_sparse_tile(const GemmArgs& g, hipStream_t s) {
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN;
  const int nM = static_cast<int>((g.M + BM - 1) / BM), nN = static_cast<int>((g.N + BN - 1) / BN);
  if (nM <= 0 || nN <= 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_sparse_kernel<T, T, T, TD, WGM, WGN, TM, TN, BK>), grid_of(g, nM, nN),
                     dim3(64 * WGM * WGN), 0, s, g, nM, nN);
  return hipGetLastError();
}

template <typename T, typename TD>
hipError_t run_sparse(int cfg, const GemmArgs& g, hipStream_t s) {
  switch (cfg) {
#define QMK_TILE_SCASE(id, wgm, wgn, tm, tn, bk) \
  case id:                                       \
    return run_sparse_tile<T, TD, wgm, wgn, tm, tn, bk>(g, s);
    QMK_TILE_LIST(QMK_TILE_SCASE)
#undef QMK_TILE_SCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t run_density(int cfg, const GemmArgs& g, hipStream_t s) {
  switch (cfg) {
#define QMK_TILE_DCASE(id, wgm, wgn, tm, tn, bk) \
  case id:                                       \
    return run_density_tile<T, wgm, wgn, tm, tn, bk>(g, s);
    QMK_TILE_LIST(QMK_TILE_DCASE)
#undef QMK_TILE_DCASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace qmk
