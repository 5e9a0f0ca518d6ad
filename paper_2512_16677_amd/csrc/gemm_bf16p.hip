// BF16x3 contraction on pre-split operands (mixed precision mode).
//
// Every operand arrives as two bf16 planes, hi = bf16(x) and lo = bf16(x - hi)
// (x rounded to FP32 first), written once by its producer: the AO kernel
// writes the AO array as two planes, a streaming pass splits the adjoint
// weights W, and C is split when it is set.  A product is then
//   a b  ~  a_lo b_hi + a_hi b_lo + a_hi b_hi
// on v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the dropped lo*lo term
// is ~2^-18 |a b|), and the loop does no arithmetic on the operands: global
// loads go straight to LDS through registers, 16 bytes per lane.
//
// Layouts.  B is always reduction-major ("K-major": eight consecutive
// reduction indices are contiguous) and is staged as [row][k], 64 bytes per
// row with its 16-byte chunks XOR-permuted by row bits (see kswz), so that
// the 16-byte fragment reads and the stores of the lanes served in one LDS
// cycle hit different bank groups.  A is either K-major (the
// W C product reads C^T) or row-major ("MN-major": the AO array in the forward
// product and W in the W^T ao product have their points / MOs contiguous);
// an MN-major A is staged as [k][row] and its MFMA fragments are read with
// gfx950's transposing LDS load (ds_read_b64_tr_b16), which hands lane i of
// each 16-lane group four consecutive k of row i.  Its row pitch is padded to
// 32 or 96 bytes modulo 128, so the four k-rows one 16-lane group touches lie
// in four different 32-byte bank windows.
//
// Loads are unguarded along the reduction index: every operand buffer is
// zero-padded to a multiple of 32 there.  Rows past the operand's row count
// are staged as zeros (their chunks are loaded from the last row in range, so
// every load stays in bounds).  Stores are guarded on both indices.
//
// Two staging schemes (the tile's DEPTH):
//   DEPTH 1, 2: each thread loads its chunks into registers DEPTH K steps
//     ahead and stores them to one of two LDS buffers;
//   DEPTH >= 3 (or -2): an LDS ring of DEPTH (2) stages filled by
//     global_load_lds_dwordx4
//     (each lane's 16 bytes go from global memory straight to LDS), so the
//     loads of steps kt + 1 .. kt + DEPTH are in flight while step kt
//     computes and no registers hold operand data; the MFMA fragments of
//     step kt + 1 are read from LDS under the MFMAs of step kt.  The ring lays a tile out without
//     padding (a load instruction fills 1 KB of consecutive LDS); an
//     MN-major tile permutes the 16-byte chunks of each k-row instead (see
//     mn_xor), and rows past the operand's row count hold copies of the last
//     row's chunks: they only reach outputs that are not stored.
#include <algorithm>
#include <type_traits>

#include "qmk_internal.h"

namespace qmk {
// Launch of the persistent form, shared by the per-product translation units.
struct BfpPersist {
  const GemmArgs* jobs;
  const WorkItem* items;
  int n_items, grid;
  int* occupancy;  // != NULL: report resident workgroups per CU, launch nothing
};

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

constexpr int BK = 32;
// K-major staging: rows of BK elements (64 bytes, no padding); 16-byte chunk
// c of row r sits at chunk c ^ kswz(r).  Eight consecutive rows read at one
// chunk then cover all eight 16-byte bank groups of 128 bytes, and sixteen
// rows all sixteen of 256 bytes; a thread's stores (four chunks of a row,
// rows in order) are permutations of contiguous runs.
constexpr int KLD = BK;
// Only bits 1..3 of the row enter, so a 16-row fragment block (rows r0 + i,
// r0 a multiple of 16) has the swizzle of i.
__device__ __forceinline__ int kswz(int r) { return ((r >> 1) & 3) ^ (((r >> 3) & 1) * 3); }

// MN-major staging pitch (elements) for R rows: R*2 bytes made 32 or 96 mod 128.
constexpr int mn_pitch(int R) { return ((R * 2) % 128 == 32 || (R * 2) % 128 == 96) ? R : R + 16; }

template <int BM, int BN, bool A_MN>
struct PSmem {
  static constexpr int A_ELEMS = A_MN ? BK * mn_pitch(BM) : BM * KLD;
  static constexpr int B_ELEMS = BN * KLD;
  __bf16 A[2][2][A_ELEMS];  // [buffer][hi, lo]
  __bf16 B[2][2][B_ELEMS];
};

// One operand tile (R rows x BK reduction indices, both planes) in flight:
// 16-byte chunks spread over NT threads, the same chunks of both planes per
// thread.  Element (row, l) of a plane is at plane[row * s_row + l * s_l];
// MN: s_row = 1 (chunks of 8 rows at one l), else s_l = 1 (chunks of 8 l of
// one row).  The byte offset of every chunk from the tile's base and its
// staging offset are computed once per tile; a K step only moves the two
// (wave-uniform) plane pointers.  When NT does not divide the chunk count,
// the surplus threads load and store a chunk again (the same bytes to the
// same place); a chunk past the last row in range is loaded from that last
// row and stored as zeros, so every load is in bounds and unconditional.
template <int R, int NT, bool MN>
struct PTile {
  static constexpr int CH = MN ? BK * (R / 8) : R * (BK / 8);  // chunks per plane
  static constexpr int PER = (CH + NT - 1) / NT;
  uint32_t goff[PER];  // byte offset from the tile's plane base
  int32_t loff[PER];   // element offset in one plane's staging buffer
  bool ok[PER];
  u32x4 v[2][PER];

  __device__ __forceinline__ void init(int64_t s_row, int64_t s_l, int64_t rows_left, int tid) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      int q = tid + NT * u;
      if (CH % NT != 0) q %= CH;
      int64_t row, off;
      if constexpr (MN) {
        const int l = q / (R / 8);
        row = static_cast<int64_t>(q % (R / 8)) * 8;
        const int64_t rr = row < rows_left ? row : ((rows_left - 1) & ~int64_t(7));
        off = rr + l * s_l;
        loff[u] = l * mn_pitch(R) + static_cast<int>(row);
      } else {
        row = q / (BK / 8);
        const int kq = q % (BK / 8);
        const int64_t rr = row < rows_left ? row : rows_left - 1;
        off = rr * s_row + kq * 8;
        loff[u] = static_cast<int>(row) * KLD + (kq ^ kswz(static_cast<int>(row))) * 8;
      }
      goff[u] = static_cast<uint32_t>(off * 2);
      ok[u] = row < rows_left;
    }
  }

  __device__ __forceinline__ void load(const __bf16* hi, const __bf16* lo) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      v[0][u] = *reinterpret_cast<const u32x4*>(reinterpret_cast<const char*>(hi) + goff[u]);
      v[1][u] = *reinterpret_cast<const u32x4*>(reinterpret_cast<const char*>(lo) + goff[u]);
    }
  }

  template <bool FULL>
  __device__ __forceinline__ void stash(__bf16* hi, __bf16* lo) const {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      *reinterpret_cast<u32x4*>(hi + loff[u]) = (FULL || ok[u]) ? v[0][u] : u32x4{0u, 0u, 0u, 0u};
      *reinterpret_cast<u32x4*>(lo + loff[u]) = (FULL || ok[u]) ? v[1][u] : u32x4{0u, 0u, 0u, 0u};
    }
  }
};

// MFMA fragment of rows r0 .. r0+15 of an MN-major staged tile: lane 16g + i
// receives k = 8g .. 8g+7 of row r0 + i (two transposing 8-byte reads).
template <int PITCH>
__device__ __forceinline__ bf16x8 frag_mn(const __bf16* t, int r0, int lane) {
  const int g = lane >> 4, q = lane & 15;
  const __bf16* p0 = t + (8 * g + (q >> 2)) * PITCH + r0 + 4 * (q & 3);
  const __bf16* p1 = p0 + 4 * PITCH;
  const s16x4 x0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (lds_s16x4*)((__attribute__((address_space(3))) char*)(p0)));
  const s16x4 x1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (lds_s16x4*)((__attribute__((address_space(3))) char*)(p1)));
  typedef short s16x8 __attribute__((ext_vector_type(8)));
  const s16x8 x = __builtin_shufflevector(x0, x1, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, x);
}

// Fragment of a K-major staged tile: lane 16g + i receives k = 8g .. 8g+7 of
// row r0 + i.
__device__ __forceinline__ bf16x8 frag_k(const __bf16* t, int r0, int lane) {
  // r0 is a multiple of 16, so the swizzle of row r0 + i is that of i
  const int i = lane & 15;
  return *reinterpret_cast<const bf16x8*>(t + (r0 + i) * KLD + ((lane >> 4) ^ kswz(i)) * 8);
}

// ---------------------------------------------------------------------------
// LDS ring staging (DEPTH >= 3, or -2 for a two-stage ring small enough
// that two workgroups share a CU).

// Ring stages of a tile's DEPTH (0: register staging).
constexpr int ring_stages(int depth) { return depth >= 3 ? depth : (depth < 0 ? -depth : 0); }

// MN-major ring tile of R rows: 16-byte chunk c of k-row l sits at chunk
// c ^ mn_xor(l).  A 16-lane group of the transposing fragment read touches
// 32 consecutive bytes of each of four consecutive k-rows (l0 .. l0+3), and
// the 32 lanes served together touch the rows l0 .. l0+3 and l0+8 .. l0+11:
// eight 32-byte windows, which the permutation puts on eight different
// 32-byte bank windows for every k-row pitch R * 2 that is a multiple of 64
// bytes (pitch = 0 mod 256: rows by their bits 0, 1 and 3; 128: bits 1 and
// 3; 64 or 192: bit 3).  Rows l and l + 4 share the permutation.
template <int R>
__device__ __forceinline__ int mn_xor(int l) {
  constexpr int p = (R * 2) % 256;
  if constexpr (p == 0) return 2 * (l & 3) + 8 * ((l >> 3) & 1);
  else if constexpr (p == 128) return 2 * ((l >> 1) & 1) + 4 * ((l >> 3) & 1);
  else if constexpr (p == 64 || p == 192) return 2 * ((l >> 3) & 1);
  else return 0;
}

// MFMA fragment of rows r0 .. r0+15 of an MN-major ring tile (as frag_mn).
template <int R>
__device__ __forceinline__ bf16x8 frag_mnx(const __bf16* t, int r0, int lane) {
  const int g = lane >> 4, q = lane & 15;
  const int l = 8 * g + (q >> 2);
  const int e = r0 + 4 * (q & 3);
  const __bf16* p0 = t + l * R + (((e >> 3) ^ mn_xor<R>(l)) << 3) + (e & 7);
  const __bf16* p1 = p0 + 4 * R;
  const s16x4 x0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (lds_s16x4*)((__attribute__((address_space(3))) char*)(p0)));
  const s16x4 x1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (lds_s16x4*)((__attribute__((address_space(3))) char*)(p1)));
  typedef short s16x8 __attribute__((ext_vector_type(8)));
  const s16x8 x = __builtin_shufflevector(x0, x1, 0, 1, 2, 3, 4, 5, 6, 7);
  return __builtin_bit_cast(bf16x8, x);
}

// One stage of the ring: [A hi][A lo][B hi][B lo], BK reduction indices
// each, 1 KB per load instruction.
template <int BM, int BN, int S>
struct RingSmem {
  static constexpr int STAGE = (BM + BN) * BK * 2;  // elements
  __bf16 ring[S * STAGE];
};

__device__ __forceinline__ uint32_t lds_address(const void* p) {
  return static_cast<uint32_t>(
      reinterpret_cast<uintptr_t>((const __attribute__((address_space(3))) char*)(p)));
}

// One load instruction: lane l's 16 bytes at g land at LDS byte lds + 16 l
// (the wave-uniform base goes through M0).  The compiler does not see these
// LDS writes; ring_sync waits for them.
__device__ __forceinline__ void dma16(const void* g, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %1, off" : : "s"(lds), "v"(g)
               : "memory", "m0");
}

// Waits until at most N of this wave's vector memory instructions are
// outstanding and its LDS reads have returned, then joins the workgroup
// barrier.  The memory clobber keeps the next step's LDS reads below it.
template <int N>
__device__ __forceinline__ void ring_sync() {
  static_assert(N >= 0 && N < 64, "vmcnt holds 6 bits");
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" : : "n"(N) : "memory");
}

// K loop of one tile on an S-stage ring.  Every wave issues the same number
// of load instructions per stage (IPW; a wave short of real ones repeats
// one, writing the same bytes again), so vmcnt counts stages.
// PF: the MFMA fragments of stage kt + 1 are read into a second register
// set right after the barrier of step kt and under the MFMAs of stage kt, so
// the LDS reads of one stage overlap the MFMAs of the previous one.  The
// barrier of step kt then also means that every wave holds its fragments of
// stage kt: that stage's slot is free, and the loads of stage kt + S go into
// it (all S slots are in flight or being read).  Without PF (fewer
// registers) step kt waits for stage kt, reads its fragments and computes,
// with the loads of stage kt + S - 1 going into the slot read in step kt - 1.
template <bool A_MN, int WGM, int WGN, int TM, int TN, int S, bool LIST, bool PF>
__device__ __forceinline__ void bf16p_ring(__bf16* ring, const __bf16* Ah, const __bf16* Al, const __bf16* Bh,
                                           const __bf16* Bl, int64_t sAi, int64_t sAl, int64_t sBj, int64_t sBl,
                                           int64_t rows_a, int64_t rows_b, int64_t nk, const int16_t* list,
                                           f32x4 (&acc)[TM][TN]) {
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN, NW = WGM * WGN;
  constexpr int NI = (BM + BN) / 8;  // load instructions per stage: 1 KB each
  constexpr int IPW = (NI + NW - 1) / NW;
  constexpr int STAGE = RingSmem<BM, BN, S>::STAGE;
  static_assert(S >= 2 && S <= 5, "ring depth");
  static_assert((S - 1) * IPW < 64, "outstanding loads exceed vmcnt");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WGN, wn = w % WGN;
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const uint32_t ring_lds = __builtin_amdgcn_readfirstlane(lds_address(ring));

  // per instruction: this lane's source (tile base + chunk offset), the
  // bytes one K step moves it, and the LDS offset of its 1 KB in a stage
  const char* gp[IPW];
  int64_t step[IPW];
  uint32_t ldso[IPW];
#pragma unroll
  for (int i = 0; i < IPW; ++i) {
    int ig = wu + NW * i;
    if (NI % NW != 0 && ig >= NI) ig -= NI;
    ldso[i] = static_cast<uint32_t>(ig) * 1024u;
    const bool is_a = ig < BM / 8;
    const bool lo = is_a ? ig >= BM / 16 : ig >= BM / 8 + BN / 16;
    const int j = is_a ? (lo ? ig - BM / 16 : ig) : (lo ? ig - BM / 8 - BN / 16 : ig - BM / 8);
    const int sl = 64 * j + lane;  // 16-byte slot within the plane's tile
    int64_t off;
    if (is_a && A_MN) {
      const int l = sl / (BM / 8), c = sl % (BM / 8);
      const int64_t row = static_cast<int64_t>((c ^ mn_xor<BM>(l)) * 8);
      const int64_t rr = row < rows_a ? row : ((rows_a - 1) & ~int64_t(7));
      off = rr * sAi + l * sAl;
    } else {
      const int r = sl >> 2, kq = (sl & 3) ^ kswz(sl >> 2);
      const int64_t rows = is_a ? rows_a : rows_b;
      const int64_t rr = r < rows ? r : rows - 1;
      off = rr * (is_a ? sAi : sBj) + kq * 8;
    }
    const __bf16* base = is_a ? (lo ? Al : Ah) : (lo ? Bl : Bh);
    gp[i] = reinterpret_cast<const char*>(base + off);
    step[i] = static_cast<int64_t>(BK) * (is_a ? sAl : sBl) * 2;
  }
  auto issue = [&](int slot, int64_t kt) {
    const int64_t t = LIST ? static_cast<int64_t>(__builtin_amdgcn_readfirstlane(list[kt])) : kt;
    const uint32_t sb = ring_lds + static_cast<uint32_t>(slot * STAGE * 2);
#pragma unroll
    for (int i = 0; i < IPW; ++i) dma16(gp[i] + t * step[i], sb + ldso[i]);
  };
  struct Frags {
    bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
  };
  auto read_a = [&](int slot, int a, Frags& f) {
    const __bf16* A0 = ring + slot * STAGE;
    const __bf16* A1 = A0 + BM * BK;
    const int r0 = (wm * TM + a) * 16;
    if constexpr (A_MN) {
      f.ah[a] = frag_mnx<BM>(A0, r0, lane);
      f.al[a] = frag_mnx<BM>(A1, r0, lane);
    } else {
      f.ah[a] = frag_k(A0, r0, lane);
      f.al[a] = frag_k(A1, r0, lane);
    }
  };
  auto read_b = [&](int slot, Frags& f) {
    const __bf16* B0 = ring + slot * STAGE + 2 * BM * BK;
    const __bf16* B1 = B0 + BN * BK;
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int r0 = (wn * TN + b) * 16;
      f.bh[b] = frag_k(B0, r0, lane);
      f.bl[b] = frag_k(B1, r0, lane);
    }
  };
  auto sync = [&](int64_t later) {  // stages issued after the one to read
    if (later >= 4) ring_sync<(S > 4 ? 4 : 0) * IPW>();
    else if (later == 3) ring_sync<(S > 3 ? 3 : 0) * IPW>();
    else if (later == 2) ring_sync<2 * IPW>();
    else if (later == 1) ring_sync<IPW>();
    else ring_sync<0>();
  };
  // Step kt: f holds stage kt (slot rs).  With MORE (a stage kt + 1
  // follows) the B fragments of stage kt + 1 are read into g first and its
  // A fragments of row block a after the MFMAs of row block a, which frees
  // f.ah[a], f.al[a]; the scheduling barriers keep the reads in that order,
  // so both sets together hold one stage plus the B fragments.
  auto step_kt = [&](auto more_c, int64_t kt, int rs, Frags& f, Frags& g) {
    constexpr bool MORE = decltype(more_c)::value;
    const int ns = rs + 1 == S ? 0 : rs + 1;
    if constexpr (MORE) {
      sync(min(nk - 2 - kt, static_cast<int64_t>(S - 2)));
      if (kt + S < nk) issue(rs, kt + S);
      read_b(ns, g);
    }
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      // the three products of one accumulator are TN instructions apart
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.al[a], f.bh[b], acc[a][b], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[a], f.bl[b], acc[a][b], 0, 0, 0);
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(f.ah[a], f.bh[b], acc[a][b], 0, 0, 0);
      if constexpr (MORE) {
        __builtin_amdgcn_sched_barrier(0);
        read_a(ns, a, g);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  using More = std::integral_constant<bool, true>;
  using Last = std::integral_constant<bool, false>;

  if (nk <= 0) return;
  if constexpr (!PF) {
#pragma unroll
    for (int st = 0; st < S - 1; ++st)
      if (st < nk) issue(st, st);
    int slot = 0;
    for (int64_t kt = 0; kt < nk; ++kt) {
      sync(min(nk - 1 - kt, static_cast<int64_t>(S - 2)));
      if (kt + S - 1 < nk) issue(slot == 0 ? S - 1 : slot - 1, kt + S - 1);
      Frags f;
      read_b(slot, f);
#pragma unroll
      for (int a = 0; a < TM; ++a) read_a(slot, a, f);
      step_kt(Last{}, kt, slot, f, f);
      slot = slot + 1 == S ? 0 : slot + 1;
    }
    return;
  }
#pragma unroll
  for (int st = 0; st < S; ++st)
    if (st < nk) issue(st, st);
  sync(min(nk - 1, static_cast<int64_t>(S - 1)));
  Frags f0, f1;
  read_b(0, f0);
#pragma unroll
  for (int a = 0; a < TM; ++a) read_a(0, a, f0);
  int slot = 0;
  int64_t kt = 0;
  for (; kt + 2 < nk; kt += 2) {
    step_kt(More{}, kt, slot, f0, f1);
    slot = slot + 1 == S ? 0 : slot + 1;
    step_kt(More{}, kt + 1, slot, f1, f0);
    slot = slot + 1 == S ? 0 : slot + 1;
  }
  if (kt + 1 < nk) {
    step_kt(More{}, kt, slot, f0, f1);
    slot = slot + 1 == S ? 0 : slot + 1;
    step_kt(Last{}, kt + 1, slot, f1, f0);
  } else {
    step_kt(Last{}, kt, slot, f0, f1);
  }
}

// The K loop of one tile.  FULL: every row of both operand tiles is in
// range (no zero fill).  The loop is unrolled by two so that both staging
// buffers are compile-time constants.
// list (screened products): the K steps to visit, nk of them; otherwise
// steps 0 .. nk-1.
template <bool A_MN, bool FULL, int WGM, int WGN, int TM, int TN, int DEPTH, bool LIST>
__device__ __forceinline__ void bf16p_loop(PSmem<16 * WGM * TM, 16 * WGN * TN, A_MN>& sm,
                                           PTile<16 * WGM * TM, 64 * WGM * WGN, A_MN> (&la)[DEPTH],
                                           PTile<16 * WGN * TN, 64 * WGM * WGN, false> (&lb)[DEPTH],
                                           const __bf16* Ah, const __bf16* Al, const __bf16* Bh,
                                           const __bf16* Bl, int64_t stepA, int64_t stepB, int64_t nk,
                                           const int16_t* list, f32x4 (&acc)[TM][TN]) {
  constexpr int BM = 16 * WGM * TM;
  constexpr int AP = mn_pitch(BM);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WGN, wn = w % WGN;
  auto load = [&](int r, int64_t kt) {
    const int64_t t = LIST ? static_cast<int64_t>(__builtin_amdgcn_readfirstlane(list[kt])) : kt;
    la[r].load(Ah + t * stepA, Al + t * stepA);
    lb[r].load(Bh + t * stepB, Bl + t * stepB);
  };
  auto stash = [&](int r, int buf) {
    la[r].template stash<FULL>(sm.A[buf][0], sm.A[buf][1]);
    lb[r].template stash<FULL>(sm.B[buf][0], sm.B[buf][1]);
  };
  auto compute = [&](int buf) {
    bf16x8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
    for (int a = 0; a < TM; ++a) {
      const int r0 = (wm * TM + a) * 16;
      if constexpr (A_MN) {
        ah[a] = frag_mn<AP>(sm.A[buf][0], r0, lane);
        al[a] = frag_mn<AP>(sm.A[buf][1], r0, lane);
      } else {
        ah[a] = frag_k(sm.A[buf][0], r0, lane);
        al[a] = frag_k(sm.A[buf][1], r0, lane);
      }
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int r0 = (wn * TN + b) * 16;
      bh[b] = frag_k(sm.B[buf][0], r0, lane);
      bl[b] = frag_k(sm.B[buf][1], r0, lane);
    }
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh[b], acc[a][b], 0, 0, 0);
      }
  };

  if (nk <= 0) return;
  if constexpr (DEPTH == 1) {
    load(0, 0);
    stash(0, 0);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; kt += 2) {
      if (kt + 1 < nk) load(0, kt + 1);
      compute(0);
      if (kt + 1 < nk) stash(0, 1);
      __syncthreads();
      if (kt + 1 >= nk) break;
      if (kt + 2 < nk) load(0, kt + 2);
      compute(1);
      if (kt + 2 < nk) stash(0, 0);
      __syncthreads();
    }
  } else {
    load(0, 0);
    stash(0, 0);
    if (nk > 1) load(1, 1);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; kt += 2) {
      // step kt from LDS buffer 0; registers 1 hold step kt+1
      if (kt + 2 < nk) load(0, kt + 2);
      compute(0);
      if (kt + 1 < nk) stash(1, 1);
      __syncthreads();
      if (kt + 1 >= nk) break;
      // step kt+1 from LDS buffer 1; registers 0 hold step kt+2
      if (kt + 3 < nk) load(1, kt + 3);
      compute(1);
      if (kt + 2 < nk) stash(0, 0);
      __syncthreads();
    }
  }
}

// SCR: 0 dense; the screened products on points sorted by nearest nucleus
// (g.act: bit c of word (block * act_words + c / 32) set if the 64-point
// block has a non-zero AO in 16-AO chunk c):
//   2 forward: the K steps (32 AOs) with an active chunk in some 64-point
//     block of the tile's rows are listed and visited; row i of D is stored
//     at row perm[i];
//   3 W C product (rows AOs, columns sorted points): a tile with no active
//     (block, chunk) pair is not computed (its zeros are stored);
//   4 W^T ao product (K over the sorted points of split s): the K steps whose
//     64-point block has an active chunk among the tile's AO columns.
// Skipped steps and tiles hold exact zeros of the AO operand, so every
// output is a sum of the same non-zero terms as in the dense product.
// PF: ring tiles read the next stage's fragments under the current MFMAs
// (the persistent form, which holds more state, and the two-stage tiles,
// which must fit two workgroups per CU, do without).
template <bool A_MN, int WGM, int WGN, int TM, int TN, int DEPTH>
using SmemOf = std::conditional_t<(ring_stages(DEPTH) > 0),
                                  RingSmem<16 * WGM * TM, 16 * WGN * TN,
                                           (ring_stages(DEPTH) > 0 ? ring_stages(DEPTH) : 1)>,
                                  PSmem<16 * WGM * TM, 16 * WGN * TN, A_MN>>;

template <bool A_MN, typename TD, int WGM, int WGN, int TM, int TN, int DEPTH, int SCR, bool PF = true>
__device__ __forceinline__ void bf16p_body(const GemmArgs& g, int mt, int nt, int z,
                                           SmemOf<A_MN, WGM, WGN, TM, TN, DEPTH>& sm,
                                           int16_t* s_list, int* s_n) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN;
  const int c = z / g.nsplit, s = z - c * g.nsplit;
  const int64_t i0 = static_cast<int64_t>(mt) * BM, j0 = static_cast<int64_t>(nt) * BN;
  const int64_t oa = c * g.oAc + s * g.oAs + i0 * g.sAi, ob = c * g.oBc + s * g.oBs + j0 * g.sBj;
  const __bf16* Ah = static_cast<const __bf16*>(g.A) + oa;
  const __bf16* Al = static_cast<const __bf16*>(g.A2) + oa;
  const __bf16* Bh = static_cast<const __bf16*>(g.B) + ob;
  const __bf16* Bl = static_cast<const __bf16*>(g.B2) + ob;
  TD* __restrict__ Dp = static_cast<TD*>(g.D) + z * g.oDz;
  const int64_t Ls = min(g.Lchunk, g.L - s * g.Lchunk);
  const int tid = threadIdx.x;
  const int64_t rows_a = g.M - i0, rows_b = g.N - j0;

  f32x4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};

  int64_t nk = (Ls + BK - 1) / BK;
  if constexpr (SCR == 2 || SCR == 4) {
    // wave 0 lists the active K steps (at most kSparseMaxStages; the host
    // sizes the reduction ranges accordingly)
    if (tid < 64) {
      int count = 0;
      int64_t cb0 = 0, cb1 = 0, w0 = 0, w1 = 0;
      uint32_t m0 = 0, m1 = 0;
      if constexpr (SCR == 2) {
        cb0 = i0 >> 6;
        cb1 = (min(i0 + BM, g.M) - 1) >> 6;
      } else {
        const int64_t c0 = j0 / kSparseChunk, c1 = (min(j0 + BN, g.N) - 1) / kSparseChunk;
        w0 = c0 >> 5;
        w1 = c1 >> 5;
        m0 = (~0u << (c0 & 31)) & (w1 == w0 ? (~0u >> (31 - (c1 & 31))) : ~0u);
        m1 = w1 == w0 ? 0u : (~0u >> (31 - (c1 & 31)));
      }
      const int64_t nchunk = (g.L + kSparseChunk - 1) / kSparseChunk;
      const int64_t p0 = static_cast<int64_t>(s) * g.Lchunk;
      for (int64_t base = 0; base < nk; base += 64) {
        const int64_t t = base + tid;
        bool on = false;
        if (t < nk) {
          if constexpr (SCR == 2) {
            const int64_t c1 = min((t + 1) * BK / kSparseChunk, nchunk);
            for (int64_t c = t * BK / kSparseChunk; c < c1 && !on; ++c)
              for (int64_t b = cb0; b <= cb1 && !on; ++b)
                on = (g.act[b * g.act_words + (c >> 5)] >> (c & 31)) & 1u;
          } else {
            const uint32_t* wd = g.act + ((p0 + t * BK) >> 6) * g.act_words;
            on = ((wd[w0] & m0) | (w1 != w0 ? (wd[w1] & m1) : 0u)) != 0u;
          }
        }
        const uint64_t mask = __ballot(on);
        if (on) s_list[count + __popcll(mask & ((1ull << tid) - 1))] = static_cast<int16_t>(t);
        count += __popcll(mask);
      }
      if (tid == 0) *s_n = count;
    }
    __syncthreads();
    nk = *s_n;
  }
  if constexpr (SCR == 3) {
    // output tile (AO rows [i0, i0 + BM), sorted points [j0, j0 + BN))
    const int64_t c0 = i0 / kSparseChunk, c1 = (min(i0 + BM, g.M) - 1) / kSparseChunk;
    const int64_t b0 = j0 >> 6, b1 = (min(j0 + BN, g.N) - 1) >> 6;
    bool on = false;
    for (int64_t b = b0; b <= b1 && !on; ++b)
      for (int64_t c = c0; c <= c1 && !on; ++c) on = (g.act[b * g.act_words + (c >> 5)] >> (c & 31)) & 1u;
    if (!on) nk = 0;
  }
  constexpr bool LIST = SCR == 2 || SCR == 4;
  if constexpr (ring_stages(DEPTH) > 0) {
    bf16p_ring<A_MN, WGM, WGN, TM, TN, ring_stages(DEPTH), LIST, PF>(sm.ring, Ah, Al, Bh, Bl, g.sAi, g.sAl, g.sBj,
                                                                     g.sBl, rows_a, rows_b, nk, s_list, acc);
  } else {
    // DEPTH register stages: the global loads of K step k + DEPTH are issued
    // before the MFMAs of step k, so each load has DEPTH steps of MFMA work
    // to arrive (DEPTH 2 costs one more operand tile of registers per thread).
    PTile<BM, NT, A_MN> la[DEPTH];
    PTile<BN, NT, false> lb[DEPTH];
#pragma unroll
    for (int r = 0; r < DEPTH; ++r) {
      la[r].init(g.sAi, g.sAl, rows_a, tid);
      lb[r].init(g.sBj, g.sBl, rows_b, tid);
    }
    const int64_t stepA = BK * g.sAl, stepB = BK * g.sBl;
    if (rows_a >= BM && rows_b >= BN)
      bf16p_loop<A_MN, true, WGM, WGN, TM, TN, DEPTH, LIST>(sm, la, lb, Ah, Al, Bh, Bl, stepA, stepB, nk, s_list,
                                                            acc);
    else
      bf16p_loop<A_MN, false, WGM, WGN, TM, TN, DEPTH, LIST>(sm, la, lb, Ah, Al, Bh, Bl, stepA, stepB, nk,
                                                             s_list, acc);
  }

  // accumulator element r of lane l: row 4 (l / 16) + r, column l % 16
  const int lane = tid & 63, w = tid >> 6;
  const int wm = w / WGN, wn = w % WGN;
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + (wm * TM + a) * 16 + 4 * (lane >> 4) + r;
        const int64_t gj = j0 + (wn * TN + b) * 16 + (lane & 15);
        if (gi < g.M && gj < g.N) {
          const int64_t row = SCR == 2 ? static_cast<int64_t>(g.perm[gi]) : gi;
          Dp[row * g.sDi + gj * g.sDj] = static_cast<TD>(acc[a][b][r]);
        }
      }
}

template <bool A_MN, typename TD, int WGM, int WGN, int TM, int TN, int DEPTH, int SCR>
__global__ __launch_bounds__(64 * WGM * WGN, DEPTH < 0 ? 2 : 1) void gemm_bf16p_kernel(GemmArgs g, int nM, int nN) {
  __shared__ __align__(16) SmemOf<A_MN, WGM, WGN, TM, TN, DEPTH> sm;
  __shared__ int16_t s_list[(SCR == 2 || SCR == 4) ? kSparseMaxStages : 1];
  __shared__ int s_n;
  int mt, nt, z;
  if (!grid_tile(g, nM, nN, blockIdx.x, mt, nt, z)) return;
  bf16p_body<A_MN, TD, WGM, WGN, TM, TN, DEPTH, SCR, (DEPTH > 0)>(g, mt, nt, z, sm, s_list, &s_n);
}

// Persistent form (batch executor): the grid walks a list of (job, M tile,
// N tile, z) items, each job holding one molecule's arguments.
template <bool A_MN, typename TD, int WGM, int WGN, int TM, int TN, int DEPTH>
__global__ __launch_bounds__(64 * WGM * WGN, DEPTH < 0 ? 2 : 1) void gemm_bf16p_persist(
    const GemmArgs* __restrict__ jobs, const WorkItem* __restrict__ items, int n_items) {
  __shared__ __align__(16) SmemOf<A_MN, WGM, WGN, TM, TN, DEPTH> sm;
  __shared__ int16_t s_list[1];
  __shared__ int s_n;
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const WorkItem it = items[i];
    bf16p_body<A_MN, TD, WGM, WGN, TM, TN, DEPTH, 0, false>(jobs[it.job], it.a, it.b, it.c, sm, s_list, &s_n);
    __syncthreads();  // LDS is restaged by the next item
  }
}

// {WGM, WGN, TM, TN, DEPTH}; the reduction step is always 32.  DEPTH 1, 2:
// register staging; DEPTH >= 3: LDS ring of DEPTH stages; DEPTH -2: LDS ring
// of two stages, compiled for two waves per SIMD so that two 4-wave
// workgroups share a CU (one's output stores and barrier waits overlap the
// other's K loop); these read each stage's fragments after its barrier.
#define QMK_BF16P_TILE_LIST(X) \
  X(0, 2, 2, 4, 4, 1)          \
  X(1, 2, 2, 4, 4, 2)          \
  X(2, 4, 2, 4, 4, 1)          \
  X(3, 2, 4, 4, 4, 1)          \
  X(4, 4, 1, 2, 5, 1)          \
  X(5, 4, 1, 2, 5, 2)          \
  X(6, 2, 2, 4, 2, 1)          \
  X(7, 2, 2, 4, 2, 2)          \
  X(8, 2, 2, 2, 4, 2)          \
  X(9, 4, 2, 2, 4, 2)          \
  X(10, 2, 2, 5, 5, 1)         \
  X(11, 2, 1, 5, 5, 1)         \
  X(12, 1, 2, 5, 5, 1)         \
  X(13, 4, 1, 4, 5, 1)         \
  X(14, 2, 4, 4, 2, 2)         \
  X(15, 2, 2, 4, 5, 1)         \
  X(16, 4, 2, 4, 4, 3)         \
  X(17, 2, 2, 4, 4, 3)         \
  X(18, 2, 2, 4, 4, 4)         \
  X(19, 4, 1, 4, 5, 3)         \
  X(20, 4, 2, 4, 5, 3)         \
  X(21, 2, 2, 5, 5, 3)         \
  X(22, 1, 2, 5, 5, 4)         \
  X(23, 2, 4, 5, 4, 3)         \
  X(24, 8, 1, 2, 5, 3)         \
  X(25, 2, 2, 4, 5, -2)        \
  X(26, 2, 2, 5, 4, -2)

[[maybe_unused]] constexpr TileCfg kBfpTiles[] = {
#define QMK_BFP_ENTRY(id, wgm, wgn, tm, tn, depth) {wgm, wgn, tm, tn, BK},
    QMK_BF16P_TILE_LIST(QMK_BFP_ENTRY)
#undef QMK_BFP_ENTRY
};
[[maybe_unused]] constexpr int kBfpDepth[] = {
#define QMK_BFP_DEPTH(id, wgm, wgn, tm, tn, depth) depth,
    QMK_BF16P_TILE_LIST(QMK_BFP_DEPTH)
#undef QMK_BFP_DEPTH
};

template <bool A_MN, typename TD, int SCR, int WGM, int WGN, int TM, int TN, int DEPTH>
hipError_t run_bfp_tile(const GemmArgs& g, hipStream_t s) {
  constexpr int BM = 16 * WGM * TM, BN = 16 * WGN * TN;
  const int nM = static_cast<int>((g.M + BM - 1) / BM), nN = static_cast<int>((g.N + BN - 1) / BN);
  if (nM <= 0 || nN <= 0) return hipSuccess;
  hipLaunchKernelGGL((gemm_bf16p_kernel<A_MN, TD, WGM, WGN, TM, TN, DEPTH, SCR>), grid_of(g, nM, nN),
                     dim3(64 * WGM * WGN),
                     0, s, g, nM, nN);
  return hipGetLastError();
}

template <bool A_MN, typename TD, int WGM, int WGN, int TM, int TN, int DEPTH>
hipError_t run_bfp_tile_persist(const BfpPersist& pl, hipStream_t s) {
  auto k = gemm_bf16p_persist<A_MN, TD, WGM, WGN, TM, TN, DEPTH>;
  if (pl.occupancy) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, 64 * WGM * WGN, 0);
    *pl.occupancy = (e == hipSuccess && n > 0) ? n : 1;
    return e;
  }
  if (pl.n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k, dim3(pl.grid), dim3(64 * WGM * WGN), 0, s, pl.jobs, pl.items, pl.n_items);
  return hipGetLastError();
}

template <bool A_MN, typename TD>
hipError_t run_bfp_persist(int cfg, const BfpPersist& pl, hipStream_t s) {
  switch (cfg) {
#define QMK_BFP_PCASE(id, wgm, wgn, tm, tn, depth) \
  case id:                                         \
    return run_bfp_tile_persist<A_MN, TD, wgm, wgn, tm, tn, depth>(pl, s);
    QMK_BF16P_TILE_LIST(QMK_BFP_PCASE)
#undef QMK_BFP_PCASE
    default:
      return hipErrorInvalidValue;
  }
}

template <bool A_MN, typename TD, int SCR>
hipError_t run_bfp(int cfg, const GemmArgs& g, hipStream_t s) {
  switch (cfg) {
#define QMK_BFP_CASE(id, wgm, wgn, tm, tn, depth) \
  case id:                                        \
    return run_bfp_tile<A_MN, TD, SCR, wgm, wgn, tm, tn, depth>(g, s);
    QMK_BF16P_TILE_LIST(QMK_BFP_CASE)
#undef QMK_BFP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

#ifdef QMK_GEMM_UNIT
#if QMK_GEMM_UNIT == 1
hipError_t bf16p_unit_fwd(int cfg, const GemmArgs& g, int o32, int scr, hipStream_t s) {
  if (scr) return o32 ? run_bfp<true, float, 2>(cfg, g, s) : run_bfp<true, double, 2>(cfg, g, s);
  return o32 ? run_bfp<true, float, 0>(cfg, g, s) : run_bfp<true, double, 0>(cfg, g, s);
}
hipError_t bf16p_unit_fwd_persist(int cfg, const BfpPersist& pl, int o32, hipStream_t s) {
  return o32 ? run_bfp_persist<true, float>(cfg, pl, s) : run_bfp_persist<true, double>(cfg, pl, s);
}
#endif
#if QMK_GEMM_UNIT == 2
hipError_t bf16p_unit_gbar(int cfg, const GemmArgs& g, int scr, hipStream_t s) {
  return scr ? run_bfp<false, float, 3>(cfg, g, s) : run_bfp<false, float, 0>(cfg, g, s);
}
hipError_t bf16p_unit_gbar_persist(int cfg, const BfpPersist& pl, hipStream_t s) {
  return run_bfp_persist<false, float>(cfg, pl, s);
}
#endif
#if QMK_GEMM_UNIT == 3
hipError_t bf16p_unit_dc(int cfg, const GemmArgs& g, int scr, hipStream_t s) {
  return scr ? run_bfp<true, double, 4>(cfg, g, s) : run_bfp<true, double, 0>(cfg, g, s);
}
hipError_t bf16p_unit_dc_persist(int cfg, const BfpPersist& pl, hipStream_t s) {
  return run_bfp_persist<true, double>(cfg, pl, s);
}
#endif
#else
// The three products are instantiated in their own translation units (this
// file compiled with QMK_GEMM_UNIT = 1..3); the unit without it holds the
// tile table and the dispatch.
hipError_t bf16p_unit_fwd(int cfg, const GemmArgs& g, int o32, int scr, hipStream_t s);
hipError_t bf16p_unit_gbar(int cfg, const GemmArgs& g, int scr, hipStream_t s);
hipError_t bf16p_unit_dc(int cfg, const GemmArgs& g, int scr, hipStream_t s);
hipError_t bf16p_unit_fwd_persist(int cfg, const BfpPersist& pl, int o32, hipStream_t s);
hipError_t bf16p_unit_gbar_persist(int cfg, const BfpPersist& pl, hipStream_t s);
hipError_t bf16p_unit_dc_persist(int cfg, const BfpPersist& pl, hipStream_t s);

int gemm_bf16p_blocks_per_cu(GemmKind kind, int cfg, int out_is_f32) {
  int n = 1;
  if (launch_gemm_bf16p_persist(kind, cfg, nullptr, nullptr, 0, 0, out_is_f32, &n, nullptr) != hipSuccess) return 1;
  return n;
}

int gemm_bf16p_num_tiles() { return sizeof(kBfpTiles) / sizeof(kBfpTiles[0]); }
TileCfg gemm_bf16p_tile(int cfg) { return kBfpTiles[cfg]; }
size_t gemm_bf16p_tile_lds_bytes(int cfg) {
  const TileCfg& t = kBfpTiles[cfg];
  const int bm = 16 * t.wgm * t.tm, bn = 16 * t.wgn * t.tn;
  const int rs = ring_stages(kBfpDepth[cfg]);
  if (rs > 0) return static_cast<size_t>(rs) * (bm + bn) * BK * 4;  // ring
  // the larger of the two staging layouts of A (MN-major for the forward and
  // W^T ao products, K-major for the W C product)
  const size_t a = std::max<size_t>(static_cast<size_t>(BK) * mn_pitch(bm), static_cast<size_t>(bm) * KLD);
  return 2 * 2 * (a + static_cast<size_t>(bn) * KLD) * 2;
}

// forward: A = AO planes (MN-major), B = C planes [n][k]
// Gbar:    A = C^T planes [k][n] (K-major), B = W planes [p][c][n]
// dC:      A = W planes (MN-major over n), B = AO planes (K-major over p)
bool gemm_bf16p_args_ok(int cfg, const GemmArgs& g) {
  if (cfg < 0 || cfg >= gemm_bf16p_num_tiles()) return false;
  // the loaders address a tile's chunks by 32-bit byte offsets from the
  // tile's base: (rows - 1) * row stride + (BK - 1) * reduction stride + 8
  const TileCfg& t = kBfpTiles[cfg];
  const int64_t ea = (16 * t.wgm * t.tm - 1) * g.sAi + (BK - 1) * g.sAl + 8;
  const int64_t eb = (16 * t.wgn * t.tn - 1) * g.sBj + (BK - 1) * g.sBl + 8;
  return ea >= 0 && eb >= 0 && 2 * ea <= 0x7fffffffLL && 2 * eb <= 0x7fffffffLL;
}

hipError_t launch_gemm_bf16p_persist(GemmKind kind, int cfg, const GemmArgs* jobs, const WorkItem* items,
                                     int n_items, int grid, int out_is_f32, int* occupancy, hipStream_t s) {
  if (cfg < 0 || cfg >= gemm_bf16p_num_tiles()) return hipErrorInvalidValue;
  const BfpPersist pl{jobs, items, n_items, grid, occupancy};
  switch (kind) {
    case GemmKind::kForward: return bf16p_unit_fwd_persist(cfg, pl, out_is_f32, s);
    case GemmKind::kGbar: return bf16p_unit_gbar_persist(cfg, pl, s);
    case GemmKind::kDcoef: return bf16p_unit_dc_persist(cfg, pl, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm_bf16p(GemmKind kind, int cfg, const GemmArgs& g, int out_is_f32, int screened,
                             hipStream_t s) {
  if (!gemm_bf16p_args_ok(cfg, g)) return hipErrorInvalidValue;
  switch (kind) {
    case GemmKind::kForward: return bf16p_unit_fwd(cfg, g, out_is_f32, screened, s);
    case GemmKind::kGbar: return bf16p_unit_gbar(cfg, g, screened, s);
    case GemmKind::kDcoef:
      // the screened step list holds at most kSparseMaxStages steps of BK points
      if (screened && (g.Lchunk > static_cast<int64_t>(kSparseMaxStages) * BK || g.Lchunk % 64 != 0))
        return hipErrorInvalidValue;
      return bf16p_unit_dc(cfg, g, screened, s);
    default: return hipErrorInvalidValue;
  }
}

#endif  // QMK_GEMM_UNIT

}  // namespace qmk
