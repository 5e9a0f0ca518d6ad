// AO value / gradient / Laplacian kernels (QMCkl paper, Section 3.1).
//
// Mapping: one lane per point, so every store of one (AO, component) pair by
// a wavefront covers 64 consecutive points (coalesced along the point axis
// of the [ao][5][point] layout).  A block serves 256 points and one group
// of nuclei: it stages that group's nucleus, shell and primitive tables in
// LDS, then walks the nuclei in order.  For each nucleus the wavefront
// takes one ballot on gmin*u < T (the per-nucleus radius of Section 3.1 in
// squared form); if no lane is inside, the nucleus' AOs are stored as zeros
// without touching a primitive.  Inside a shell the primitives are sorted by
// ascending exponent, so once gamma*u >= T holds for every lane the rest of
// the shell is skipped (Section 3.1, early exit after the first negligible
// primitive).  Radial sums g0 = R, g1 = dR/du, g2 = d2R/du2 live in
// registers; powers of the displacement are built by repeated
// multiplication (Section 3.1, angular part) and never stored.
//
// The value-only form (VAL = true) serves the MO values and the density on a
// grid (Section 5.4, orbital visualisation): it accumulates only g0 and stores
// one [ao][point] plane.
#include <type_traits>

#include "qmk_internal.h"

namespace qmk {
namespace {

template <typename T>
__device__ __forceinline__ void st(T* p, double v, int64_t) { *p = static_cast<T>(v); }

// BF16x3 mode: the AO array is stored as two bf16 planes, hi = bf16(x) and
// lo = bf16(x - hi) of the FP32-rounded value x, the lo plane `plane`
// elements after the hi plane.  The two lanes of each even/odd pair swap one
// half, so that every lane writes one 32-bit word: the even lane the hi
// values of its point and the next, the odd lane the lo values of the
// previous point and its own.  A wave's store therefore covers 128 bytes of
// each plane, and both lanes of every pair must take part.  The odd lane's
// output pointer already points at its word of the lo plane (the kernel
// moves it by plane - 1 elements once), so `plane` is not used here.
struct Bf16Pair {
  uint16_t bits;
};
__device__ __forceinline__ void st(Bf16Pair* p, double v, int64_t) {
  float f = static_cast<float>(v);
  // hi is the bf16 rounding of the FP32 value: without this barrier the two
  // conversions would be merged into one FP64 -> bf16 rounding
  asm volatile("" : "+v"(f));
  const __bf16 h = static_cast<__bf16>(f);
  const __bf16 l = static_cast<__bf16>(f - static_cast<float>(h));
  const uint32_t pk = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, h)) |
                      (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, l)) << 16);
  // quad_perm [1, 0, 3, 2]: the neighbouring lane's (hi, lo) pair
  const uint32_t rp = static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(pk), 0xB1, 0xF, 0xF, true));
  // bytes 0-3 of the selection are pk, 4-7 rp: the even lane takes (pk.hi,
  // rp.hi), the odd lane (rp.lo, pk.lo)
  const uint32_t sel = (threadIdx.x & 1) ? 0x03020706u : 0x05040100u;
  *reinterpret_cast<uint32_t*>(p) = __builtin_amdgcn_perm(rp, pk, sel);
}
// The same split of a value already in FP32.
__device__ __forceinline__ void st(Bf16Pair* p, float f, int64_t) {
  const __bf16 h = static_cast<__bf16>(f);
  const __bf16 l = static_cast<__bf16>(f - static_cast<float>(h));
  const uint32_t pk = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, h)) |
                      (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, l)) << 16);
  const uint32_t rp = static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(pk), 0xB1, 0xF, 0xF, true));
  const uint32_t sel = (threadIdx.x & 1) ? 0x03020706u : 0x05040100u;
  *reinterpret_cast<uint32_t*>(p) = __builtin_amdgcn_perm(rp, pk, sel);
}

// Arithmetic type of the AO values: FP64, except for the split planes, whose
// hi / lo pair represents the FP32 rounding of a value to 16 significant bits
// (FP32 arithmetic errors stay far below that).
template <typename OutT>
struct AoCalc {
  typedef double type;
};
template <>
struct AoCalc<Bf16Pair> {
  typedef float type;
};

template <typename CT>
struct AxisT {
  CT v0, v1, v2, v3;
};
// Derivatives of t^e (e = 0..3, wave-uniform), given t, t^2, t^3: v0 = t^e,
// v1 = e t^(e-1), v2 = e(e-1) t^(e-2), v3 = e(e-1)(e-2) t^(e-3).
template <typename CT>
__device__ __forceinline__ AxisT<CT> axis_derivs_t(int e, CT t, CT t2, CT t3) {
  if (e == 0) return AxisT<CT>{CT(1), CT(0), CT(0), CT(0)};
  if (e == 1) return AxisT<CT>{t, CT(1), CT(0), CT(0)};
  if (e == 2) return AxisT<CT>{t2, CT(2) * t, CT(2), CT(0)};
  return AxisT<CT>{t3, CT(3) * t2, CT(6) * t, CT(6)};
}

// Stores value, gradient and Laplacian of the (l+1)(l+2)/2 Cartesian AOs of
// one shell for this lane's point.  l is wave-uniform; the components run in
// a uniform loop, one at a time, which keeps register pressure low.
//   chi      = M P g0
//   d_i chi  = M (d_i P g0 + 2 d_i P g1)          (d_i: displacement)
//   lap chi  = M (lap P g0 + (4l+6) P g1 + 4 u P g2)
template <typename OutT, typename CT = typename AoCalc<OutT>::type>
__device__ __forceinline__ void shell_vgl(int l, CT dx, CT dy, CT dz, CT u, CT g0, CT g1, CT g2,
                                          const double* __restrict__ M, OutT* __restrict__ o,
                                          int64_t sK, int64_t sC, int64_t plane) {
  const CT lapr = CT(4 * l + 6) * g1 + CT(4) * u * g2;
  const CT tg1 = CT(2) * g1;
  const CT dx2 = dx * dx, dy2 = dy * dy, dz2 = dz * dz;
  const CT dx3 = dx2 * dx, dy3 = dy2 * dy, dz3 = dz2 * dz;
  // components (a, b, c) with a descending, then b descending, in one loop
  const int ncart = (l + 1) * (l + 2) / 2;
  int a = l, b = 0;
#pragma unroll 1
  for (int idx = 0; idx < ncart; ++idx) {
    {
      const int c = l - a - b;
      const AxisT<CT> X = axis_derivs_t(a, dx, dx2, dx3);
      const AxisT<CT> Y = axis_derivs_t(b, dy, dy2, dy3);
      const AxisT<CT> Z = axis_derivs_t(c, dz, dz2, dz3);
      const CT yz = Y.v0 * Z.v0;
      const CT P = X.v0 * yz;
      const CT lapP = X.v2 * yz + X.v0 * (Y.v2 * Z.v0 + Y.v0 * Z.v2);
      const CT m = static_cast<CT>(M[idx]);
      const CT tp = P * tg1;
      OutT* q = o + idx * sK;
      st(q, m * P * g0, plane);
      st(q + sC, m * (X.v1 * yz * g0 + dx * tp), plane);
      st(q + 2 * sC, m * (X.v0 * Y.v1 * Z.v0 * g0 + dy * tp), plane);
      st(q + 3 * sC, m * (X.v0 * Y.v0 * Z.v1 * g0 + dz * tp), plane);
      st(q + 4 * sC, m * (lapP * g0 + P * lapr), plane);
    }
    if (b > 0) {
      --b;
    } else {
      --a;
      b = l - a;
    }
  }
}

// Values only: chi = M P g0.
template <typename OutT>
__device__ __forceinline__ void shell_value(int l, double dx, double dy, double dz, double g0,
                                            const double* __restrict__ M, OutT* __restrict__ o,
                                            int64_t sK) {
  const double dx2 = dx * dx, dy2 = dy * dy, dz2 = dz * dz;
  const double dx3 = dx2 * dx, dy3 = dy2 * dy, dz3 = dz2 * dz;
  int idx = 0;
#pragma unroll 1
  for (int a = l; a >= 0; --a) {
#pragma unroll 1
    for (int b = l - a; b >= 0; --b, ++idx) {
      const int c = l - a - b;
      const double px = a == 0 ? 1.0 : (a == 1 ? dx : (a == 2 ? dx2 : dx3));
      const double py = b == 0 ? 1.0 : (b == 1 ? dy : (b == 2 ? dy2 : dy3));
      const double pz = c == 0 ? 1.0 : (c == 1 ? dz : (c == 2 ? dz2 : dz3));
      st(o + idx * sK, M[idx] * (px * py * pz) * g0, 0);
    }
  }
}

template <typename OutT, bool VAL>
__device__ __forceinline__ void shell_zero(int l, OutT* __restrict__ o, int64_t sK, int64_t sC,
                                           int64_t plane, bool store) {
  if (!store) return;
  const int n = (l + 1) * (l + 2) / 2;
  for (int i = 0; i < n; ++i) {
    OutT* q = o + i * sK;
#pragma unroll
    for (int c = 0; c < (VAL ? 1 : 5); ++c) st(q + c * sC, 0.0, plane);
  }
}

// SCR = 0: dense.  SCR = 1: activity pass of the screened evaluation: marks
// in out.act the 16-AO chunks in which some point of the wave's 64-point
// block has a primitive inside the cutoff (the first, smallest exponent
// decides, as in the radial sums) and stores nothing.  SCR = 2: screened
// store: a shell whose chunks are all inactive is neither evaluated nor
// stored, unless one of them was active in the previous evaluation into the
// same array (out.act_prev), in which case it is stored as zeros.  So every
// inactive chunk of the array holds zeros without being written again, and
// an active chunk holds all of its values.
template <typename OutT, bool VAL, int SCR = 0>
__device__ __forceinline__ void ao_vgl_body(const AoTables& t, const PointArgs& pts,
                                            const AoOut& out, int bx, int gy,
                                            unsigned char* smem) {
  const NucGroup g = t.group[gy];
  const int np = g.p_end - g.p_begin, ns = g.sh_end - g.sh_begin, nn = g.nuc_end - g.nuc_begin;
  PrimDev* s_prim = reinterpret_cast<PrimDev*>(smem);
  ShellDev* s_shell = reinterpret_cast<ShellDev*>(s_prim + np);
  NucDev* s_nuc = reinterpret_cast<NucDev*>(s_shell + ns);
  for (int i = threadIdx.x; i < np; i += blockDim.x) s_prim[i] = t.prim[g.p_begin + i];
  for (int i = threadIdx.x; i < ns; i += blockDim.x) s_shell[i] = t.shell[g.sh_begin + i];
  for (int i = threadIdx.x; i < nn; i += blockDim.x) s_nuc[i] = t.nuc[g.nuc_begin + i];
  __syncthreads();

  const int64_t p = static_cast<int64_t>(bx) * blockDim.x + threadIdx.x;
  const bool valid = p < pts.P;
  double rx = 0.0, ry = 0.0, rz = 0.0;
  if (valid) {
    const int64_t src = pts.perm ? static_cast<int64_t>(pts.perm[p]) : p;
    rx = pts.coord[src * pts.s_pt];
    ry = pts.coord[src * pts.s_pt + pts.s_ax];
    rz = pts.coord[src * pts.s_pt + 2 * pts.s_ax];
  }
  constexpr bool kPairs = std::is_same<OutT, Bf16Pair>::value;
  // split planes: the odd lane of each pair writes the lo plane, one point back
  OutT* const obase = static_cast<OutT*>(out.out) + p * out.sP +
                      ((kPairs && (threadIdx.x & 1)) ? out.plane - 1 : 0);
  const double T = t.T;

  for (int a = 0; a < nn; ++a) {
    const NucDev nu = s_nuc[a];
    const double dx = rx - nu.x, dy = ry - nu.y, dz = rz - nu.z;
    const double u = dist2(dx, dy, dz);
    const bool near = valid && (nu.gmin * u < T);
    if constexpr (SCR == 1) {
      if (!__any(near)) continue;
      for (int s = nu.sh_begin; s < nu.sh_end; ++s) {
        const ShellDev sh = s_shell[s];
        const bool on0 = near && sh.p_begin < sh.p_end && (s_prim[sh.p_begin].gamma * u < T);
        if (__any(on0) && (threadIdx.x & 63) == 0) {
          uint32_t* const w = out.act + (p >> 6) * out.act_words;
          const int c0 = sh.ao_off / kSparseChunk;
          const int c1 = (sh.ao_off + (sh.l + 1) * (sh.l + 2) / 2 - 1) / kSparseChunk;
          for (int c = c0; c <= c1; ++c) atomicOr(w + (c >> 5), 1u << (c & 31));
        }
      }
      continue;
    }
    const bool any_near = __any(near);
    if (SCR == 0 && !any_near) {
      for (int s = nu.sh_begin; s < nu.sh_end; ++s) {
        const ShellDev sh = s_shell[s];
        shell_zero<OutT, VAL>(sh.l, obase + sh.ao_off * out.sK, out.sK, out.sC, out.plane, valid || kPairs);
      }
      continue;
    }
    for (int s = nu.sh_begin; s < nu.sh_end; ++s) {
      const ShellDev sh = s_shell[s];
      if constexpr (SCR == 2) {
        // the wave's block: chunks of this shell active now, or before
        const int64_t blk = (static_cast<int64_t>(bx) * blockDim.x + (threadIdx.x & ~63)) >> 6;
        const int c0 = sh.ao_off / kSparseChunk;
        const int c1 = (sh.ao_off + (sh.l + 1) * (sh.l + 2) / 2 - 1) / kSparseChunk;
        bool now = false, was = false;
        for (int c = c0; c <= c1; ++c) {
          now = now || ((out.act[blk * out.act_words + (c >> 5)] >> (c & 31)) & 1u);
          was = was || ((out.act_prev[blk * out.act_words + (c >> 5)] >> (c & 31)) & 1u);
        }
        if (!now || !any_near) {
          if (now || was)
            shell_zero<OutT, VAL>(sh.l, obase + sh.ao_off * out.sK, out.sK, out.sC, out.plane, valid || kPairs);
          continue;
        }
      }
      typedef typename AoCalc<OutT>::type CT;  // the radial sums' arithmetic type
      CT g0 = CT(0), g1 = CT(0), g2 = CT(0);
      for (int k = sh.p_begin; k < sh.p_end; ++k) {
        const PrimDev pr = s_prim[k];
        const double x = pr.gamma * u;  // the cutoff test in FP64 in every mode
        const bool on = near && (x < T);
        if (!__any(on)) break;  // ascending exponents: every later one is cut too
        if (on) {
          const CT gm = static_cast<CT>(pr.gamma);
          const CT e = static_cast<CT>(pr.coef) * exp(static_cast<CT>(-x));
          g0 += e;
          g1 -= gm * e;
          g2 += gm * gm * e;
        }
      }
      // (the split-plane store needs both lanes of every pair: lanes past the
      // last point store the zeros their empty sums give)
      if (valid || kPairs) {
        if (VAL)
          shell_value(__builtin_amdgcn_readfirstlane(sh.l), dx, dy, dz, static_cast<double>(g0),
                      t.ao_factor + sh.ao_off, obase + sh.ao_off * out.sK, out.sK);
        else
          shell_vgl<OutT>(__builtin_amdgcn_readfirstlane(sh.l), static_cast<CT>(dx), static_cast<CT>(dy),
                          static_cast<CT>(dz), static_cast<CT>(u), g0, g1, g2, t.ao_factor + sh.ao_off,
                          obase + sh.ao_off * out.sK, out.sK, out.sC, out.plane);
      }
    }
  }
}

template <typename OutT, bool VAL, int SCR = 0>
__global__ __launch_bounds__(256, 4) void ao_vgl_kernel(AoTables t, PointArgs pts, AoOut out) {
  extern __shared__ __align__(16) unsigned char smem[];
  ao_vgl_body<OutT, VAL, SCR>(t, pts, out, blockIdx.x, blockIdx.y, smem);
}

// Persistent form: the grid walks a list of (molecule, point block, group).
template <typename OutT>
__global__ __launch_bounds__(256) void ao_vgl_persist(const AoJob* __restrict__ jobs,
                                                      const WorkItem* __restrict__ items,
                                                      int n_items) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const WorkItem it = items[i];
    const AoJob& j = jobs[it.job];
    ao_vgl_body<OutT, false>(j.t, j.pts, j.out, it.a, it.b, smem);
    __syncthreads();  // LDS is restaged by the next item
  }
}

}  // namespace

hipError_t launch_ao_vgl_persist(const AoJob* jobs, const WorkItem* items, int n_items, int grid,
                                 size_t smem, int out_is_f32, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (out_is_f32 == 2)
    hipLaunchKernelGGL(ao_vgl_persist<Bf16Pair>, dim3(grid), dim3(256), smem, s, jobs, items, n_items);
  else if (out_is_f32)
    hipLaunchKernelGGL(ao_vgl_persist<float>, dim3(grid), dim3(256), smem, s, jobs, items, n_items);
  else
    hipLaunchKernelGGL(ao_vgl_persist<double>, dim3(grid), dim3(256), smem, s, jobs, items, n_items);
  return hipGetLastError();
}

int ao_persist_blocks_per_cu(int f32, size_t smem) {
  int n = 0;
  hipError_t e = f32 == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ao_vgl_persist<Bf16Pair>, 256, smem)
                 : f32    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ao_vgl_persist<float>, 256, smem)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ao_vgl_persist<double>, 256, smem);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_ao_vgl(const AoTables& t, const PointArgs& pts, const AoOut& out, int out_is_f32,
                         int fp32_compute, hipStream_t s) {
  (void)fp32_compute;
  if (pts.P <= 0 || t.n_groups <= 0) return hipSuccess;
  const size_t smem = static_cast<size_t>(t.smem_bytes);
  dim3 grid(static_cast<unsigned>((pts.P + 255) / 256), static_cast<unsigned>(t.n_groups));
  if (out_is_f32 == 2)
    hipLaunchKernelGGL((ao_vgl_kernel<Bf16Pair, false>), grid, dim3(256), smem, s, t, pts, out);
  else if (out_is_f32)
    hipLaunchKernelGGL((ao_vgl_kernel<float, false>), grid, dim3(256), smem, s, t, pts, out);
  else
    hipLaunchKernelGGL((ao_vgl_kernel<double, false>), grid, dim3(256), smem, s, t, pts, out);
  return hipGetLastError();
}

hipError_t launch_ao_vgl_screened(const AoTables& t, const PointArgs& pts, const AoOut& out, int out_is_f32,
                                  hipStream_t s) {
  if (pts.P <= 0 || t.n_groups <= 0) return hipSuccess;
  if (!out.act || !out.act_prev) return hipErrorInvalidValue;
  const size_t smem = static_cast<size_t>(t.smem_bytes);
  dim3 grid(static_cast<unsigned>((pts.P + 255) / 256), static_cast<unsigned>(t.n_groups));
  // activity first: a chunk's bit may come from a shell of another nucleus
  // group, so the stores of the second pass need the whole bitmap
  hipLaunchKernelGGL((ao_vgl_kernel<double, false, 1>), grid, dim3(256), smem, s, t, pts, out);
  if (out_is_f32 == 2)
    hipLaunchKernelGGL((ao_vgl_kernel<Bf16Pair, false, 2>), grid, dim3(256), smem, s, t, pts, out);
  else if (out_is_f32)
    hipLaunchKernelGGL((ao_vgl_kernel<float, false, 2>), grid, dim3(256), smem, s, t, pts, out);
  else
    hipLaunchKernelGGL((ao_vgl_kernel<double, false, 2>), grid, dim3(256), smem, s, t, pts, out);
  return hipGetLastError();
}

hipError_t launch_ao_value(const AoTables& t, const PointArgs& pts, const AoOut& out, int out_is_f32,
                           hipStream_t s) {
  if (pts.P <= 0 || t.n_groups <= 0) return hipSuccess;
  const size_t smem = static_cast<size_t>(t.smem_bytes);
  dim3 grid(static_cast<unsigned>((pts.P + 255) / 256), static_cast<unsigned>(t.n_groups));
  if (out_is_f32)
    hipLaunchKernelGGL((ao_vgl_kernel<float, true>), grid, dim3(256), smem, s, t, pts, out);
  else
    hipLaunchKernelGGL((ao_vgl_kernel<double, true>), grid, dim3(256), smem, s, t, pts, out);
  return hipGetLastError();
}

}  // namespace qmk
