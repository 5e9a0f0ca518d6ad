// Adjoint AO stage: gradients of L = sum(W * mo_vgl) with respect to the
// electron and nuclear coordinates.  Force estimators need derivatives of
// the orbitals up to third order (QMCkl paper, Section 3.6); parameter
// derivatives are the other use (Section 3.5, last paragraph).
//
// With Gbar[k][c][p] = sum_n W[p][c][n] C[n][k] (an MFMA product), the
// contribution of AO k at point p to dL/dr_i is
//   t_i = Gbar0 d_i chi + sum_j Gbar(1+j) d_i d_j chi + Gbar4 d_i lap chi,
// and because chi depends on r - R_A only, nucleus A receives -t_i.
// The AO derivatives are recomputed here from the coordinates (radial sums
// g0..g3 and angular monomials in registers), never stored.  The mapping
// matches the forward AO kernel: one lane per point, the nucleus group's
// tables staged in LDS, one ballot per nucleus on the cutoff radius, and an
// early exit over the ascending exponents.  Reductions are deterministic:
// per-wave nucleus sums are written to a partial array and summed in a
// fixed order by a second kernel.
#include "qmk_internal.h"

namespace qmk {
namespace {

// Contracts the third-order AO derivatives of one shell with Gbar.  l is
// wave-uniform; the Cartesian components of each l are unrolled at compile
// time (adj_components), so every power of the displacement is a known
// product rather than a run-time selection.
//   d_i chi     = M (P_i g0 + 2 d_i P g1)
//   d_i d_j chi = M (P_ij g0 + 2 (d_j P_i + d_i P_j) g1 + 2 delta_ij P g1
//                    + 4 d_i d_j P g2)
//   d_i lap chi = M (lapP_i g0 + (2 d_i lapP + (4l+6) P_i) g1
//                    + ((8l+20) d_i P + 4 u P_i) g2 + 8 u d_i P g3)
// Summed against Gbar as  sum_j Gj d_i d_j chi  =  M (g0 (Hess P . G)_i
//   + 2 g1 (P_i (G.d) + d_i (G.grad P) + G_i P) + 4 g2 d_i P (G.d)).
// The five Gbar values of a component are loaded one component ahead (those
// of the first component before the radial sums, by the caller), so that
// their latency overlaps the arithmetic.  At 800 AOs x 143,360 points the
// unrolled form takes 0.89 ms (FP64), against 1.09 ms for a run-time
// component loop with selected powers.
// The arithmetic type is Gbar's: with FP32 Gbar (the mixed-precision modes)
// the radial sums and the derivative contraction run in FP32 (0.47 ms; 0.71
// ms with FP64 arithmetic on the same FP32 Gbar, loaded where used); the
// point-nucleus distances, the cutoff decisions and the sums over shells and
// nuclei stay FP64.
template <typename GT>
__device__ __forceinline__ void load_gbar(const GT* __restrict__ q, int64_t sC, GT* G) {
#pragma unroll
  for (int c = 0; c < 5; ++c) G[c] = q[c * sC];
}

// Cartesian component `idx` of a shell of angular momentum l: (a, b, l-a-b)
// with a descending, then b descending.
constexpr int cart_a(int l, int idx) {
  int a = l;
  while (idx > l - a) {
    idx -= l - a + 1;
    --a;
  }
  return a;
}
constexpr int cart_b(int l, int idx) {
  int a = l;
  while (idx > l - a) {
    idx -= l - a + 1;
    --a;
  }
  return l - a - idx;
}

// Derivatives of t^E (E known at compile time) of order 0..3.
template <typename CT>
struct AxisT {
  CT v0, v1, v2, v3;
};
template <int E, typename CT>
__device__ __forceinline__ AxisT<CT> axis_c(CT t, CT t2, CT t3) {
  AxisT<CT> r;
  if constexpr (E == 0) {
    r = AxisT<CT>{CT(1), CT(0), CT(0), CT(0)};
  } else if constexpr (E == 1) {
    r = AxisT<CT>{t, CT(1), CT(0), CT(0)};
  } else if constexpr (E == 2) {
    r = AxisT<CT>{t2, CT(2) * t, CT(2), CT(0)};
  } else {
    r = AxisT<CT>{t3, CT(3) * t2, CT(6) * t, CT(6)};
  }
  return r;
}

// Shell quantities shared by its components (CT: the arithmetic type).
template <typename CT>
struct ShellRadial {
  CT dx, dy, dz, dx2, dy2, dz2, dx3, dy3, dz3;
  CT g0, g1, g2, tg1, fg2, fug2, eug3, c1, c2;
};

// Component I of a shell of angular momentum L, then the rest: the powers of
// the displacement are compile-time choices (no selects), and the component
// loop is unrolled per L.
// Gc holds the component's five Gbar values, loaded one component ahead
// (the first component's by the caller, before the radial sums), so that the
// loads overlap the arithmetic.  A compiler barrier closes each component,
// so that the unrolled components do not pile their loads and temporaries
// up at once.
template <typename GT, int L, int I>
__device__ __forceinline__ void adj_components(const ShellRadial<GT>& r, const double* __restrict__ M,
                                               const GT* __restrict__ gb, int64_t sK, int64_t sC,
                                               const GT* Gc, GT& tx, GT& ty, GT& tz) {
  typedef GT CT;
  if constexpr (I < (L + 1) * (L + 2) / 2) {
    constexpr int a = cart_a(L, I), b = cart_b(L, I), c = L - a - b;
    CT G[5], Gn[5] = {CT(0), CT(0), CT(0), CT(0), CT(0)};
#pragma unroll
    for (int q = 0; q < 5; ++q) G[q] = Gc[q];
    if constexpr (I + 1 < (L + 1) * (L + 2) / 2) load_gbar(gb + (I + 1) * sK, sC, Gn);
    // fresh copies of the powers: without them common products of different
    // components would be kept alive across the whole shell
    CT px = r.dx, px2 = r.dx2, px3 = r.dx3, py = r.dy, py2 = r.dy2, py3 = r.dy3, pz = r.dz, pz2 = r.dz2,
       pz3 = r.dz3;
    asm volatile("" : "+v"(px), "+v"(px2), "+v"(px3), "+v"(py), "+v"(py2), "+v"(py3), "+v"(pz), "+v"(pz2),
                 "+v"(pz3));
    const AxisT<CT> X = axis_c<a>(px, px2, px3);
    const AxisT<CT> Y = axis_c<b>(py, py2, py3);
    const AxisT<CT> Z = axis_c<c>(pz, pz2, pz3);
    const CT G0 = G[0], G1 = G[1], G2 = G[2], G3 = G[3], G4 = G[4];
    const CT P = X.v0 * Y.v0 * Z.v0;
    const CT Px = X.v1 * Y.v0 * Z.v0, Py = X.v0 * Y.v1 * Z.v0, Pz = X.v0 * Y.v0 * Z.v1;
    const CT Pxx = X.v2 * Y.v0 * Z.v0, Pyy = X.v0 * Y.v2 * Z.v0, Pzz = X.v0 * Y.v0 * Z.v2;
    const CT Pxy = X.v1 * Y.v1 * Z.v0, Pxz = X.v1 * Y.v0 * Z.v1, Pyz = X.v0 * Y.v1 * Z.v1;
    const CT lapP = Pxx + Pyy + Pzz;
    const CT lPx = X.v3 * Y.v0 * Z.v0 + X.v1 * (Y.v2 * Z.v0 + Y.v0 * Z.v2);
    const CT lPy = Y.v3 * X.v0 * Z.v0 + Y.v1 * (X.v2 * Z.v0 + X.v0 * Z.v2);
    const CT lPz = Z.v3 * X.v0 * Y.v0 + Z.v1 * (X.v2 * Y.v0 + X.v0 * Y.v2);
    const CT Gd = G1 * r.dx + G2 * r.dy + G3 * r.dz;
    const CT GdP = G1 * Px + G2 * Py + G3 * Pz;
    const CT HGx = Pxx * G1 + Pxy * G2 + Pxz * G3;
    const CT HGy = Pxy * G1 + Pyy * G2 + Pyz * G3;
    const CT HGz = Pxz * G1 + Pyz * G2 + Pzz * G3;
    const CT m = static_cast<CT>(M[I]);
    // per direction i: G0 d_i chi + sum_j Gj d_i d_j chi + G4 d_i lap chi (over M)
    const CT Pg = P * Gd * r.fg2, Pe = P * r.eug3, Pl = P * r.c2 * r.g2;
    tx += m * (G0 * (Px * r.g0 + r.dx * P * r.tg1) + r.g0 * HGx + r.tg1 * (Px * Gd + r.dx * GdP + G1 * P) +
               r.dx * Pg + G4 * (lPx * r.g0 + (CT(2) * r.dx * lapP + r.c1 * Px) * r.g1 + r.dx * Pl + r.fug2 * Px +
                                 r.dx * Pe));
    ty += m * (G0 * (Py * r.g0 + r.dy * P * r.tg1) + r.g0 * HGy + r.tg1 * (Py * Gd + r.dy * GdP + G2 * P) +
               r.dy * Pg + G4 * (lPy * r.g0 + (CT(2) * r.dy * lapP + r.c1 * Py) * r.g1 + r.dy * Pl + r.fug2 * Py +
                                 r.dy * Pe));
    tz += m * (G0 * (Pz * r.g0 + r.dz * P * r.tg1) + r.g0 * HGz + r.tg1 * (Pz * Gd + r.dz * GdP + G3 * P) +
               r.dz * Pg + G4 * (lPz * r.g0 + (CT(2) * r.dz * lapP + r.c1 * Pz) * r.g1 + r.dz * Pl + r.fug2 * Pz +
                                 r.dz * Pe));
    asm volatile("" ::: "memory");  // keeps the next component's loads below this one
    adj_components<GT, L, I + 1>(r, M, gb, sK, sC, Gn, tx, ty, tz);
  }
}

template <typename GT, int L>
__device__ __forceinline__ void shell_adjoint_l(GT dx, GT dy, GT dz, GT u, GT g0, GT g1, GT g2, GT g3,
                                                const double* __restrict__ M, const GT* __restrict__ gb,
                                                int64_t sK, int64_t sC, const GT* G_first, GT& tx, GT& ty,
                                                GT& tz) {
  typedef GT CT;
  ShellRadial<CT> r;
  r.dx = dx;
  r.dy = dy;
  r.dz = dz;
  r.dx2 = dx * dx;
  r.dy2 = dy * dy;
  r.dz2 = dz * dz;
  r.dx3 = r.dx2 * dx;
  r.dy3 = r.dy2 * dy;
  r.dz3 = r.dz2 * dz;
  r.g0 = g0;
  r.g1 = g1;
  r.g2 = g2;
  r.tg1 = CT(2) * g1;
  r.fg2 = CT(4) * g2;
  r.fug2 = CT(4) * u * g2;
  r.eug3 = CT(8) * u * g3;
  r.c1 = CT(4 * L + 6);
  r.c2 = CT(8 * L + 20);
  adj_components<GT, L, 0>(r, M, gb, sK, sC, G_first, tx, ty, tz);
}

// Contracts the shell's third-order AO derivatives with Gbar (l <= 3,
// wave-uniform).
template <typename GT>
__device__ __forceinline__ void shell_adjoint(int l, GT dx, GT dy, GT dz, GT u, GT g0, GT g1, GT g2, GT g3,
                                              const double* __restrict__ M, const GT* __restrict__ gb,
                                              int64_t sK, int64_t sC, const GT* G_first, GT& tx, GT& ty,
                                              GT& tz) {
  switch (l) {
    case 0: shell_adjoint_l<GT, 0>(dx, dy, dz, u, g0, g1, g2, g3, M, gb, sK, sC, G_first, tx, ty, tz); break;
    case 1: shell_adjoint_l<GT, 1>(dx, dy, dz, u, g0, g1, g2, g3, M, gb, sK, sC, G_first, tx, ty, tz); break;
    case 2: shell_adjoint_l<GT, 2>(dx, dy, dz, u, g0, g1, g2, g3, M, gb, sK, sC, G_first, tx, ty, tz); break;
    default: shell_adjoint_l<GT, 3>(dx, dy, dz, u, g0, g1, g2, g3, M, gb, sK, sC, G_first, tx, ty, tz); break;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename GT>
__device__ __forceinline__ void ao_adjoint_body(const AoTables& t, const PointArgs& pts,
                                                const GT* __restrict__ gbar, int64_t sK,
                                                int64_t sC, double* __restrict__ elec_out,
                                                int64_t elec_group_stride,
                                                double* __restrict__ nuc_partial, int bx, int gy,
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
  const int64_t wave = p >> 6;
  const int lane = threadIdx.x & 63;
  const bool valid = p < pts.P;
  // with a point order (screened adjoint), point p of G-bar is point perm[p]
  // of the caller's coordinates and electron gradients
  const int64_t src = valid && pts.perm ? static_cast<int64_t>(pts.perm[p]) : p;
  double rx = 0.0, ry = 0.0, rz = 0.0;
  if (valid) {
    rx = pts.coord[src * pts.s_pt];
    ry = pts.coord[src * pts.s_pt + pts.s_ax];
    rz = pts.coord[src * pts.s_pt + 2 * pts.s_ax];
  }
  const GT* gb_p = gbar + p;
  const double T = t.T;
  double ex = 0.0, ey = 0.0, ez = 0.0;

  for (int a = 0; a < nn; ++a) {
    const NucDev nu = s_nuc[a];
    const double dx = rx - nu.x, dy = ry - nu.y, dz = rz - nu.z;
    const double u = dist2(dx, dy, dz);
    const bool near = valid && (nu.gmin * u < T);
    double tx = 0.0, ty = 0.0, tz = 0.0;
    if (__any(near)) {
      typedef GT CT;  // the arithmetic type of the radial sums and the contraction
      const CT cx = static_cast<CT>(dx), cy = static_cast<CT>(dy), cz = static_cast<CT>(dz);
      const CT cu = static_cast<CT>(u);
      for (int s = nu.sh_begin; s < nu.sh_end; ++s) {
        const ShellDev sh = s_shell[s];
        CT g0 = CT(0), g1 = CT(0), g2 = CT(0), g3 = CT(0);
        CT G_first[5] = {CT(0), CT(0), CT(0), CT(0), CT(0)};
        if (near) load_gbar(gb_p + sh.ao_off * sK, sC, G_first);
        for (int k = sh.p_begin; k < sh.p_end; ++k) {
          const PrimDev pr = s_prim[k];
          const double x = pr.gamma * u;  // the cutoff test in FP64, as in the forward pass
          const bool on = near && (x < T);
          if (!__any(on)) break;
          if (on) {
            const CT gm = static_cast<CT>(pr.gamma);
            const CT e = static_cast<CT>(pr.coef) * exp(static_cast<CT>(-x));
            const CT ge = gm * e;
            g0 += e;
            g1 -= ge;
            g2 += gm * ge;
            g3 -= gm * gm * ge;
          }
        }
        if (near) {
          CT sx = CT(0), sy = CT(0), sz = CT(0);
          shell_adjoint(__builtin_amdgcn_readfirstlane(sh.l), cx, cy, cz, cu, g0, g1, g2, g3,
                        t.ao_factor + sh.ao_off, gb_p + sh.ao_off * sK, sK, sC, G_first, sx, sy, sz);
          tx += static_cast<double>(sx);
          ty += static_cast<double>(sy);
          tz += static_cast<double>(sz);
        }
      }
    }
    ex += tx;
    ey += ty;
    ez += tz;
    const double sx = wave_sum(tx), sy = wave_sum(ty), sz = wave_sum(tz);
    if (lane == 0) {
      double* o = nuc_partial + (wave * t.nucl_dev + g.nuc_begin + a) * 3;
      o[0] = -sx;
      o[1] = -sy;
      o[2] = -sz;
    }
  }
  if (valid) {
    double* o = elec_out + gy * elec_group_stride + src * 3;
    o[0] = ex;
    o[1] = ey;
    o[2] = ez;
  }
}

template <typename GT>
__global__ __launch_bounds__(256) void ao_adjoint_kernel(AoTables t, PointArgs pts,
                                                         const GT* __restrict__ gbar, int64_t sK,
                                                         int64_t sC, double* __restrict__ elec_out,
                                                         int64_t elec_group_stride,
                                                         double* __restrict__ nuc_partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  ao_adjoint_body<GT>(t, pts, gbar, sK, sC, elec_out, elec_group_stride, nuc_partial, blockIdx.x,
                      blockIdx.y, smem);
}

template <typename GT>
__global__ __launch_bounds__(256) void ao_adjoint_persist(const AdjJob* __restrict__ jobs,
                                                          const WorkItem* __restrict__ items,
                                                          int n_items) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    const WorkItem it = items[i];
    const AdjJob& j = jobs[it.job];
    ao_adjoint_body<GT>(j.t, j.pts, static_cast<const GT*>(j.gbar), j.sK, j.sC, j.elec_out,
                        j.elec_group_stride, j.nuc_partial, it.a, it.b, smem);
    __syncthreads();
  }
}

// Block-wide fixed-order sum of one value per thread (256 threads).
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  return red[0];
}

__global__ __launch_bounds__(256) void reduce_nuc_batch_kernel(const NucRedJob* __restrict__ jobs,
                                                               const int64_t* __restrict__ prefix,
                                                               int n_jobs) {
  __shared__ double red[256];
  const int64_t e = blockIdx.x;
  const int jb = find_job(prefix, n_jobs, e);
  const NucRedJob& j = jobs[jb];
  const int64_t loc = e - prefix[jb];
  const int A = static_cast<int>(loc / 3), i = static_cast<int>(loc - 3 * (loc / 3));
  const int a = j.dev_of[A];
  double acc = 0.0;
  if (a >= 0)
    for (int64_t w = threadIdx.x; w < j.n_waves; w += 256) acc += j.part[(w * j.nucl_dev + a) * 3 + i];
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) j.out[loc] = tot;
}

__global__ void reduce_batch_kernel(const RedJob* __restrict__ jobs,
                                    const int64_t* __restrict__ prefix, int n_jobs, int64_t total) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int jb = find_job(prefix, n_jobs, e);
  const RedJob& j = jobs[jb];
  const int64_t loc = e - prefix[jb];
  const int64_t r = loc / j.cols, c = loc - r * j.cols;
  double acc = 0.0;
  for (int64_t z = 0; z < j.nz; ++z) acc += j.ws[z * j.z_stride + r * j.ld_ws + c];
  j.out[r * j.ld_out + c] = acc;
}

// One block per output entry: strided partial sums then a fixed-order tree
// in LDS, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void reduce_nuc_kernel(const double* __restrict__ part,
                                                         int64_t n_waves, int32_t nucl_dev,
                                                         const int32_t* __restrict__ dev_of,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  const int e = blockIdx.x;
  const int A = e / 3, i = e - 3 * A;
  const int a = dev_of[A];
  double acc = 0.0;
  if (a >= 0)
    for (int64_t w = threadIdx.x; w < n_waves; w += 256) acc += part[(w * nucl_dev + a) * 3 + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[e] = red[0];
}

}  // namespace

hipError_t launch_ao_adjoint_persist(const AdjJob* jobs, const WorkItem* items, int n_items,
                                     int grid, size_t smem, int gbar_is_f32, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (gbar_is_f32)
    hipLaunchKernelGGL(ao_adjoint_persist<float>, dim3(grid), dim3(256), smem, s, jobs, items, n_items);
  else
    hipLaunchKernelGGL(ao_adjoint_persist<double>, dim3(grid), dim3(256), smem, s, jobs, items, n_items);
  return hipGetLastError();
}

int adj_persist_blocks_per_cu(int f32, size_t smem) {
  int n = 0;
  hipError_t e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ao_adjoint_persist<float>, 256, smem)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, ao_adjoint_persist<double>, 256, smem);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_reduce_batch(const RedJob* jobs, const int64_t* prefix, int n_jobs, int64_t total,
                               hipStream_t s) {
  if (total <= 0 || n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_batch_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256),
                     0, s, jobs, prefix, n_jobs, total);
  return hipGetLastError();
}

hipError_t launch_reduce_nuc_batch(const NucRedJob* jobs, const int64_t* prefix, int n_jobs,
                                   int64_t total, hipStream_t s) {
  if (total <= 0 || n_jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_nuc_batch_kernel, dim3(static_cast<unsigned>(total)), dim3(256), 0, s,
                     jobs, prefix, n_jobs);
  return hipGetLastError();
}

hipError_t launch_ao_adjoint(const AoTables& t, const PointArgs& pts, const void* gbar,
                             int gbar_is_f32, int64_t sK, int64_t sC, double* elec_out,
                             int64_t elec_group_stride, double* nuc_partial, int64_t* n_waves,
                             hipStream_t s) {
  const int64_t nblk = (pts.P + 255) / 256;
  *n_waves = nblk * 4;
  if (pts.P <= 0 || t.n_groups <= 0) return hipSuccess;
  dim3 grid(static_cast<unsigned>(nblk), static_cast<unsigned>(t.n_groups));
  const size_t smem = static_cast<size_t>(t.smem_bytes);
  if (gbar_is_f32)
    hipLaunchKernelGGL(ao_adjoint_kernel<float>, grid, dim3(256), smem, s, t, pts,
                       static_cast<const float*>(gbar), sK, sC, elec_out, elec_group_stride,
                       nuc_partial);
  else
    hipLaunchKernelGGL(ao_adjoint_kernel<double>, grid, dim3(256), smem, s, t, pts,
                       static_cast<const double*>(gbar), sK, sC, elec_out, elec_group_stride,
                       nuc_partial);
  return hipGetLastError();
}

hipError_t launch_reduce_nuc(const double* nuc_partial, int64_t n_waves, int32_t nucl_dev,
                             const int32_t* dev_of, int32_t nucl_num, double* d_nucl,
                             hipStream_t s) {
  const int n = nucl_num * 3;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_nuc_kernel, dim3(n), dim3(256), 0, s, nuc_partial, n_waves, nucl_dev,
                     dev_of, d_nucl);
  return hipGetLastError();
}

}  // namespace qmk
