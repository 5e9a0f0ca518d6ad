// MO cusp correction (QMCkl paper, Section 3.3).
//
// Inside the sphere of radius r_A around nucleus A, MO i becomes
//   phi_i - phi_i^{s_A} + sum_{k=0..3} f_{k,i,A} |r - R_A|^k,
// where phi_i^{s_A} is the part of MO i carried by the s-type AOs on A.  Both
// the removed part and the polynomial are radial functions h(r) of
// r = |r - R_A|, so the correction adds to the five components of mo_vgl
//   value h,  gradient h'(r) d / r,  Laplacian h''(r) + 2 h'(r) / r.
//
// One lane per point finds the sphere (if any; the spheres do not overlap)
// that contains its point and appends (point, nucleus) to a compact list.
// Such points are rare, so a second kernel spreads them out: one wave per
// (listed point, block of 64 MOs) updates that block of the point's mo_vgl
// row.
#include "qmk_internal.h"

namespace qmk {
namespace {

__global__ void cusp_clear_kernel(int32_t* count) {
  if (threadIdx.x == 0) *count = 0;
}

// One lane per point: the sphere (if any) that contains it goes to the list
// as the pair (point, nucleus).  The spheres (centre, squared radius) are
// staged in LDS 256 at a time.
__global__ __launch_bounds__(256) void cusp_find_kernel(CuspArgs c, PointArgs pts, int32_t* count,
                                                        int32_t* list) {
  __shared__ double4 sph[256];
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool valid = p < pts.P;
  double rx = 0.0, ry = 0.0, rz = 0.0;
  if (valid) {
    rx = pts.coord[p * pts.s_pt];
    ry = pts.coord[p * pts.s_pt + pts.s_ax];
    rz = pts.coord[p * pts.s_pt + 2 * pts.s_ax];
  }
  int hit = -1;
  for (int a0 = 0; a0 < c.n_nuc; a0 += 256) {
    const int na = min(256, c.n_nuc - a0);
    __syncthreads();  // the previous chunk has been read
    if (static_cast<int>(threadIdx.x) < na) {
      const CuspNuc nu = c.nuc[a0 + threadIdx.x];
      sph[threadIdx.x] = make_double4(nu.x, nu.y, nu.z, nu.rc * nu.rc);
    }
    __syncthreads();
    if (valid && hit < 0) {
      for (int t = 0; t < na; ++t) {
        const double4 q = sph[t];
        const double dx = rx - q.x, dy = ry - q.y, dz = rz - q.z;
        if (dx * dx + dy * dy + dz * dz < q.w) {
          hit = a0 + t;
          break;
        }
      }
    }
  }
  if (hit >= 0) {
    const int32_t k = atomicAdd(count, 1);  // at most once per point: k < P
    list[2 * k] = static_cast<int32_t>(p);
    list[2 * k + 1] = hit;
  }
}

// One wave per (listed point, block of 64 MOs); the grid strides over the
// count that the find kernel left.  Lane t forms the radial sums of the
// nucleus' s shell t (they depend on the point, not on the MO) and every
// lane takes them by shuffle.
template <typename TD>
__global__ __launch_bounds__(256) void cusp_apply_kernel(CuspArgs c, PointArgs pts, TD* __restrict__ mo,
                                                         int64_t N, const int32_t* count,
                                                         const int32_t* list) {
  const int lane = threadIdx.x & 63;
  const int64_t nblk = (N + 63) / 64;
  const int64_t n_items = static_cast<int64_t>(*count) * nblk;
  const int64_t n_waves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
  for (int64_t w = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6; w < n_items;
       w += n_waves) {
    const int64_t h = w / nblk;
    const int64_t q = list[2 * h];
    const int a = list[2 * h + 1];
    const int64_t i = (w - h * nblk) * 64 + lane;
    const bool on = i < N;
    const CuspNuc nu = c.nuc[a];
    const double dx = pts.coord[q * pts.s_pt] - nu.x;
    const double dy = pts.coord[q * pts.s_pt + pts.s_ax] - nu.y;
    const double dz = pts.coord[q * pts.s_pt + 2 * pts.s_ax] - nu.z;
    const double u = dist2(dx, dy, dz);
    const double r = sqrt(u);
    const double ir = 1.0 / r;  // a point exactly on the nucleus: the cusp diverges
    const int ns = nu.s_end - nu.s_begin;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;  // phi^s and its first two radial derivatives
    for (int j0 = 0; j0 < ns; j0 += 64) {
      double m = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
      if (j0 + lane < ns) {
        const CuspS sj = c.s[nu.s_begin + j0 + lane];
        m = sj.m;
        for (int k = sj.p_begin; k < sj.p_end; ++k) {
          const PrimDev pr = c.prim[k];
          const double x = pr.gamma * u;
          if (x >= c.T) break;  // ascending exponents, as in the AO stage
          const double e = pr.coef * exp(-x);
          g0 += e;
          g1 -= pr.gamma * e;
          g2 += pr.gamma * pr.gamma * e;
        }
      }
      const int nj = min(64, ns - j0);
      for (int t = 0; t < nj; ++t) {
        const double mt = __shfl(m, t, 64), h0 = __shfl(g0, t, 64);
        const double h1 = __shfl(g1, t, 64), h2 = __shfl(g2, t, 64);
        // chi = M g0(u), chi' = 2 r M g1, chi'' = M (2 g1 + 4 u g2)
        const double wt = on ? c.cs[static_cast<int64_t>(nu.s_begin + j0 + t) * N + i] * mt : 0.0;
        s0 += wt * h0;
        s1 += wt * 2.0 * r * h1;
        s2 += wt * (2.0 * h1 + 4.0 * u * h2);
      }
    }
    if (!on) continue;
    const double* f = c.f + static_cast<int64_t>(a) * 4 * N;
    const double f0 = f[i], f1 = f[N + i], f2 = f[2 * N + i], f3 = f[3 * N + i];
    const double h0 = f0 + r * (f1 + r * (f2 + r * f3)) - s0;
    const double h1 = f1 + r * (2.0 * f2 + 3.0 * r * f3) - s1;
    const double h2 = 2.0 * f2 + 6.0 * r * f3 - s2;
    const double g = h1 * ir;
    TD* row = mo + q * 5 * N;
    row[i] = static_cast<TD>(static_cast<double>(row[i]) + h0);
    row[N + i] = static_cast<TD>(static_cast<double>(row[N + i]) + g * dx);
    row[2 * N + i] = static_cast<TD>(static_cast<double>(row[2 * N + i]) + g * dy);
    row[3 * N + i] = static_cast<TD>(static_cast<double>(row[3 * N + i]) + g * dz);
    row[4 * N + i] = static_cast<TD>(static_cast<double>(row[4 * N + i]) + h2 + 2.0 * g);
  }
}

}  // namespace

hipError_t launch_cusp(const CuspArgs& c, const PointArgs& pts, void* mo, int out_is_f32, int64_t N,
                       int32_t* count, int32_t* list, hipStream_t s) {
  if (pts.P <= 0 || c.n_nuc <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(cusp_clear_kernel, dim3(1), dim3(64), 0, s, count);
  hipLaunchKernelGGL(cusp_find_kernel, dim3(static_cast<unsigned>((pts.P + 255) / 256)), dim3(256), 0, s, c,
                     pts, count, list);
  const dim3 grid(1024);  // 4096 waves, striding over the listed (point, MO block) items
  if (out_is_f32)
    hipLaunchKernelGGL(cusp_apply_kernel<float>, grid, dim3(256), 0, s, c, pts, static_cast<float*>(mo), N,
                       count, list);
  else
    hipLaunchKernelGGL(cusp_apply_kernel<double>, grid, dim3(256), 0, s, c, pts, static_cast<double*>(mo), N,
                       count, list);
  return hipGetLastError();
}

}  // namespace qmk
