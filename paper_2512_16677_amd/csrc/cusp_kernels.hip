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
// that contains its point.  Such points are rare, so the wave then serves
// them one at a time: one lane per s shell of the nucleus evaluates that
// shell's radial sums at the point, and every lane takes them by shuffle to
// update 64 MOs per pass of the point's mo_vgl row.
#include "qmk_internal.h"

namespace qmk {
namespace {

template <typename TD>
__global__ __launch_bounds__(256) void cusp_kernel(CuspArgs c, PointArgs pts, TD* __restrict__ mo,
                                                   int64_t N) {
  const int lane = threadIdx.x & 63;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double rx = 0.0, ry = 0.0, rz = 0.0;
  int hit = -1;
  if (p < pts.P) {
    rx = pts.coord[p * pts.s_pt];
    ry = pts.coord[p * pts.s_pt + pts.s_ax];
    rz = pts.coord[p * pts.s_pt + 2 * pts.s_ax];
    for (int a = 0; a < c.n_nuc; ++a) {
      const CuspNuc nu = c.nuc[a];
      const double dx = rx - nu.x, dy = ry - nu.y, dz = rz - nu.z;
      if (dx * dx + dy * dy + dz * dz < nu.rc * nu.rc) {
        hit = a;
        break;
      }
    }
  }
  uint64_t mask = __ballot(hit >= 0);
  while (mask) {
    const int src = __builtin_ctzll(mask);
    mask &= mask - 1;
    const int64_t q = __shfl(p, src, 64);
    const int a = __shfl(hit, src, 64);
    const CuspNuc nu = c.nuc[a];
    const double dx = __shfl(rx, src, 64) - nu.x;
    const double dy = __shfl(ry, src, 64) - nu.y;
    const double dz = __shfl(rz, src, 64) - nu.z;
    const double u = dx * dx + dy * dy + dz * dz;
    const double r = sqrt(u);
    const double ir = 1.0 / r;  // a point exactly on the nucleus: the cusp diverges
    TD* row = mo + q * 5 * N;
    const int ns = nu.s_end - nu.s_begin;
    // The radial sums of the point's s shells do not depend on the MO: lane
    // t forms those of shell j0 + t, and every lane takes them by shuffle.
    // The first 64 shells are formed once per point, any further ones per
    // pass.
    auto radial = [&](int j0, double& m, double& g0, double& g1, double& g2) {
      m = g0 = g1 = g2 = 0.0;
      if (j0 + lane >= ns) return;
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
    };
    double m_first, g0_first, g1_first, g2_first;
    radial(0, m_first, g0_first, g1_first, g2_first);
    for (int64_t i0 = 0; i0 < N; i0 += 64) {
      const int64_t i = i0 + lane;
      const bool on = i < N;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;  // phi^s and its first two radial derivatives
      for (int j0 = 0; j0 < ns; j0 += 64) {
        double m = m_first, g0 = g0_first, g1 = g1_first, g2 = g2_first;
        if (j0 > 0) radial(j0, m, g0, g1, g2);
        const int nj = min(64, ns - j0);
        for (int t = 0; t < nj; ++t) {
          const double mt = __shfl(m, t, 64), h0 = __shfl(g0, t, 64);
          const double h1 = __shfl(g1, t, 64), h2 = __shfl(g2, t, 64);
          // chi = M g0(u), chi' = 2 r M g1, chi'' = M (2 g1 + 4 u g2)
          const double w = on ? c.cs[static_cast<int64_t>(nu.s_begin + j0 + t) * N + i] * mt : 0.0;
          s0 += w * h0;
          s1 += w * 2.0 * r * h1;
          s2 += w * (2.0 * h1 + 4.0 * u * h2);
        }
      }
      if (!on) continue;
      const double* f = c.f + static_cast<int64_t>(a) * 4 * N;
      const double f0 = f[i], f1 = f[N + i], f2 = f[2 * N + i], f3 = f[3 * N + i];
      const double h0 = f0 + r * (f1 + r * (f2 + r * f3)) - s0;
      const double h1 = f1 + r * (2.0 * f2 + 3.0 * r * f3) - s1;
      const double h2 = 2.0 * f2 + 6.0 * r * f3 - s2;
      const double g = h1 * ir;
      row[i] = static_cast<TD>(static_cast<double>(row[i]) + h0);
      row[N + i] = static_cast<TD>(static_cast<double>(row[N + i]) + g * dx);
      row[2 * N + i] = static_cast<TD>(static_cast<double>(row[2 * N + i]) + g * dy);
      row[3 * N + i] = static_cast<TD>(static_cast<double>(row[3 * N + i]) + g * dz);
      row[4 * N + i] = static_cast<TD>(static_cast<double>(row[4 * N + i]) + h2 + 2.0 * g);
    }
  }
}

}  // namespace

hipError_t launch_cusp(const CuspArgs& c, const PointArgs& pts, void* mo, int out_is_f32, int64_t N,
                       hipStream_t s) {
  if (pts.P <= 0 || c.n_nuc <= 0) return hipSuccess;
  const dim3 grid(static_cast<unsigned>((pts.P + 255) / 256));
  if (out_is_f32)
    hipLaunchKernelGGL(cusp_kernel<float>, grid, dim3(256), 0, s, c, pts, static_cast<float*>(mo), N);
  else
    hipLaunchKernelGGL(cusp_kernel<double>, grid, dim3(256), 0, s, c, pts, static_cast<double*>(mo), N);
  return hipGetLastError();
}

}  // namespace qmk
