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

template <typename GT>
__device__ __forceinline__ double ldg(const GT* p) { return static_cast<double>(*p); }

// Contracts the third-order AO derivatives of one shell with Gbar.
//   d_i chi     = M (P_i g0 + 2 d_i P g1)
//   d_i d_j chi = M (P_ij g0 + 2 (d_j P_i + d_i P_j) g1 + 2 delta_ij P g1
//                    + 4 d_i d_j P g2)
//   d_i lap chi = M (lapP_i g0 + (2 d_i lapP + (4L+6) P_i) g1
//                    + ((8L+20) d_i P + 4 u P_i) g2 + 8 u d_i P g3)
template <int L, typename GT>
__device__ __forceinline__ void shell_adjoint(double dx, double dy, double dz, double u, double g0,
                                              double g1, double g2, double g3,
                                              const double* __restrict__ M,
                                              const GT* __restrict__ gb, int64_t sK, int64_t sC,
                                              double& tx, double& ty, double& tz) {
  // D[axis][m][e]: m-th derivative of d^e, for e <= L, m <= 3.
  double px[L + 1], py[L + 1], pz[L + 1];
  px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
  for (int i = 1; i <= L; ++i) {
    px[i] = px[i - 1] * dx;
    py[i] = py[i - 1] * dy;
    pz[i] = pz[i - 1] * dz;
  }
  const double d[3] = {dx, dy, dz};
  int idx = 0;
#pragma unroll
  for (int a = L; a >= 0; --a) {
#pragma unroll
    for (int b = L - a; b >= 0; --b, ++idx) {
      const int c = L - a - b;
      const int e[3] = {a, b, c};
      const double* pw[3] = {px, py, pz};
      double D[3][4];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int n = e[ax] - m;
          double coef = 1.0;
#pragma unroll
          for (int q = 0; q < m; ++q) coef *= static_cast<double>(e[ax] - q);
          D[ax][m] = n >= 0 ? coef * pw[ax][n >= 0 ? n : 0] : 0.0;
        }
      }
      const double P = D[0][0] * D[1][0] * D[2][0];
      const double Pi[3] = {D[0][1] * D[1][0] * D[2][0], D[0][0] * D[1][1] * D[2][0],
                            D[0][0] * D[1][0] * D[2][1]};
      double Pij[3][3];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int m[3] = {0, 0, 0};
          m[i] += 1;
          m[j] += 1;
          Pij[i][j] = D[0][m[0]] * D[1][m[1]] * D[2][m[2]];
        }
      const double lapP = Pij[0][0] + Pij[1][1] + Pij[2][2];
      double glP[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double sacc = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          int m[3] = {0, 0, 0};
          m[i] += 1;
          m[j] += 2;
          sacc += D[0][m[0]] * D[1][m[1]] * D[2][m[2]];
        }
        glP[i] = sacc;
      }
      const GT* q = gb + idx * sK;
      const double G0 = ldg(q), G1 = ldg(q + sC), G2 = ldg(q + 2 * sC), G3 = ldg(q + 3 * sC),
                   G4 = ldg(q + 4 * sC);
      const double Gj[3] = {G1, G2, G3};
      const double m = M[idx];
      double t[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double gi = Pi[i] * g0 + 2.0 * d[i] * P * g1;
        double hs = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double h = Pij[i][j] * g0 + 2.0 * (d[j] * Pi[i] + d[i] * Pi[j]) * g1 +
                     4.0 * d[i] * d[j] * P * g2;
          if (i == j) h += 2.0 * P * g1;
          hs += Gj[j] * h;
        }
        const double gl = glP[i] * g0 + (2.0 * d[i] * lapP + (4.0 * L + 6.0) * Pi[i]) * g1 +
                          ((8.0 * L + 20.0) * d[i] * P + 4.0 * u * Pi[i]) * g2 +
                          8.0 * u * d[i] * P * g3;
        t[i] = m * (G0 * gi + hs + G4 * gl);
      }
      tx += t[0];
      ty += t[1];
      tz += t[2];
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename GT>
__global__ __launch_bounds__(256) void ao_adjoint_kernel(AoTables t, PointArgs pts,
                                                         const GT* __restrict__ gbar, int64_t sK,
                                                         int64_t sC, double* __restrict__ elec_out,
                                                         int64_t elec_group_stride,
                                                         double* __restrict__ nuc_partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  const NucGroup g = t.group[blockIdx.y];
  const int np = g.p_end - g.p_begin, ns = g.sh_end - g.sh_begin, nn = g.nuc_end - g.nuc_begin;
  PrimDev* s_prim = reinterpret_cast<PrimDev*>(smem);
  ShellDev* s_shell = reinterpret_cast<ShellDev*>(s_prim + np);
  NucDev* s_nuc = reinterpret_cast<NucDev*>(s_shell + ns);
  for (int i = threadIdx.x; i < np; i += blockDim.x) s_prim[i] = t.prim[g.p_begin + i];
  for (int i = threadIdx.x; i < ns; i += blockDim.x) s_shell[i] = t.shell[g.sh_begin + i];
  for (int i = threadIdx.x; i < nn; i += blockDim.x) s_nuc[i] = t.nuc[g.nuc_begin + i];
  __syncthreads();

  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const bool valid = p < pts.P;
  double rx = 0.0, ry = 0.0, rz = 0.0;
  if (valid) {
    rx = pts.coord[p * pts.s_pt];
    ry = pts.coord[p * pts.s_pt + pts.s_ax];
    rz = pts.coord[p * pts.s_pt + 2 * pts.s_ax];
  }
  const GT* gb_p = gbar + p;
  const double T = t.T;
  double ex = 0.0, ey = 0.0, ez = 0.0;

  for (int a = 0; a < nn; ++a) {
    const NucDev nu = s_nuc[a];
    const double dx = rx - nu.x, dy = ry - nu.y, dz = rz - nu.z;
    const double u = dx * dx + dy * dy + dz * dz;
    const bool near = valid && (nu.gmin * u < T);
    double tx = 0.0, ty = 0.0, tz = 0.0;
    if (__any(near)) {
      for (int s = nu.sh_begin; s < nu.sh_end; ++s) {
        const ShellDev sh = s_shell[s];
        double g0 = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
        for (int k = sh.p_begin; k < sh.p_end; ++k) {
          const PrimDev pr = s_prim[k];
          const double x = pr.gamma * u;
          const bool on = near && (x < T);
          if (!__any(on)) break;
          if (on) {
            const double e = pr.coef * exp(-x);
            const double ge = pr.gamma * e;
            g0 += e;
            g1 -= ge;
            g2 += pr.gamma * ge;
            g3 -= pr.gamma * pr.gamma * ge;
          }
        }
        if (near) {
          const GT* q = gb_p + sh.ao_off * sK;
          const double* M = t.ao_factor + sh.ao_off;
          switch (sh.l) {
            case 0: shell_adjoint<0>(dx, dy, dz, u, g0, g1, g2, g3, M, q, sK, sC, tx, ty, tz); break;
            case 1: shell_adjoint<1>(dx, dy, dz, u, g0, g1, g2, g3, M, q, sK, sC, tx, ty, tz); break;
            case 2: shell_adjoint<2>(dx, dy, dz, u, g0, g1, g2, g3, M, q, sK, sC, tx, ty, tz); break;
            default: shell_adjoint<3>(dx, dy, dz, u, g0, g1, g2, g3, M, q, sK, sC, tx, ty, tz); break;
          }
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
    double* o = elec_out + blockIdx.y * elec_group_stride + p * 3;
    o[0] = ex;
    o[1] = ey;
    o[2] = ez;
  }
}

__global__ void reduce_nuc_kernel(const double* __restrict__ part, int64_t n_waves,
                                  int32_t nucl_dev, const int32_t* __restrict__ dev_of,
                                  int32_t nucl_num, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nucl_num * 3) return;
  const int A = e / 3, i = e - 3 * A;
  const int a = dev_of[A];
  double acc = 0.0;
  if (a >= 0)
    for (int64_t w = 0; w < n_waves; ++w) acc += part[(w * nucl_dev + a) * 3 + i];
  out[e] = acc;
}

}  // namespace

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
  hipLaunchKernelGGL(reduce_nuc_kernel, dim3((n + 255) / 256), dim3(256), 0, s, nuc_partial,
                     n_waves, nucl_dev, dev_of, nucl_num, d_nucl);
  return hipGetLastError();
}

}  // namespace qmk
