// AO -> MO contraction and adjoint GEMMs on MFMA (QMCkl paper, Section 3.2:
// the MO values, gradients and Laplacians are one matrix product of the
// concatenated AO array with the coefficient matrix).
//
// One strided, batched kernel serves the three products of the path:
//   forward   mo[p][c][n]   = sum_k ao[k][c][p] Ct[k][n]        (batch c)
//   Gbar      Gb[k][c][p]   = sum_n C[n][k] W[p][c][n]          (batch c)
//             (rows k, columns p: a 16-lane group of the accumulator stores
//             16 consecutive points, so the output is written in full lines)
//   dC        ws[c,s][n][k] = sum_{p in split s} W[p][c][n] ao[k][c][p]
//   density   part[t][p]    = sum_{n in tile t} occ[n] (sum_k ao[k][p] Ct[k][n])^2
//   screened  mo[perm[q]][c][n] = sum_{k in active chunks} aos[k][c][q] Ct[k][n]
//             (aos: the AO array in sorted point order)
//   Jastrow   part[c,k][slot] = sum over the slot's (i, j) of
//             w_k(i, j) sum_l Ra[c][l][i] rt^k[c][l][j]   (no output matrix)
// (see GemmArgs for the index algebra).  A tile is WGM x WGN wavefronts,
// each owning TM x TN MFMA 16x16x4 blocks (FP64 or FP32); the shapes on
// offer are listed in QMK_TILE_LIST and chosen per problem by the host
// autotuner (padding waste of N_MO = 400 on 128-wide tiles is 22%, on
// 80-wide tiles zero).  Operand tiles go
// global -> registers -> LDS with one tile of prefetch (double-buffered
// LDS, one barrier per K step).  Tile order is XCD-aware: the eight
// consecutive workgroup ids land on the eight XCDs, so ids are remapped so
// that all N tiles of one M tile run on the same XCD back to back and the
// M-tile of A is fetched from HBM once per XCD L2.
#include "gemm_impl.h"

namespace qmk {

#ifdef QMK_GEMM_UNIT
#if QMK_GEMM_UNIT == 1
hipError_t gemm_unit_f64_fwd(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s) {
  const bool alt = o32 != 0;
  if (pl) return alt ? run_persist<double, double, double, float, true, true>(cfg, *pl, s) : run_persist<double, double, double, double, true, true>(cfg, *pl, s);
  return alt ? run<double, double, double, float, true, true>(cfg, *g, s) : run<double, double, double, double, true, true>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 2
hipError_t gemm_unit_f64_gbar(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s) {
  const bool alt = w32 != 0;
  if (pl) return alt ? run_persist<double, double, float, double, true, false>(cfg, *pl, s) : run_persist<double, double, double, double, true, false>(cfg, *pl, s);
  return alt ? run<double, double, float, double, true, false>(cfg, *g, s) : run<double, double, double, double, true, false>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 3
hipError_t gemm_unit_f64_dc(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s) {
  const bool alt = w32 != 0;
  if (pl) return alt ? run_persist<double, float, double, double, true, false>(cfg, *pl, s) : run_persist<double, double, double, double, true, false>(cfg, *pl, s);
  return alt ? run<double, float, double, double, true, false>(cfg, *g, s) : run<double, double, double, double, true, false>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 4
hipError_t gemm_unit_f32_fwd(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s) {
  const bool alt = o32 != 0;
  if (pl) return alt ? run_persist<float, float, float, float, true, true>(cfg, *pl, s) : run_persist<float, float, float, double, true, true>(cfg, *pl, s);
  return alt ? run<float, float, float, float, true, true>(cfg, *g, s) : run<float, float, float, double, true, true>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 5
hipError_t gemm_unit_f32_gbar(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s) {
  const bool alt = w32 != 0;
  if (pl) return alt ? run_persist<float, float, float, float, true, false>(cfg, *pl, s) : run_persist<float, float, double, float, true, false>(cfg, *pl, s);
  return alt ? run<float, float, float, float, true, false>(cfg, *g, s) : run<float, float, double, float, true, false>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 6
hipError_t gemm_unit_f32_dc(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s) {
  const bool alt = w32 != 0;
  if (pl) return alt ? run_persist<float, float, float, double, true, false>(cfg, *pl, s) : run_persist<float, double, float, double, true, false>(cfg, *pl, s);
  return alt ? run<float, float, float, double, true, false>(cfg, *g, s) : run<float, double, float, double, true, false>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 9
// Screened adjoint products (points in sorted order; see gemm_body EPI 3, 4).
hipError_t gemm_unit_screened_adj(GemmKind kind, int cfg, const GemmArgs* g, Prec prec, int w32,
                                  hipStream_t s) {
  if (kind == GemmKind::kGbar) {
    if (prec == Prec::kF64)
      return w32 ? run<double, double, float, double, true, false, 3>(cfg, *g, s)
                 : run<double, double, double, double, true, false, 3>(cfg, *g, s);
    return w32 ? run<float, float, float, float, true, false, 3>(cfg, *g, s)
               : run<float, float, double, float, true, false, 3>(cfg, *g, s);
  }
  if (prec == Prec::kF64)
    return w32 ? run<double, float, double, double, true, false, 4>(cfg, *g, s)
               : run<double, double, double, double, true, false, 4>(cfg, *g, s);
  return w32 ? run<float, float, float, double, true, false, 4>(cfg, *g, s)
             : run<float, double, float, double, true, false, 4>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 8
hipError_t gemm_unit_sparse(int cfg, const GemmArgs* g, Prec prec, int o32, hipStream_t s) {
  if (prec == Prec::kF64)
    return o32 ? run_sparse<double, float>(cfg, *g, s) : run_sparse<double, double>(cfg, *g, s);
  return o32 ? run_sparse<float, float>(cfg, *g, s) : run_sparse<float, double>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 10
// Three-body Jastrow product with its fused weighted reduction (gemm_body
// EPI 5).
hipError_t gemm_unit_jastrow(int cfg, const GemmArgs* g, hipStream_t s) {
  return run<double, double, double, double, true, true, 5>(cfg, *g, s);
}
#endif
#if QMK_GEMM_UNIT == 7
hipError_t gemm_unit_density(int cfg, const GemmArgs* g, Prec prec, hipStream_t s) {
  return prec == Prec::kF64 ? run_density<double>(cfg, *g, s) : run_density<float>(cfg, *g, s);
}
#endif
#else
// Products of each (precision, kind) are instantiated in their own
// translation unit (this file compiled with QMK_GEMM_UNIT = 1..10) so that
// they build in parallel; the unit without QMK_GEMM_UNIT holds the tables
// and the dispatch.
hipError_t gemm_unit_f64_fwd(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s);
hipError_t gemm_unit_f64_gbar(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s);
hipError_t gemm_unit_f64_dc(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s);
hipError_t gemm_unit_f32_fwd(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s);
hipError_t gemm_unit_f32_gbar(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s);
hipError_t gemm_unit_f32_dc(int cfg, const GemmArgs* g, const PersistLaunch* pl, int w32, int o32,
                         hipStream_t s);

hipError_t gemm_unit_density(int cfg, const GemmArgs* g, Prec prec, hipStream_t s);
hipError_t gemm_unit_jastrow(int cfg, const GemmArgs* g, hipStream_t s);
hipError_t gemm_unit_sparse(int cfg, const GemmArgs* g, Prec prec, int o32, hipStream_t s);
hipError_t gemm_unit_screened_adj(GemmKind kind, int cfg, const GemmArgs* g, Prec prec, int w32,
                                  hipStream_t s);
namespace {
hipError_t unit_dispatch(GemmKind kind, Prec prec, int cfg, const GemmArgs* g, const PersistLaunch* pl,
                         int w32, int o32, hipStream_t s) {
  if (prec == Prec::kF64) {
    switch (kind) {
      case GemmKind::kForward: return gemm_unit_f64_fwd(cfg, g, pl, w32, o32, s);
      case GemmKind::kGbar: return gemm_unit_f64_gbar(cfg, g, pl, w32, o32, s);
      case GemmKind::kDcoef: return gemm_unit_f64_dc(cfg, g, pl, w32, o32, s);
    }
  } else {
    switch (kind) {
      case GemmKind::kForward: return gemm_unit_f32_fwd(cfg, g, pl, w32, o32, s);
      case GemmKind::kGbar: return gemm_unit_f32_gbar(cfg, g, pl, w32, o32, s);
      case GemmKind::kDcoef: return gemm_unit_f32_dc(cfg, g, pl, w32, o32, s);
    }
  }
  return hipErrorInvalidValue;
}
}  // namespace

int gemm_num_tiles(Prec prec) {
  return prec == Prec::kBF16P ? gemm_bf16p_num_tiles() : kNumTiles;
}

TileCfg gemm_tile(Prec prec, int cfg) {
  return prec == Prec::kBF16P ? gemm_bf16p_tile(cfg) : kTiles[cfg];
}

size_t gemm_tile_lds_bytes(Prec prec, int cfg) {
  if (prec == Prec::kBF16P) return gemm_bf16p_tile_lds_bytes(cfg);
  const TileCfg& t = kTiles[cfg];
  const size_t esz = prec == Prec::kF64 ? 8 : 4;
  const size_t pad = 16 / esz;
  return 2 * static_cast<size_t>(t.bk) *
         ((16 * t.wgm * t.tm + pad) + (16 * t.wgn * t.tn + pad)) * esz;
}

hipError_t launch_gemm_sparse(Prec prec, int cfg, const GemmArgs& g, int out_is_f32, hipStream_t s) {
  if (prec == Prec::kBF16P || cfg < 0 || cfg >= kNumTiles) return hipErrorInvalidValue;
  return gemm_unit_sparse(cfg, &g, prec, out_is_f32, s);
}

hipError_t launch_gemm_screened_adj(GemmKind kind, Prec prec, int cfg, const GemmArgs& g, int w_is_f32,
                                    hipStream_t s) {
  if (prec == Prec::kBF16P || cfg < 0 || cfg >= kNumTiles ||
      (kind != GemmKind::kGbar && kind != GemmKind::kDcoef))
    return hipErrorInvalidValue;
  return gemm_unit_screened_adj(kind, cfg, &g, prec, w_is_f32, s);
}

hipError_t launch_gemm_jastrow(int cfg, const GemmArgs& g, hipStream_t s) {
  if (cfg < 0 || cfg >= kNumTiles) return hipErrorInvalidValue;
  return gemm_unit_jastrow(cfg, &g, s);
}

hipError_t launch_gemm_density(Prec prec, int cfg, const GemmArgs& g, hipStream_t s) {
  if (prec == Prec::kBF16P || cfg < 0 || cfg >= kNumTiles) return hipErrorInvalidValue;
  return gemm_unit_density(cfg, &g, prec, s);
}

hipError_t launch_gemm_typed(GemmKind kind, Prec prec, int cfg, const GemmArgs& g, int w_is_f32,
                             int out_is_f32, hipStream_t s) {
  if (prec == Prec::kBF16P) return launch_gemm_bf16p(kind, cfg, g, out_is_f32, 0, s);
  if (cfg < 0 || cfg >= kNumTiles) return hipErrorInvalidValue;
  return unit_dispatch(kind, prec, cfg, &g, nullptr, w_is_f32, out_is_f32, s);
}

hipError_t launch_gemm_persist(GemmKind kind, Prec prec, int cfg, const GemmArgs* jobs,
                               const WorkItem* items, int n_items, int grid, int w_is_f32,
                               int out_is_f32, hipStream_t s) {
  if (prec == Prec::kBF16P)
    return launch_gemm_bf16p_persist(kind, cfg, jobs, items, n_items, grid, out_is_f32, nullptr, s);
  if (cfg < 0 || cfg >= kNumTiles) return hipErrorInvalidValue;
  PersistLaunch pl{jobs, items, n_items, grid, nullptr};
  return unit_dispatch(kind, prec, cfg, nullptr, &pl, w_is_f32, out_is_f32, s);
}

int gemm_persist_blocks_per_cu(GemmKind kind, Prec prec, int cfg, int w_is_f32, int out_is_f32) {
  int n = 1;
  if (prec == Prec::kBF16P) return gemm_bf16p_blocks_per_cu(kind, cfg, out_is_f32);
  if (cfg < 0 || cfg >= kNumTiles) return 1;
  PersistLaunch pl{nullptr, nullptr, 0, 0, &n};
  (void)unit_dispatch(kind, prec, cfg, nullptr, &pl, w_is_f32, out_is_f32, nullptr);
  return n;
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

#endif  // QMK_GEMM_UNIT

}  // namespace qmk
