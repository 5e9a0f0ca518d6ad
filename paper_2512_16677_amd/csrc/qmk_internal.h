// Internal declarations shared by the host runtime and the HIP kernels.
// Not part of the public ABI (include/qmk.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>

namespace qmk {

constexpr int kMaxL = 3;            // highest angular momentum supported (f)
constexpr int kGroupMaxPrim = 2048; // primitives staged in LDS per nucleus group
constexpr int kGroupMaxShell = 512;
constexpr int kGroupMaxNuc = 128;
// AOs per nucleus group.  The AO kernels launch one workgroup per (256
// points, group), so the cap also sets how finely the AO axis is split over
// workgroups: at 120 an 800-AO system runs 7 workgroups per point block
// instead of 1, which removes the tail of a grid of only ~2 workgroups per CU.
constexpr int kGroupMaxAo = 120;
constexpr int kPointPad = 256;      // points are padded to a multiple of this
constexpr int kAoPad = 128;         // AOs (K) padded to a multiple of this
constexpr int kMoPad = 128;         // MOs (N) padded to a multiple of this
// Coefficients per row of the Jastrow weight polynomials (degree <= 8).
constexpr int kJasCoef = 9;
constexpr int kSparseChunk = 16;    // AOs per chunk of the screened product's bitmap
constexpr int kSparseMaxStages = 1024;  // K stages a screened product can list (K <= 16384)

// One nucleus as the AO kernels see it.  gmin = smallest exponent of all its
// primitives: if gmin*u >= T for every point of a wavefront, the whole
// nucleus is skipped (the per-nucleus radius test, in squared form).
struct NucDev {
  double x, y, z, gmin;
  int32_t sh_begin, sh_end;  // shells, indices local to the nucleus' group
  int32_t orig;              // index of the nucleus in the caller's array
  int32_t pad1;
};

// One shell: its AOs are ao_off .. ao_off + (l+1)(l+2)/2 - 1; its primitives
// p_begin .. p_end-1 are sorted by ascending exponent.
struct ShellDev {
  int32_t ao_off, l, p_begin, p_end;
};

// Contiguous range of nuclei whose shells and primitives fit in LDS.
struct NucGroup {
  int32_t nuc_begin, nuc_end, sh_begin, sh_end, p_begin, p_end, n_ao, pad1;
};

// Primitive table entry: exponent gamma and folded coefficient a*f*N_s.
struct PrimDev {
  double gamma, coef;
};

struct AoTables {
  const NucDev* nuc;
  const ShellDev* shell;
  const PrimDev* prim;
  const double* ao_factor;  // M_n per AO
  const NucGroup* group;
  int32_t n_groups;
  int32_t ao_num;
  double T;                 // cutoff on gamma*u: (B-1) ln 2
  int32_t smem_bytes;       // LDS needed by the largest group
  int32_t nucl_dev;         // number of nuclei with at least one shell
};

struct PointArgs {
  const double* coord;      // device
  int64_t s_pt, s_ax;       // coord of point p, axis i: coord[p*s_pt + i*s_ax]
  int64_t P;                // number of points
  const int32_t* perm;      // AO kernel only: point p reads coordinates perm[p] (NULL: p)
};

// Squared point-nucleus distance with one fixed rounding sequence, so that
// every kernel that screens on it (AO values, their activity bitmap, the
// adjoint, the cusp correction's s part) takes the same decisions.
__device__ __forceinline__ double dist2(double dx, double dy, double dz) {
  return __fma_rn(dz, dz, __fma_rn(dy, dy, dx * dx));
}

// Strided AO output: element (k, c, p) at out[k*sK + c*sC + p*sP].
struct AoOut {
  void* out;
  int64_t sK, sC, sP;
  // screened (sorted-point) evaluation: bit c of act[(p/64)*act_words + c/32]
  // is set if any point of the 64-point block of p has a non-zero AO in chunk
  // c (16 AOs); act_prev is the bitmap of the previous evaluation into the
  // same array (see launch_ao_vgl_screened)
  uint32_t* act;
  int64_t act_words;
  const uint32_t* act_prev;
  // split bf16 output (launch_ao_vgl with out_is_f32 = 2): elements from the
  // hi plane at `out` to the lo plane; P must be padded to a multiple of 256
  // and every point offset even
  int64_t plane;
};

// Cusp correction tables (see cusp_kernels.hip).  One entry per nucleus
// with a cusp sphere: centre, radius, its s-type AOs s_begin .. s_end-1.
struct CuspNuc {
  double x, y, z, rc;
  int32_t s_begin, s_end, pad0, pad1;
};
// One s-type AO: normalisation factor M and its primitives (folded
// coefficients, ascending exponents) p_begin .. p_end-1 of CuspArgs::prim.
struct CuspS {
  double m;
  int32_t p_begin, p_end;
};
struct CuspArgs {
  const CuspNuc* nuc;
  const CuspS* s;
  const PrimDev* prim;
  const double* cs;  // [s-AO j][mo i]: C[i][AO of j]
  const double* f;   // [nucleus a][k][mo i]: polynomial coefficients f_k
  double T;          // exponent cutoff of the AO stage
  int32_t n_nuc;
};

// Generic strided batched GEMM  D(i,j) = sum_l A(i,l) B(l,j)  for a batch
// index z = c*nsplit + s:
//   A(i,l) = A[c*oAc + s*oAs + i*sAi + l*sAl]     (l restricted to split s)
//   B(l,j) = B[c*oBc + s*oBs + l*sBl + j*sBj]
//   D(i,j) = D[z*oDz + i*sDi + j*sDj]
// Loads outside i < M, l < L_s, j < N read zero; stores are guarded the same
// way.  L_s = min(Lchunk, L - s*Lchunk).
struct GemmArgs {
  const void* A;
  int64_t sAi, sAl, oAc, oAs;
  const void* B;
  int64_t sBl, sBj, oBc, oBs;
  void* D;
  int64_t sDi, sDj, oDz;
  int64_t M, N, L, Lchunk;
  int32_t nsplit, nbatch;   // gridDim.y = nbatch * nsplit
  // BF16x3 kernel only: second (lo) plane of a pre-split operand.
  const void* A2;
  const void* B2;
  // Workgroup -> tile order of the grid launch.  0: the N tiles of one M tile
  // run back to back on one XCD (A tile reused from that XCD's L2).  1: the
  // tiles of all z in contiguous ranges per XCD, blocked so that the tiles
  // resident together share both operands (split products, whose z slab of
  // both operands is shared by every tile of that z; see grid_tile).
  // 2: the M tiles of one N tile run back to back on one XCD (B tile reused;
  // for products with few M tiles and a long N axis).
  int32_t map_slab;
  // Direct-load products only.  Bit 0: every row l of A is readable along i
  // up to M rounded up to 16 bytes (a padded, allocated stride); bit 1: the
  // same for the rows of an l-major B along j up to N.  The values read
  // there only reach outputs that are not stored.
  int32_t pad_ok;
  // Density epilogue only: occupation of column j (device, N entries).
  const double* occ;
  // Screened forward product only: activity bitmap of (64-point block,
  // 16-AO chunk) pairs, act_words 32-bit words per block, and the original
  // row of each sorted row.
  const uint32_t* act;
  const int32_t* perm;
  int64_t act_words;
  // Three-body Jastrow product only (FP64, batch c = walker, split s = power
  // k of the rescaled e-e distances rt, which B holds with the diagonal
  // marked < 0): row i of the product is (m = 1 + i / j_nn, nucleus
  // a = i % j_nn), column j an electron.  jx[c][a][j] holds
  // x = exp(-kappa |r_j - R_a|) (N per nucleus), jq[s][m-1][a][0..kJasCoef)
  // the coefficients (ascending powers, zero-padded) of the polynomial in x
  // that weighs output (i, j).  Each wave stores the weighted sum of its
  // outputs in its own slot of D (see the product's epilogue).
  const double* jx;
  const double* jq;
  int64_t j_nn;
  int32_t j_mh;
};

// Tile of workgroup `bid` of a grid launch; false if it has none.  The
// eight consecutive workgroup ids land on the eight XCDs of the MI355X.
__device__ __forceinline__ bool grid_tile(const GemmArgs& g, int nM, int nN, int bid, int& mt,
                                          int& nt, int& z) {
  const int x = bid & 7, j = bid >> 3;
  if (g.map_slab == 1) {
    // The tiles of every z in one list cut into eight contiguous ranges,
    // one per XCD, so that no XCD idles when there are fewer than eight z.
    // Within a z the N tiles go in groups of gn and each group visits every
    // M tile: the ~32 workgroups one XCD holds at a time share both operand
    // tiles through its L2.
    const int tiles = nM * nN;
    const int64_t total = static_cast<int64_t>(tiles) * g.nbatch * g.nsplit;
    const int64_t per = (total + 7) / 8;
    const int64_t item = static_cast<int64_t>(x) * per + j;
    if (j >= per || item >= total) return false;
    z = static_cast<int>(item / tiles);
    const int r = static_cast<int>(item - static_cast<int64_t>(z) * tiles);
    const int gn = min(nN, max(1, (32 + nM - 1) / nM));
    const int grp = r / (nM * gn), n0 = grp * gn;
    const int width = min(gn, nN - n0);
    const int rem = r - grp * nM * gn;
    mt = rem / width;
    nt = n0 + rem % width;
    return true;
  }
  z = blockIdx.y;
  if (g.map_slab == 2) {
    nt = (j / nM) * 8 + x;
    mt = j % nM;
    return nt < nN;
  }
  if (nM >= 8) {
    mt = (j / nN) * 8 + x;
    nt = j % nN;
    return mt < nM;
  }
  mt = bid / nN;
  nt = bid % nN;
  return mt < nM;
}

// Grid of a launch for GemmArgs g and tile counts nM x nN.
inline dim3 grid_of(const GemmArgs& g, int nM, int nN) {
  const int nz = g.nbatch * g.nsplit;
  if (g.map_slab == 1) {
    const int64_t total = static_cast<int64_t>(nM) * nN * nz;
    return dim3(static_cast<unsigned>(8 * ((total + 7) / 8)), 1);
  }
  if (g.map_slab == 2) return dim3(8 * nM * ((nN + 7) / 8), nz);
  const int gx = nM >= 8 ? 8 * nN * ((nM + 7) / 8) : nM * nN;
  return dim3(gx, nz);
}

enum class GemmKind { kForward, kGbar, kDcoef, kDensity, kJastrow };
// kBF16P: BF16x3 products on operands pre-split into bf16 hi / lo planes.
// The values are part of the persisted tile-table keys.
enum class Prec { kF64 = 0, kF32 = 1, kBF16P = 3 };

// Launchers (return hipError_t of the launch).
// out_is_f32: 0 FP64, 1 FP32, 2 split bf16 planes (hi, lo; see AoOut::plane).
hipError_t launch_ao_vgl(const AoTables& t, const PointArgs& pts, const AoOut& out, int out_is_f32,
                         int fp32_compute, hipStream_t s);
// Screened evaluation of sorted points into an array that the previous
// screened evaluation (bitmap out.act_prev) left with zeros in all of its
// inactive chunks: an activity pass fills out.act (cleared by the caller),
// then the store pass writes only the shells of chunks active now, and zeros
// for the shells of chunks active before but not now.  Afterwards every
// inactive chunk holds zeros again.
hipError_t launch_ao_vgl_screened(const AoTables& t, const PointArgs& pts, const AoOut& out, int out_is_f32,
                                  hipStream_t s);
// Values only, one plane: element (k, p) at out.out[k*out.sK + p*out.sP].
hipError_t launch_ao_value(const AoTables& t, const PointArgs& pts, const AoOut& out, int out_is_f32,
                           hipStream_t s);
// Adds the cusp correction to mo_vgl[P][5][N] (FP64 or FP32) in place.
// Scratch: *count (cleared here) and list[2 P] for the (point, nucleus)
// pairs inside a sphere.
hipError_t launch_cusp(const CuspArgs& c, const PointArgs& pts, void* mo, int out_is_f32, int64_t N,
                       int32_t* count, int32_t* list, hipStream_t s);
// GEMM tile shape: WGM x WGN wavefronts of TM x TN 16x16 MFMA blocks, K step BK.
struct TileCfg {
  int wgm, wgn, tm, tn, bk;
  constexpr int bm() const { return 16 * wgm * tm; }
  constexpr int bn() const { return 16 * wgn * tn; }
};
int gemm_num_tiles(Prec prec);
TileCfg gemm_tile(Prec prec, int cfg);
size_t gemm_tile_lds_bytes(Prec prec, int cfg);
// Screened adjoint products in sorted point order (kind kGbar or kDcoef;
// FP64 or FP32 tile cfg).
hipError_t launch_gemm_screened_adj(GemmKind kind, Prec prec, int cfg, const GemmArgs& g, int w_is_f32,
                                    hipStream_t s);
// Screened forward product (FP64 or FP32 tile cfg; D in FP64 or FP32).
hipError_t launch_gemm_sparse(Prec prec, int cfg, const GemmArgs& g, int out_is_f32, hipStream_t s);
// Point sort by nearest nucleus (stable counting sort): perm[i] = original
// index of sorted point i.  key: P entries; scratch of
// sort_scratch_bytes(P, n_nuc) bytes; 1 <= n_nuc <= kSortMaxNuclei.
constexpr int kSortMaxNuclei = 16384;
size_t sort_scratch_bytes(int64_t P, int64_t n_nuc);
hipError_t launch_sort_points(const PointArgs& pts, const double* nuc_xyz, int64_t n_nuc, int32_t* key,
                              int32_t* perm, void* scratch, size_t scratch_bytes, hipStream_t s);
// Determinants det[b] and adjugates adj[b] (row-major n x n) of a batch of
// row-major n x n FP64 matrices, 1 <= n <= 32.
hipError_t launch_det_adj(int n, int64_t batch, const double* A, double* det, double* adj, hipStream_t s);
// Three-body Jastrow pieces (jastrow_kernels.hip; see there for layouts).
hipError_t launch_een_en(const PointArgs& pts, int64_t ne, const double* nuc, int64_t nn, double kappa, int mh,
                         double* ra, double* x, hipStream_t s);
// g0: scratch of 7 doubles per point.
hipError_t launch_een_ee(const PointArgs& pts, int64_t ne, int64_t nn, double kappa, int nord, const double* x,
                         const double* q0, double* g0, double* rt, double* j0, hipStream_t s);
hipError_t launch_een_finish(const double* part, int64_t slots, const double* j0, int64_t nw, int64_t ne,
                             double* J, hipStream_t s);
// The Jastrow product with its fused weighted reduction (FP64).
hipError_t launch_gemm_jastrow(int cfg, const GemmArgs& g, hipStream_t s);
// Rows of n values -> rows of ldd values (ldd >= n, a multiple of 4; zeros
// from n on; dst 16-byte aligned): FP64 -> FP32 (round to nearest), FP64 ->
// FP64 or FP32 -> FP32.
hipError_t launch_pad_rows(const void* src, int src_f32, void* dst, int dst_f32, int64_t rows, int64_t n,
                           int64_t ldd, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
// dst row q = src row perm[q] for q < rows (rows of row_bytes bytes, a
// multiple of 4).
hipError_t launch_gather_rows(const void* src, const int32_t* perm, int64_t rows, int64_t row_bytes, void* dst,
                              hipStream_t s);
// Density product (FP64 or FP32 tile cfg): partial row sums of
// occ[j] D(i, j)^2 per (N tile, wave) slot; see gemm_body.
hipError_t launch_gemm_density(Prec prec, int cfg, const GemmArgs& g, hipStream_t s);
hipError_t launch_gemm_typed(GemmKind kind, Prec prec, int cfg, const GemmArgs& g, int w_is_f32,
                             int out_is_f32, hipStream_t s);
// BF16x3 kernel on pre-split bf16 planes (gemm_bf16p.hip): g.A / g.A2 and
// g.B / g.B2 are the hi / lo planes; reached through launch_gemm_typed with
// Prec::kBF16P.
int gemm_bf16p_num_tiles();
TileCfg gemm_bf16p_tile(int cfg);
size_t gemm_bf16p_tile_lds_bytes(int cfg);
// screened = 1: the products of the screened contraction (points sorted by
// nearest nucleus, g.act / g.perm / g.act_words set as for the FP64 and FP32
// screened products; the W^T ao product needs Lchunk a multiple of 64 and at
// most kSparseMaxStages * 32).
hipError_t launch_gemm_bf16p(GemmKind kind, int cfg, const GemmArgs& g, int out_is_f32, int screened,
                             hipStream_t s);
// Resident workgroups per compute unit of the persistent form.
int gemm_bf16p_blocks_per_cu(GemmKind kind, int cfg, int out_is_f32);
// W[p][c][n] (P x 5 x N, FP64 or FP32) split into bf16 planes hi / lo laid
// out [Pp][5][Nw] (Nw a multiple of 8), zero beyond P and N.  perm != NULL:
// plane row p holds W row perm[p] (the screened products' point order).
hipError_t launch_split_w(const void* w, int w_is_f32, int64_t P, int64_t N, int64_t Pp, int64_t Nw,
                          const int32_t* perm, void* hi, void* lo, hipStream_t s);

// Autotuner (tuner.cpp).
struct GemmProblem {
  GemmKind kind;
  Prec prec;
  int w32, o32;
  int64_t M, N, L;
  int nbatch = 5;  // components per product (1: values only)
  int sparse = 0;  // screened forward product
};
bool tile_feasible(Prec prec, int cfg);
int default_tile(const GemmProblem& p);
// Returns the tile for p, timing every feasible tile through `enqueue` on
// stream s the first time p is seen.  *err receives a HIP error, if any.
int choose_tile(const GemmProblem& p, int device, hipStream_t s,
                const std::function<hipError_t(int)>& enqueue, hipError_t* err);
// The tile an earlier decision recorded for p (this process, or the
// persisted tables), else the least-padded-work tile; never times anything.
int cached_tile(const GemmProblem& p, int device);
void forget_tuning();
// Raw access to the tile cache (batch executor): -1 if absent.
int tune_cache_get(const std::string& key);
void tune_cache_put(const std::string& key, int cfg);
bool tuning_on();
std::string device_arch(int device);
hipError_t launch_reduce_splits(const double* ws, int64_t nz, int64_t rows, int64_t cols,
                                int64_t ld_ws, int64_t z_stride, double* out, int64_t ld_out,
                                hipStream_t s);
// ---------------------------------------------------------------------------
// Persistent (work-list) execution used by the batch executor: one launch
// of a grid sized to the GPU walks a list of items, each item naming a job
// (one molecule's arguments) and the block coordinates it stands for.
struct WorkItem {
  int32_t job, a, b, c;  // AO stages: a = point block, b = nucleus group;
                         // products: a = M tile, b = N tile, c = batch index z
};
struct AoJob {
  AoTables t;
  PointArgs pts;
  AoOut out;
};
struct AdjJob {
  AoTables t;
  PointArgs pts;
  const void* gbar;
  int64_t sK, sC;
  double* elec_out;
  int64_t elec_group_stride;
  double* nuc_partial;
};
// out[r*ld_out + c] = sum_z ws[z*z_stride + r*ld_ws + c] for r < rows, c < cols
struct RedJob {
  const double* ws;
  int64_t nz, rows, cols, ld_ws, z_stride;
  double* out;
  int64_t ld_out;
};
struct NucRedJob {
  const double* part;
  int64_t n_waves;
  int32_t nucl_dev, nucl_num;
  const int32_t* dev_of;
  double* out;
};

// out_is_f32: 0 FP64, 1 FP32, 2 bf16 hi / lo planes (out.plane apart), as
// for launch_ao_vgl.
hipError_t launch_ao_vgl_persist(const AoJob* jobs, const WorkItem* items, int n_items, int grid,
                                 size_t smem, int out_is_f32, hipStream_t s);
hipError_t launch_ao_adjoint_persist(const AdjJob* jobs, const WorkItem* items, int n_items,
                                     int grid, size_t smem, int gbar_is_f32, hipStream_t s);
hipError_t launch_gemm_persist(GemmKind kind, Prec prec, int cfg, const GemmArgs* jobs,
                               const WorkItem* items, int n_items, int grid, int w_is_f32,
                               int out_is_f32, hipStream_t s);
hipError_t launch_reduce_batch(const RedJob* jobs, const int64_t* prefix, int n_jobs, int64_t total,
                               hipStream_t s);
hipError_t launch_reduce_nuc_batch(const NucRedJob* jobs, const int64_t* prefix, int n_jobs,
                                   int64_t total, hipStream_t s);
// Persistent form of the pre-split BF16x3 kernel (no screening).
// occupancy != NULL: stores the resident workgroups per compute unit and
// launches nothing.
hipError_t launch_gemm_bf16p_persist(GemmKind kind, int cfg, const GemmArgs* jobs, const WorkItem* items,
                                     int n_items, int grid, int out_is_f32, int* occupancy, hipStream_t s);
// Whether the strides of g fit the 32-bit tile offsets of the pre-split
// kernel's loaders for tile cfg.
bool gemm_bf16p_args_ok(int cfg, const GemmArgs& g);
// Largest j with prefix[j] <= e (prefix[0] = 0, increasing): the job of
// flat element e in the batched element-wise kernels.
__device__ __forceinline__ int find_job(const int64_t* prefix, int n_jobs, int64_t e) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// Batched W split (batch executor): job j covers elements prefix[j] ..
// prefix[j+1]-1 of a flat range, one per eight weights of its planes (fewer
// than 2^32 per job).
struct SplitJob {
  const void* w;
  int64_t P, N, Pp, Nw;
  int32_t vec;
  void* hi;
  void* lo;
};
hipError_t launch_split_w_batch(const SplitJob* jobs, const int64_t* prefix, int n_jobs, int64_t total,
                                int w_is_f32, hipStream_t s);
// One molecule's weights copied into padded rows: rows rows of n values from
// src into rows of ldd (a multiple of 4, zeros from n on) at dst.
struct PadJob {
  const void* src;
  void* dst;
  int64_t rows, n, ldd;
};
// Every job of the list, same element type (FP32 when f32, else FP64);
// prefix[j] = sum of rows * ldd / 4 over the jobs before j, total the sum.
hipError_t launch_pad_rows_batch(const PadJob* jobs, const int64_t* prefix, int n_jobs, int64_t total, int f32,
                                 hipStream_t s);
// Resident blocks per compute unit of the persistent kernels.
int ao_persist_blocks_per_cu(int f32, size_t smem);
int adj_persist_blocks_per_cu(int f32, size_t smem);
int gemm_persist_blocks_per_cu(GemmKind kind, Prec prec, int cfg, int w_is_f32, int out_is_f32);

// Adjoint AO stage.  gbar: [ao][5][point] with strides (sK, sC, 1).
// elec_out + blockIdx.y*elec_group_stride receives sum_k t[p][k][:] of the
// group's nuclei as [point][3]; nuc_partial[(wave*nucl_dev + a)*3 + i]
// receives minus the wave's sum over its points for device nucleus a.
// Returns the number of waves through *n_waves.
hipError_t launch_ao_adjoint(const AoTables& t, const PointArgs& pts, const void* gbar,
                             int gbar_is_f32, int64_t sK, int64_t sC, double* elec_out,
                             int64_t elec_group_stride, double* nuc_partial, int64_t* n_waves,
                             hipStream_t s);
// d_nucl[A][i] = sum_w nuc_partial[(w*nucl_dev + dev_of[A])*3 + i], or 0 for
// nuclei without shells (dev_of[A] < 0).
hipError_t launch_reduce_nuc(const double* nuc_partial, int64_t n_waves, int32_t nucl_dev,
                             const int32_t* dev_of, int32_t nucl_num, double* d_nucl,
                             hipStream_t s);

}  // namespace qmk
