// Internal view of a context, shared by the context API (context.cpp) and
// the batch executor (batch.cpp).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/qmk.h"
#include "qmk_internal.h"

namespace qmk {

constexpr uint32_t kMagic = 0x514d4b43u;  // "QMKC"

inline int n_cart(int l) { return (l + 1) * (l + 2) / 2; }
inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, n > 0 ? n : 16);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = n;
    return hipSuccess;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(dev) == hipSuccess) ok = true;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace qmk

using qmk::DevBuf;

struct qmk_ctx_s {
  uint32_t magic = qmk::kMagic;
  int device = 0;
  std::string err;

  // time stamps: `date` moves with everything the AOs depend on
  int64_t date = 1;
  int32_t bits = 53;
  int32_t mode = QMK_FP64;

  int64_t nucl_num = 0;
  std::vector<double> nucl;

  bool has_basis = false;
  int64_t shell_num = 0, prim_num = 0, ao_num = 0;
  std::vector<int64_t> sh_nuc, sh_off;
  std::vector<int32_t> sh_l;
  std::vector<double> expo, coef, pf, sf, af;  // factors as used (given or computed)

  bool has_coef = false;
  int64_t mo_num = 0;
  std::vector<double> C;  // [mo][ao]

  bool has_points = false;
  int64_t walk_num = 0, elec_num = 0;
  char transp = 'N';
  const double* pts = nullptr;
  DevBuf own_pts;

  // device tables
  bool tables_dirty = true;
  DevBuf d_nuc, d_shell, d_prim, d_aofac, d_group, d_devof;
  qmk::AoTables tab{};
  int32_t n_groups = 0, nucl_dev = 0;

  // MO coefficient copies for the current mode
  bool coef_dirty = true;
  int coef_mode = -1;
  int64_t Kp = 0, Np = 0;
  DevBuf d_Ct, d_C;          // FP64 or FP32 copies: C^T [Kp][Np], C [Np][Kp]
  DevBuf d_Cb_hi, d_Cb_lo;   // BF16x3: C [Np][Kp] split into bf16 hi / lo
  DevBuf d_Ctb_hi, d_Ctb_lo; // BF16x3: C^T [Kp][Np] split

  // AO array [Kp][5][Pp] (double or float), valid at ao_date
  DevBuf ao;
  int64_t ao_Pp = 0, ao_Kp = 0, ao_date = -1;
  int ao_f32 = -1;
  // the adjoint's dC product reads the forward's AO array of the same points
  // (true) or evaluates the AO values again (false; qmk_set_ao_retention)
  bool ao_retain = true;

  // AO values only [Kp][Pp], valid at aov_date (used when the full AO array
  // is stale for the current points)
  DevBuf aov;
  int64_t aov_Pp = 0, aov_Kp = 0, aov_date = -1;
  int aov_f32 = -1;

  // density: occupied MOs compacted into Cocc^T [Kp][No_p] and occ [No_p]
  DevBuf d_Cocc_t, d_occ, ws_den;
  std::vector<double> occ_key;
  int64_t occ_coef_version = -1, n_occ = 0, Nop = 0;
  int occ_f32 = -1;
  int64_t coef_version = 0;

  // screened contraction: points sorted by nearest nucleus, the AO array in
  // that order [Kp][5][Pp] and its activity bitmap, valid at aos_date
  bool sparse = false;
  DevBuf d_sort_key, d_sort_scratch, d_perm, d_act, aos, d_nuc_xyz, w_sorted;
  // bitmap of the previous screened evaluation into aos (swapped with d_act)
  DevBuf d_act_prev;
  int64_t aos_Pp = 0, aos_Kp = 0, aos_date = -1, act_words = 0, nuc_xyz_version = -1;
  int aos_f32 = -1;

  // MO cusp correction: inputs, and device tables valid for cusp_key
  bool cusp_on = false;
  std::vector<double> cusp_charge, cusp_rc;
  int64_t cusp_version = 0, geom_version = 0;
  int64_t cusp_key[4] = {-1, -1, -1, -1};  // geom, coef, cusp versions, mode
  DevBuf d_cusp_nuc, d_cusp_s, d_cusp_prim, d_cusp_cs, d_cusp_f, d_cusp_pts, d_cusp_ao;
  DevBuf d_cusp_list;  // [0]: count of points inside a sphere; from [4]: (point, nucleus) pairs
  qmk::CuspArgs cusp{};

  // three-body Jastrow: operands of the product, rescaled e-n distances,
  // per-electron parts and m = 0 weight sums, weight polynomials and
  // per-wave partial sums
  DevBuf een_ra, een_x, een_rt, een_j0, een_g0, een_q, een_part;
  std::vector<double> een_key;  // coefficients and order behind een_q

  DevBuf gbar, ws_dc, ws_nuc, ws_elec;
  DevBuf w_f32;  // adjoint weights with padded rows: the FP32 copy of FP64 W (FP32 mode), or a copy
                 // of W whose own rows cannot be loaded in 16-byte pieces
  DevBuf w_split;  // adjoint weights as bf16 hi and lo planes [Pp][5][Nw] (BF16x3 mode)
  int64_t gbar_Pp = 0, gbar_Kp = 0;
  int gbar_f32 = -1;

  int64_t launches = 0;
  int forced_tile[5] = {-1, -1, -1, -1, -1};  // per GemmKind; -1 = autotuned

  // tracing: events around launches, per kernel class
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  double t_ms[QMK_KERNEL_CLASSES] = {};
  int64_t t_n[QMK_KERNEL_CLASSES] = {};
  ~qmk_ctx_s() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : event_pool) (void)hipEventDestroy(e);
  }

  int64_t P() const { return walk_num * elec_num; }
  bool f32_storage() const { return mode != QMK_FP64; }
  // layout of the context's AO array: 0 FP64, 1 FP32, 2 bf16 hi and lo
  // planes (the BF16x3 products read pre-split operands)
  int ao_format() const { return mode == QMK_FP64 ? 0 : (mode == QMK_MIXED_F32 ? 1 : 2); }
};


namespace qmk {

#define QMK_CHECK_CTX(ctx)                          \
  do {                                              \
    if (!qmk::valid_ctx(ctx)) return QMK_INVALID_CONTEXT; \
  } while (0)
#define QMK_HIP(ctx, expr, what)                               \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) return qmk::hip_fail(ctx, e_, what); \
  } while (0)

// Helpers of context.cpp used by the batch executor.
qmk_status fail(qmk_ctx ctx, qmk_status st, const std::string& msg);
qmk_status bad_arg(qmk_ctx ctx, int k, const std::string& msg);
qmk_status check_dev_arg(qmk_ctx ctx, int k, const void* p);
qmk_status hip_fail(qmk_ctx ctx, hipError_t e, const char* what);
bool valid_ctx(qmk_ctx ctx);
qmk_status ensure_tables(qmk_ctx ctx);
qmk_status ensure_coef(qmk_ctx ctx);
qmk_status check_ready(qmk_ctx ctx, bool need_coef);
PointArgs point_args(qmk_ctx ctx);
Prec gemm_prec(qmk_ctx ctx);
Prec product_prec(qmk_ctx ctx, GemmKind kind);
bool device_accessible(const void* p, int device);
// Arguments of the product Gbar[k][c][p] = sum_n W[p][c][n] C[n][k].  Both
// kernels compute Gbar with rows k and columns p; the FP64 / FP32 kernels read
// C [n][k] and W ([P][5][Nw]: rows of Nw >= N weights), the BF16x3 kernel the
// split C^T planes (Ct_hi / Ct_lo) and the split W planes (w / w_lo,
// [Pp][5][Nw]).
GemmArgs gbar_args(Prec prec, const void* w, const void* w_lo, int64_t Nw, const void* C, const void* Ct_hi,
                   const void* Ct_lo, void* gbar, int64_t P, int64_t Pp, int64_t K, int64_t Kp,
                   int64_t N, int64_t Np);

}  // namespace qmk
