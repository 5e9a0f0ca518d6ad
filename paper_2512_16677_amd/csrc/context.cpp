// Host runtime of the C ABI declared in include/qmk.h: contexts, input
// validation, basis preprocessing, time stamps and kernel orchestration.
//
// Structure follows the QMCkl paper's call model (Section 2.2): a context
// holds the inputs, the cached intermediates and their time stamps; a get
// call "provides" each dependency -- recomputing it only if its time stamp
// is older than the inputs it depends on -- and then computes the
// requested quantity.  Here the cached intermediate is the AO array (and
// the device copies of the basis tables and MO coefficients); the MO array
// is written straight into the caller's buffer by the contraction.
#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "ctx_internal.h"

using namespace qmk;

namespace {

thread_local std::string g_create_error;

// ---------------------------------------------------------------------------
// Normalisation (QMCkl paper, Section 3.1: the factors f_ks, N_s and M_n),
// written through Gaussian moments
//   I(n, alpha) = int t^(2n) exp(-alpha t^2) dt = Gamma(n + 1/2) alpha^-(n+1/2)
// f normalises the axis primitive x^l exp(-g r^2): f^-2 = I(l,2g) I(0,2g)^2;
// N_s normalises the contracted axis function; M(a,b,c)^2 is the ratio of the
// axis moment to the moment of x^a y^b z^c, which makes every Cartesian AO
// unit-norm.
double moment(int n, double alpha) {
  return std::tgamma(n + 0.5) / std::pow(alpha, n + 0.5);
}
double axis_norm2(int l, double alpha) {
  const double i0 = moment(0, alpha);
  return moment(l, alpha) * i0 * i0;
}

}  // namespace

namespace qmk {

qmk_status fail(qmk_ctx ctx, qmk_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}
qmk_status bad_arg(qmk_ctx ctx, int k, const std::string& msg) {
  return fail(ctx, QMK_INVALID_ARG_BASE + k, "argument " + std::to_string(k) + ": " + msg);
}
qmk_status hip_fail(qmk_ctx ctx, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(ctx, QMK_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
  return fail(ctx, QMK_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
}
bool valid_ctx(qmk_ctx ctx) { return ctx != nullptr && ctx->magic == kMagic; }

// True if the GPU `device` can read and write p: device memory of that GPU,
// managed memory, or pinned host memory mapped into the device's address
// space.  Pageable host memory (or an unknown address) is rejected before
// any kernel would touch it.
bool device_accessible(const void* p, int device) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  switch (a.type) {
    case hipMemoryTypeDevice:
    case hipMemoryTypeArray:
      return a.device == device;
    case hipMemoryTypeManaged:
    case hipMemoryTypeUnified:
      return true;
    case hipMemoryTypeHost:
      return a.devicePointer != nullptr;
    default:
      return false;
  }
}

qmk_status check_dev_arg(qmk_ctx ctx, int k, const void* p) {
  if (!p) return bad_arg(ctx, k, "NULL");
  if (!device_accessible(p, ctx->device)) return bad_arg(ctx, k, "not memory the device can access");
  return QMK_OK;
}

hipEvent_t take_event(qmk_ctx ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events when timing is enabled.
struct LaunchTimer {
  qmk_ctx ctx;
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr;
  LaunchTimer(qmk_ctx c, int k, hipStream_t st) : ctx(c), kind(k), s(st) {
    ++ctx->launches;
    if (!ctx->timing) return;
    a = take_event(ctx);
    if (a) (void)hipEventRecord(a, s);
  }
  ~LaunchTimer() {
    if (!a) return;
    hipEvent_t b = take_event(ctx);
    if (!b) {
      ctx->event_pool.push_back(a);
      return;
    }
    (void)hipEventRecord(b, s);
    ctx->pending.push_back({kind, a, b});
  }
};

void collect_timing(qmk_ctx ctx) {
  for (auto& p : ctx->pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->t_ms[p.kind] += ms;
      ctx->t_n[p.kind] += 1;
    }
    ctx->event_pool.push_back(p.a);
    ctx->event_pool.push_back(p.b);
  }
  ctx->pending.clear();
}

// Builds the device nucleus / shell / primitive tables and nucleus groups.
qmk_status build_tables(qmk_ctx ctx) {
  const int64_t S = ctx->shell_num;
  std::vector<std::vector<int64_t>> shells_of(ctx->nucl_num);
  for (int64_t s = 0; s < S; ++s) shells_of[ctx->sh_nuc[s]].push_back(s);
  std::vector<int64_t> ao_off(S + 1, 0);
  for (int64_t s = 0; s < S; ++s) ao_off[s + 1] = ao_off[s] + n_cart(ctx->sh_l[s]);

  std::vector<NucDev> nuc;
  std::vector<ShellDev> shell;
  std::vector<PrimDev> prim;
  std::vector<NucGroup> group;
  std::vector<int32_t> dev_of(ctx->nucl_num, -1);
  NucGroup cur{0, 0, 0, 0, 0, 0, 0, 0};
  size_t smem = 0;
  auto close_group = [&]() {
    if (cur.nuc_end > cur.nuc_begin) {
      group.push_back(cur);
      smem = std::max(smem, (cur.p_end - cur.p_begin) * sizeof(PrimDev) +
                                (cur.sh_end - cur.sh_begin) * sizeof(ShellDev) +
                                (cur.nuc_end - cur.nuc_begin) * sizeof(NucDev));
    }
    cur = NucGroup{(int32_t)nuc.size(), (int32_t)nuc.size(), (int32_t)shell.size(),
                   (int32_t)shell.size(), (int32_t)prim.size(), (int32_t)prim.size(), 0, 0};
  };
  for (int64_t A = 0; A < ctx->nucl_num; ++A) {
    if (shells_of[A].empty()) continue;
    int64_t np = 0;
    for (int64_t s : shells_of[A]) np += ctx->sh_off[s + 1] - ctx->sh_off[s];
    const int64_t nsh = static_cast<int64_t>(shells_of[A].size());
    int64_t nao = 0;
    for (int64_t s : shells_of[A]) nao += n_cart(ctx->sh_l[s]);
    if (np > kGroupMaxPrim || nsh > kGroupMaxShell)
      return fail(ctx, QMK_UNSUPPORTED, "nucleus " + std::to_string(A) + " has more than " +
                                            std::to_string(kGroupMaxPrim) + " primitives or " +
                                            std::to_string(kGroupMaxShell) + " shells");
    if ((cur.p_end - cur.p_begin) + np > kGroupMaxPrim ||
        (cur.sh_end - cur.sh_begin) + nsh > kGroupMaxShell ||
        (cur.nuc_end - cur.nuc_begin) + 1 > kGroupMaxNuc ||
        (cur.n_ao > 0 && cur.n_ao + nao > kGroupMaxAo))
      close_group();
    NucDev nd{};
    nd.x = ctx->nucl[3 * A];
    nd.y = ctx->nucl[3 * A + 1];
    nd.z = ctx->nucl[3 * A + 2];
    nd.gmin = INFINITY;
    nd.sh_begin = static_cast<int32_t>(shell.size()) - cur.sh_begin;
    nd.orig = static_cast<int32_t>(A);
    for (int64_t s : shells_of[A]) {
      ShellDev sd{};
      sd.ao_off = static_cast<int32_t>(ao_off[s]);
      sd.l = ctx->sh_l[s];
      sd.p_begin = static_cast<int32_t>(prim.size()) - cur.p_begin;
      // primitives of the shell by ascending exponent (Section 3.1)
      std::vector<int64_t> order(ctx->sh_off[s + 1] - ctx->sh_off[s]);
      std::iota(order.begin(), order.end(), ctx->sh_off[s]);
      std::stable_sort(order.begin(), order.end(),
                       [&](int64_t a, int64_t b) { return ctx->expo[a] < ctx->expo[b]; });
      for (int64_t k : order) {
        PrimDev pd{ctx->expo[k], ctx->coef[k] * ctx->pf[k] * ctx->sf[s]};
        prim.push_back(pd);
        nd.gmin = std::min(nd.gmin, ctx->expo[k]);
      }
      sd.p_end = static_cast<int32_t>(prim.size()) - cur.p_begin;
      shell.push_back(sd);
    }
    nd.sh_end = static_cast<int32_t>(shell.size()) - cur.sh_begin;
    dev_of[A] = static_cast<int32_t>(nuc.size());
    nuc.push_back(nd);
    cur.nuc_end = static_cast<int32_t>(nuc.size());
    cur.sh_end = static_cast<int32_t>(shell.size());
    cur.p_end = static_cast<int32_t>(prim.size());
    cur.n_ao += static_cast<int32_t>(nao);
  }
  close_group();
  if (group.empty()) return fail(ctx, QMK_NOT_SET, "basis has no shells");

  auto up = [&](DevBuf& b, const void* src, size_t n) -> hipError_t {
    hipError_t e = b.ensure(n);
    if (e != hipSuccess) return e;
    return hipMemcpy(b.p, src, n, hipMemcpyHostToDevice);
  };
  QMK_HIP(ctx, up(ctx->d_nuc, nuc.data(), nuc.size() * sizeof(NucDev)), "upload nuclei");
  QMK_HIP(ctx, up(ctx->d_shell, shell.data(), shell.size() * sizeof(ShellDev)), "upload shells");
  QMK_HIP(ctx, up(ctx->d_prim, prim.data(), prim.size() * sizeof(PrimDev)), "upload primitives");
  QMK_HIP(ctx, up(ctx->d_aofac, ctx->af.data(), ctx->af.size() * sizeof(double)), "upload M");
  QMK_HIP(ctx, up(ctx->d_group, group.data(), group.size() * sizeof(NucGroup)), "upload groups");
  QMK_HIP(ctx, up(ctx->d_devof, dev_of.data(), dev_of.size() * sizeof(int32_t)), "upload map");

  ctx->n_groups = static_cast<int32_t>(group.size());
  ctx->nucl_dev = static_cast<int32_t>(nuc.size());
  AoTables& t = ctx->tab;
  t.nuc = ctx->d_nuc.as<NucDev>();
  t.shell = ctx->d_shell.as<ShellDev>();
  t.prim = ctx->d_prim.as<PrimDev>();
  t.ao_factor = ctx->d_aofac.as<double>();
  t.group = ctx->d_group.as<NucGroup>();
  t.n_groups = ctx->n_groups;
  t.ao_num = static_cast<int32_t>(ctx->ao_num);
  t.smem_bytes = static_cast<int32_t>(smem);
  t.nucl_dev = ctx->nucl_dev;
  ctx->tables_dirty = false;
  return QMK_OK;
}

qmk_status ensure_tables(qmk_ctx ctx) {
  if (ctx->tables_dirty) {
    qmk_status st = build_tables(ctx);
    if (st != QMK_OK) return st;
  }
  ctx->tab.T = (ctx->bits - 1) * std::log(2.0);
  return QMK_OK;
}

// Round-to-nearest-even FP32 -> BF16 (bit pattern) and back.
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
float bf16_value(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

qmk_status ensure_coef(qmk_ctx ctx) {
  const int want = ctx->mode == QMK_FP64 ? 0 : (ctx->mode == QMK_MIXED_F32 ? 1 : 2);
  if (!ctx->coef_dirty && ctx->coef_mode == want) return QMK_OK;
  if (want == 2) {
    // C split once into bf16 hi + lo (hi = bf16(c), lo = bf16(c - hi)), in
    // the two layouts the products read: [n][k] and [k][n].
    const int64_t K = ctx->ao_num, N = ctx->mo_num;
    ctx->Kp = round_up(K, kAoPad);
    ctx->Np = round_up(N, kMoPad);
    const int64_t Kp = ctx->Kp, Np = ctx->Np;
    std::vector<uint16_t> ch(Kp * Np, 0), cl(Kp * Np, 0), th(Kp * Np, 0), tl(Kp * Np, 0);
    for (int64_t n = 0; n < N; ++n)
      for (int64_t k = 0; k < K; ++k) {
        const double v = ctx->C[n * K + k];
        const uint16_t h = bf16_bits(static_cast<float>(v));
        const uint16_t l = bf16_bits(static_cast<float>(v - static_cast<double>(bf16_value(h))));
        ch[n * Kp + k] = h;
        cl[n * Kp + k] = l;
        th[k * Np + n] = h;
        tl[k * Np + n] = l;
      }
    const size_t bytes = static_cast<size_t>(Kp * Np) * 2;
    DevBuf* bufs[4] = {&ctx->d_Cb_hi, &ctx->d_Cb_lo, &ctx->d_Ctb_hi, &ctx->d_Ctb_lo};
    const std::vector<uint16_t>* src[4] = {&ch, &cl, &th, &tl};
    for (int i = 0; i < 4; ++i) {
      QMK_HIP(ctx, bufs[i]->ensure(bytes), "alloc split C");
      QMK_HIP(ctx, hipMemcpy(bufs[i]->p, src[i]->data(), bytes, hipMemcpyHostToDevice), "upload split C");
    }
    // the FP32 copies below serve the value-only products, which have no
    // BF16x3 form
  }
  const int64_t K = ctx->ao_num, N = ctx->mo_num;
  ctx->Kp = round_up(K, kAoPad);
  ctx->Np = round_up(N, kMoPad);
  const int64_t Kp = ctx->Kp, Np = ctx->Np;
  const size_t esz = want ? sizeof(float) : sizeof(double);
  std::vector<unsigned char> ct(static_cast<size_t>(Kp * Np) * esz, 0), cn(ct.size(), 0);
  for (int64_t n = 0; n < N; ++n)
    for (int64_t k = 0; k < K; ++k) {
      const double v = ctx->C[n * K + k];
      if (want) {
        reinterpret_cast<float*>(ct.data())[k * Np + n] = static_cast<float>(v);
        reinterpret_cast<float*>(cn.data())[n * Kp + k] = static_cast<float>(v);
      } else {
        reinterpret_cast<double*>(ct.data())[k * Np + n] = v;
        reinterpret_cast<double*>(cn.data())[n * Kp + k] = v;
      }
    }
  QMK_HIP(ctx, ctx->d_Ct.ensure(ct.size()), "alloc C^T");
  QMK_HIP(ctx, hipMemcpy(ctx->d_Ct.p, ct.data(), ct.size(), hipMemcpyHostToDevice), "upload C^T");
  QMK_HIP(ctx, ctx->d_C.ensure(cn.size()), "alloc C");
  QMK_HIP(ctx, hipMemcpy(ctx->d_C.p, cn.data(), cn.size(), hipMemcpyHostToDevice), "upload C");
  ctx->coef_dirty = false;
  ctx->coef_mode = want;
  return QMK_OK;
}

PointArgs point_args(qmk_ctx ctx) {
  PointArgs a{};
  a.coord = ctx->pts;
  a.P = ctx->P();
  if (ctx->transp == 'N') {
    a.s_pt = 3;
    a.s_ax = 1;
  } else {
    a.s_pt = 1;
    a.s_ax = a.P;
  }
  return a;
}

qmk_status check_ready(qmk_ctx ctx, bool need_coef) {
  if (ctx->nucl_num <= 0) return fail(ctx, QMK_NOT_SET, "nuclei not set");
  if (!ctx->has_basis) return fail(ctx, QMK_NOT_SET, "basis not set");
  if (!ctx->has_points) return fail(ctx, QMK_NOT_SET, "points not set");
  if (need_coef) {
    if (!ctx->has_coef) return fail(ctx, QMK_NOT_SET, "MO coefficients not set");
    if (ctx->C.size() != static_cast<size_t>(ctx->mo_num * ctx->ao_num))
      return fail(ctx, QMK_NOT_SET, "MO coefficients do not match the basis (ao_num changed)");
  }
  return QMK_OK;
}

// provide(ao_vgl): recompute the AO array iff its time stamp is stale (or
// `force`: the adjoint with AO retention off).
qmk_status provide_ao(qmk_ctx ctx, hipStream_t s, bool force = false) {
  qmk_status st = ensure_tables(ctx);
  if (st != QMK_OK) return st;
  // 0: FP64; 1: FP32; 2: bf16 hi and lo planes (BF16x3 mode), same bytes as FP32
  const int f32 = ctx->ao_format();
  const int64_t Pp = round_up(ctx->P(), kPointPad), Kp = round_up(ctx->ao_num, kAoPad);
  if (!force && ctx->ao_date == ctx->date && ctx->ao_f32 == f32 && ctx->ao_Pp == Pp && ctx->ao_Kp == Kp)
    return QMK_OK;
  if (ctx->ao_Pp != Pp || ctx->ao_Kp != Kp || ctx->ao_f32 != f32 || !ctx->ao.p) {
    const size_t bytes = static_cast<size_t>(Kp * 5 * Pp) * (f32 ? 4 : 8);
    ctx->ao.release();
    QMK_HIP(ctx, ctx->ao.ensure(bytes), "alloc AO array");
    // padding rows (AO >= ao_num, point >= P) stay zero for the contractions
    QMK_HIP(ctx, hipMemsetAsync(ctx->ao.p, 0, bytes, s), "clear AO array");
    ctx->ao_Pp = Pp;
    ctx->ao_Kp = Kp;
    ctx->ao_f32 = f32;
  }
  AoOut o{ctx->ao.p, 5 * Pp, Pp, 1};
  o.plane = Kp * 5 * Pp;
  {
    LaunchTimer lt(ctx, QMK_KERNEL_AO, s);
    QMK_HIP(ctx, launch_ao_vgl(ctx->tab, point_args(ctx), o, f32, f32, s), "AO kernel");
  }
  ctx->ao_date = ctx->date;
  return QMK_OK;
}

// Tile for one product: forced by qmk_set_tile, else the autotuner's choice.
// Screened contraction input: the points sorted by nearest nucleus, the AO
// array in that order and the (64-point block, 16-AO chunk) activity bitmap.
qmk_status provide_ao_sorted(qmk_ctx ctx, hipStream_t s, bool force = false) {
  qmk_status st = ensure_tables(ctx);
  if (st != QMK_OK) return st;
  const int f32 = ctx->ao_format();  // 0 FP64, 1 FP32, 2 bf16 hi and lo planes
  const int64_t P = ctx->P(), Pp = round_up(P, kPointPad), Kp = round_up(ctx->ao_num, kAoPad);
  if (!force && ctx->aos_date == ctx->date && ctx->aos_f32 == f32 && ctx->aos_Pp == Pp && ctx->aos_Kp == Kp)
    return QMK_OK;
  const int64_t nn = ctx->nucl_num;
  if (nn > kSortMaxNuclei)
    return fail(ctx, QMK_UNSUPPORTED,
                "the screened evaluation sorts points by nearest nucleus for at most " +
                    std::to_string(kSortMaxNuclei) + " nuclei");
  if (ctx->nuc_xyz_version != ctx->geom_version) {
    QMK_HIP(ctx, ctx->d_nuc_xyz.ensure(static_cast<size_t>(3 * nn) * 8), "alloc nuclei");
    QMK_HIP(ctx, hipMemcpy(ctx->d_nuc_xyz.p, ctx->nucl.data(), static_cast<size_t>(3 * nn) * 8,
                           hipMemcpyHostToDevice), "upload nuclei");
    ctx->nuc_xyz_version = ctx->geom_version;
  }
  QMK_HIP(ctx, ctx->d_sort_key.ensure(static_cast<size_t>(P) * 4), "alloc sort keys");
  QMK_HIP(ctx, ctx->d_perm.ensure(static_cast<size_t>(P) * 4), "alloc permutation");
  const size_t scratch = std::max<size_t>(sort_scratch_bytes(P, nn), 16);
  QMK_HIP(ctx, ctx->d_sort_scratch.ensure(scratch), "alloc sort scratch");
  ctx->act_words = (Kp / kSparseChunk + 31) / 32;
  const int64_t act_n = (Pp / 64) * ctx->act_words;
  // the previous evaluation's bitmap tells which chunks of the array still
  // hold non-zeros (the store pass writes no inactive chunk otherwise)
  std::swap(ctx->d_act.p, ctx->d_act_prev.p);
  std::swap(ctx->d_act.bytes, ctx->d_act_prev.bytes);
  QMK_HIP(ctx, ctx->d_act.ensure(static_cast<size_t>(act_n) * 4), "alloc activity bitmap");
  const bool fresh = ctx->aos_Pp != Pp || ctx->aos_Kp != Kp || ctx->aos_f32 != f32 || !ctx->aos.p ||
                     ctx->d_act_prev.bytes < static_cast<size_t>(act_n) * 4;
  if (fresh) {
    const size_t bytes = static_cast<size_t>(Kp * 5 * Pp) * (f32 ? 4 : 8);
    ctx->aos.release();
    QMK_HIP(ctx, ctx->aos.ensure(bytes), "alloc sorted AO array");
    QMK_HIP(ctx, hipMemsetAsync(ctx->aos.p, 0, bytes, s), "clear sorted AO array");
    ctx->aos_Pp = Pp;
    ctx->aos_Kp = Kp;
    ctx->aos_f32 = f32;
    // an all-zero array: no chunk was active before
    QMK_HIP(ctx, ctx->d_act_prev.ensure(static_cast<size_t>(act_n) * 4), "alloc activity bitmap");
    QMK_HIP(ctx, launch_fill_u32(ctx->d_act_prev.as<uint32_t>(), act_n, 0u, s), "clear activity bitmap");
  }
  PointArgs pa = point_args(ctx);
  {
    LaunchTimer lt(ctx, QMK_KERNEL_SORT, s);
    QMK_HIP(ctx, launch_sort_points(pa, ctx->d_nuc_xyz.as<double>(), nn, ctx->d_sort_key.as<int32_t>(),
                                    ctx->d_perm.as<int32_t>(), ctx->d_sort_scratch.p, scratch, s),
            "sort points");
    QMK_HIP(ctx, launch_fill_u32(ctx->d_act.as<uint32_t>(), act_n, 0u, s), "clear activity bitmap");
  }
  pa.perm = ctx->d_perm.as<int32_t>();
  AoOut o{ctx->aos.p, 5 * Pp, Pp, 1, ctx->d_act.as<uint32_t>(), ctx->act_words, ctx->d_act_prev.as<uint32_t>()};
  o.plane = Kp * 5 * Pp;
  {
    LaunchTimer lt(ctx, QMK_KERNEL_AO, s);
    QMK_HIP(ctx, launch_ao_vgl_screened(ctx->tab, pa, o, f32, s), "AO kernel (sorted points)");
  }
  ctx->aos_date = ctx->date;
  return QMK_OK;
}

// AO values for the current points: the value plane of the full AO array
// when that is current, else the value-only kernel into its own plane.
// Returns the plane and its AO-row stride.
qmk_status provide_ao_value(qmk_ctx ctx, hipStream_t s, const void** plane, int64_t* row_stride) {
  qmk_status st = ensure_tables(ctx);
  if (st != QMK_OK) return st;
  const int f32 = ctx->f32_storage() ? 1 : 0;
  const int64_t Pp = round_up(ctx->P(), kPointPad), Kp = round_up(ctx->ao_num, kAoPad);
  if (ctx->ao_date == ctx->date && ctx->ao_f32 == f32 && ctx->ao_Pp == Pp && ctx->ao_Kp == Kp) {
    *plane = ctx->ao.p;
    *row_stride = 5 * Pp;
    return QMK_OK;
  }
  *plane = nullptr;
  *row_stride = Pp;
  if (ctx->aov_date == ctx->date && ctx->aov_f32 == f32 && ctx->aov_Pp == Pp && ctx->aov_Kp == Kp) {
    *plane = ctx->aov.p;
    return QMK_OK;
  }
  if (ctx->aov_Pp != Pp || ctx->aov_Kp != Kp || ctx->aov_f32 != f32 || !ctx->aov.p) {
    const size_t bytes = static_cast<size_t>(Kp * Pp) * (f32 ? 4 : 8);
    ctx->aov.release();
    QMK_HIP(ctx, ctx->aov.ensure(bytes), "alloc AO value plane");
    QMK_HIP(ctx, hipMemsetAsync(ctx->aov.p, 0, bytes, s), "clear AO value plane");
    ctx->aov_Pp = Pp;
    ctx->aov_Kp = Kp;
    ctx->aov_f32 = f32;
  }
  AoOut o{ctx->aov.p, Pp, 0, 1};
  {
    LaunchTimer lt(ctx, QMK_KERNEL_AO, s);
    QMK_HIP(ctx, launch_ao_value(ctx->tab, point_args(ctx), o, f32, s), "AO value kernel");
  }
  ctx->aov_date = ctx->date;
  *plane = ctx->aov.p;
  return QMK_OK;
}

// Solves the 4x4 system a f = b (Gaussian elimination, partial pivoting);
// false if it is singular.
bool solve4(double a[4][4], double b[4], double f[4]) {
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
    if (a[piv][c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < 4; ++k) std::swap(a[c][k], a[piv][k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < 4; ++r) {
      const double m = a[r][c] / a[c][c];
      for (int k = c; k < 4; ++k) a[r][k] -= m * a[c][k];
      b[r] -= m * b[c];
    }
  }
  for (int c = 3; c >= 0; --c) {
    double v = b[c];
    for (int k = c + 1; k < 4; ++k) v -= a[c][k] * f[k];
    f[c] = v / a[c][c];
  }
  return true;
}

// Cusp tables for the current nuclei, basis, precision and coefficients
// (Section 3.3).  With r = |r - R_A|, R = r_A, Z = charge of A and
// phi^s the radial s part of MO i on A, the coefficients solve
//   p(R) = phi^s(R),  p'(R) = phi^s'(R),  p''(R) = phi^s''(R),
//   p'(0) = -Z (phi(R_A) - phi^s(R_A) + p(0))
// with p(r) = f0 + f1 r + f2 r^2 + f3 r^3.  phi(R_A) comes from the AO values
// at the nuclei computed by the value-only AO kernel; phi^s and its radial
// derivatives at R from the folded primitives, with the AO stage's cutoff.
qmk_status ensure_cusp(qmk_ctx ctx, hipStream_t s) {
  const int64_t key[4] = {ctx->geom_version, ctx->coef_version, ctx->cusp_version, ctx->mode};
  if (std::equal(key, key + 4, ctx->cusp_key)) return QMK_OK;
  qmk_status st = ensure_tables(ctx);
  if (st != QMK_OK) return st;
  const int64_t nn = ctx->nucl_num, K = ctx->ao_num, N = ctx->mo_num;
  const double* R = ctx->nucl.data();
  for (int64_t a = 0; a < nn; ++a)
    for (int64_t b = a + 1; b < nn; ++b) {
      if (ctx->cusp_rc[a] <= 0.0 || ctx->cusp_rc[b] <= 0.0) continue;
      const double dx = R[3 * a] - R[3 * b], dy = R[3 * a + 1] - R[3 * b + 1], dz = R[3 * a + 2] - R[3 * b + 2];
      if (ctx->cusp_rc[a] + ctx->cusp_rc[b] >= std::sqrt(dx * dx + dy * dy + dz * dz))
        return fail(ctx, QMK_INVALID_ARG_BASE + 4,
                    "cusp spheres of nuclei " + std::to_string(a) + " and " + std::to_string(b) + " overlap");
    }
  // AO offsets and s shells per nucleus
  std::vector<int64_t> ao_off(ctx->shell_num + 1, 0);
  for (int64_t sh = 0; sh < ctx->shell_num; ++sh) ao_off[sh + 1] = ao_off[sh] + n_cart(ctx->sh_l[sh]);
  std::vector<std::vector<int64_t>> s_shells(nn);
  for (int64_t sh = 0; sh < ctx->shell_num; ++sh)
    if (ctx->sh_l[sh] == 0) s_shells[ctx->sh_nuc[sh]].push_back(sh);

  // AO values at every nucleus (value-only kernel, FP64)
  const int64_t Kp = round_up(K, kAoPad);
  QMK_HIP(ctx, ctx->d_cusp_pts.ensure(static_cast<size_t>(3 * nn) * 8), "alloc cusp points");
  QMK_HIP(ctx, hipMemcpyAsync(ctx->d_cusp_pts.p, R, static_cast<size_t>(3 * nn) * 8, hipMemcpyHostToDevice, s),
          "upload cusp points");
  QMK_HIP(ctx, ctx->d_cusp_ao.ensure(static_cast<size_t>(Kp * nn) * 8), "alloc cusp AO values");
  PointArgs pa{};
  pa.coord = ctx->d_cusp_pts.as<double>();
  pa.s_pt = 3;
  pa.s_ax = 1;
  pa.P = nn;
  AoOut o{ctx->d_cusp_ao.p, nn, 0, 1};
  QMK_HIP(ctx, launch_ao_value(ctx->tab, pa, o, 0, s), "AO values at the nuclei");
  std::vector<double> chi(static_cast<size_t>(K * nn));
  QMK_HIP(ctx, hipMemcpyAsync(chi.data(), ctx->d_cusp_ao.p, chi.size() * 8, hipMemcpyDeviceToHost, s),
          "download AO values at the nuclei");
  QMK_HIP(ctx, hipStreamSynchronize(s), "wait for AO values at the nuclei");

  std::vector<CuspNuc> cn;
  std::vector<CuspS> cs;
  std::vector<PrimDev> cp;
  std::vector<double> ccs, cf;
  const double T = (ctx->bits - 1) * std::log(2.0);
  for (int64_t a = 0; a < nn; ++a) {
    const double rc = ctx->cusp_rc[a];
    if (rc <= 0.0) continue;
    CuspNuc nu{R[3 * a], R[3 * a + 1], R[3 * a + 2], rc, static_cast<int32_t>(cs.size()), 0, 0, 0};
    const double u = rc * rc;
    std::vector<double> v(N, 0.0), v1(N, 0.0), v2(N, 0.0), phiA(N, 0.0), phisA(N, 0.0);
    for (int64_t sh : s_shells[a]) {
      const int64_t k = ao_off[sh];
      CuspS sd{ctx->af[k], static_cast<int32_t>(cp.size()), 0};
      std::vector<int64_t> order(ctx->sh_off[sh + 1] - ctx->sh_off[sh]);
      std::iota(order.begin(), order.end(), ctx->sh_off[sh]);
      std::stable_sort(order.begin(), order.end(),
                       [&](int64_t x, int64_t y) { return ctx->expo[x] < ctx->expo[y]; });
      double g0 = 0.0, g1 = 0.0, g2 = 0.0;
      for (int64_t q : order) {
        const PrimDev pd{ctx->expo[q], ctx->coef[q] * ctx->pf[q] * ctx->sf[sh]};
        cp.push_back(pd);
        const double x = pd.gamma * u;
        if (x >= T) continue;
        const double e = pd.coef * std::exp(-x);
        g0 += e;
        g1 -= pd.gamma * e;
        g2 += pd.gamma * pd.gamma * e;
      }
      sd.p_end = static_cast<int32_t>(cp.size());
      cs.push_back(sd);
      const double c0 = sd.m * g0, c1 = sd.m * 2.0 * rc * g1, c2 = sd.m * (2.0 * g1 + 4.0 * u * g2);
      for (int64_t i = 0; i < N; ++i) {
        const double cik = ctx->C[i * K + k];
        ccs.push_back(cik);
        v[i] += cik * c0;
        v1[i] += cik * c1;
        v2[i] += cik * c2;
        phisA[i] += cik * chi[k * nn + a];
      }
    }
    nu.s_end = static_cast<int32_t>(cs.size());
    for (int64_t i = 0; i < N; ++i) {
      double acc = 0.0;
      for (int64_t k = 0; k < K; ++k) acc += ctx->C[i * K + k] * chi[k * nn + a];
      phiA[i] = acc;
    }
    const double Z = ctx->cusp_charge[a];
    const size_t base = cf.size();
    cf.resize(base + 4 * N);
    for (int64_t i = 0; i < N; ++i) {
      double m[4][4] = {{1.0, rc, rc * rc, rc * rc * rc},
                        {0.0, 1.0, 2.0 * rc, 3.0 * rc * rc},
                        {0.0, 0.0, 2.0, 6.0 * rc},
                        {Z, 1.0, 0.0, 0.0}};
      double b[4] = {v[i], v1[i], v2[i], -Z * (phiA[i] - phisA[i])};
      double f[4];
      if (!solve4(m, b, f))
        return fail(ctx, QMK_INVALID_ARG_BASE + 4, "cusp conditions are singular at nucleus " + std::to_string(a));
      for (int q = 0; q < 4; ++q) cf[base + q * N + i] = f[q];
    }
    cn.push_back(nu);
  }
  auto up = [&](DevBuf& b, const void* src, size_t n) -> hipError_t {
    hipError_t e = b.ensure(std::max<size_t>(n, 16));
    if (e != hipSuccess || n == 0) return e;
    return hipMemcpy(b.p, src, n, hipMemcpyHostToDevice);
  };
  QMK_HIP(ctx, up(ctx->d_cusp_nuc, cn.data(), cn.size() * sizeof(CuspNuc)), "upload cusp nuclei");
  QMK_HIP(ctx, up(ctx->d_cusp_s, cs.data(), cs.size() * sizeof(CuspS)), "upload cusp s AOs");
  QMK_HIP(ctx, up(ctx->d_cusp_prim, cp.data(), cp.size() * sizeof(PrimDev)), "upload cusp primitives");
  QMK_HIP(ctx, up(ctx->d_cusp_cs, ccs.data(), ccs.size() * 8), "upload cusp coefficients");
  QMK_HIP(ctx, up(ctx->d_cusp_f, cf.data(), cf.size() * 8), "upload cusp polynomials");
  CuspArgs& c = ctx->cusp;
  c.nuc = ctx->d_cusp_nuc.as<CuspNuc>();
  c.s = ctx->d_cusp_s.as<CuspS>();
  c.prim = ctx->d_cusp_prim.as<PrimDev>();
  c.cs = ctx->d_cusp_cs.as<double>();
  c.f = ctx->d_cusp_f.as<double>();
  c.T = T;
  c.n_nuc = static_cast<int32_t>(cn.size());
  std::copy(key, key + 4, ctx->cusp_key);
  return QMK_OK;
}

// Precision a product of this kind runs in under the context's mode: the
// Jastrow product is FP64 always; the density product has no BF16x3 form
// and runs FP32 in that mode.
Prec product_prec(qmk_ctx ctx, GemmKind kind) {
  if (kind == GemmKind::kJastrow) return Prec::kF64;
  const Prec p = gemm_prec(ctx);
  return kind == GemmKind::kDensity && p == Prec::kBF16P ? Prec::kF32 : p;
}

qmk_status pick_tile(qmk_ctx ctx, const GemmProblem& pb, hipStream_t s,
                     const std::function<hipError_t(int)>& enqueue, int* cfg) {
  const int forced = ctx->forced_tile[static_cast<int>(pb.kind)];
  if (forced >= 0) {
    // a tile forced under another precision mode may not exist in this one
    if (forced >= gemm_num_tiles(pb.prec) || !tile_feasible(pb.prec, forced))
      return fail(ctx, QMK_INVALID_ARG_BASE + 3, "the forced tile does not exist for this product's precision");
    *cfg = forced;
    return QMK_OK;
  }
  hipError_t e = hipSuccess;
  *cfg = choose_tile(pb, ctx->device, s, enqueue, &e);
  if (e != hipSuccess) return hip_fail(ctx, e, "tile autotuning");
  return QMK_OK;
}

Prec gemm_prec(qmk_ctx ctx) {
  return ctx->mode == QMK_FP64 ? Prec::kF64 : (ctx->mode == QMK_MIXED_F32 ? Prec::kF32 : Prec::kBF16P);
}

GemmArgs gbar_args(Prec prec, const void* w, const void* w_lo, int64_t Nw, const void* C, const void* Ct_hi,
                   const void* Ct_lo, void* gbar, int64_t P, int64_t Pp, int64_t K, int64_t Kp,
                   int64_t N, int64_t Np) {
  GemmArgs g{};
  g.L = g.Lchunk = N;
  g.nsplit = 1;
  g.nbatch = 5;
  if (prec == Prec::kBF16P) {
    // rows k, columns p (as below, so that Gbar is stored in full lines);
    // both operands are read along the reduction index n, as this kernel
    // needs
    g.A = Ct_hi;  // C^T [k][n], split into bf16 hi + lo
    g.A2 = Ct_lo;
    g.sAi = Np;
    g.sAl = 1;
    g.B = w;  // W planes [Pp][5][Nw]
    g.B2 = w_lo;
    g.sBl = 1;
    g.sBj = 5 * Nw;
    g.oBc = Nw;
    g.D = gbar;
    g.sDi = 5 * Pp;
    g.sDj = 1;
    g.oDz = Pp;
    g.M = K;
    g.N = P;
    g.map_slab = 2;
    return g;
  }
  // rows k, columns p: consecutive accumulator lanes own consecutive points,
  // so Gbar (point index contiguous) is stored in full lines; the N tiles of
  // W run on one XCD together with every M tile that reads them
  g.A = C;  // C [n][k]
  g.sAi = 1;
  g.sAl = Kp;
  g.pad_ok = 1;  // rows padded to Kp AOs
  g.B = w;  // W [p][c][n], rows of Nw
  g.sBl = 1;
  g.sBj = 5 * Nw;
  g.oBc = Nw;
  g.D = gbar;
  g.sDi = 5 * Pp;
  g.sDj = 1;
  g.oDz = Pp;
  g.M = K;
  g.N = P;
  g.map_slab = 2;
  return g;
}

}  // namespace qmk

// ===========================================================================
namespace qmk {

qmk_status apply_cusp(qmk_ctx ctx, void* out, int o32, hipStream_t s) {
  if (!ctx->cusp_on) return QMK_OK;
  qmk_status st = ensure_cusp(ctx, s);
  if (st != QMK_OK) return st;
  QMK_HIP(ctx, ctx->d_cusp_list.ensure(static_cast<size_t>(2 * ctx->P() + 4) * sizeof(int32_t)),
          "alloc cusp point list");
  int32_t* const cl = ctx->d_cusp_list.as<int32_t>();
  LaunchTimer lt(ctx, QMK_KERNEL_CUSP, s);
  QMK_HIP(ctx, launch_cusp(ctx->cusp, point_args(ctx), out, o32, ctx->mo_num, cl, cl + 4, s), "cusp correction");
  return QMK_OK;
}

// Screened forward product (Section 3.2, sparsity of the AOs): the AO array
// in sorted point order, and a product that visits only the K stages with a
// non-zero AO chunk in its M tile; rows go back to the caller's order.
qmk_status get_mo_vgl_screened(qmk_ctx ctx, void* out, int32_t dtype, hipStream_t s) {
  const int64_t P = ctx->P(), N = ctx->mo_num, K = ctx->ao_num;
  if (round_up(K, kAoPad) / kSparseChunk > kSparseMaxStages)
    return fail(ctx, QMK_UNSUPPORTED, "the screened product supports at most " +
                                          std::to_string(kSparseMaxStages * kSparseChunk) + " AOs");
  qmk_status st = provide_ao_sorted(ctx, s);
  if (st != QMK_OK) return st;
  const int64_t Pp = ctx->aos_Pp;
  GemmArgs ga{};
  ga.A = ctx->aos.p;
  ga.sAi = 1;
  ga.sAl = 5 * Pp;
  ga.oAc = Pp;
  ga.pad_ok = 3;  // AO rows padded to Pp points, C^T rows to Np MOs
  const bool planes = ctx->mode == QMK_MIXED_BF16X3;
  if (planes) {  // sorted AO array as bf16 hi / lo planes, C [n][k] split
    ga.A2 = static_cast<const uint16_t*>(ctx->aos.p) + ctx->aos_Kp * 5 * Pp;
    ga.B = ctx->d_Cb_hi.p;
    ga.B2 = ctx->d_Cb_lo.p;
    ga.sBl = 1;
    ga.sBj = ctx->Kp;
  } else {
    ga.B = ctx->d_Ct.p;
    ga.sBl = ctx->Np;
    ga.sBj = 1;
  }
  ga.D = out;
  ga.sDi = 5 * N;
  ga.sDj = 1;
  ga.oDz = N;
  ga.M = P;
  ga.N = N;
  ga.L = ga.Lchunk = K;
  ga.nsplit = 1;
  ga.nbatch = 5;
  ga.act = ctx->d_act.as<uint32_t>();
  ga.act_words = ctx->act_words;
  ga.perm = ctx->d_perm.as<int32_t>();
  const Prec prec = gemm_prec(ctx);
  const int o32 = dtype == QMK_F32;
  GemmProblem pb{GemmKind::kForward, prec, 0, o32, P, N, K};
  pb.sparse = 1;
  int cfg = 0;
  auto launch = [&](int c) {
    return planes ? launch_gemm_bf16p(GemmKind::kForward, c, ga, o32, 1, s) : launch_gemm_sparse(prec, c, ga, o32, s);
  };
  if ((st = pick_tile(ctx, pb, s, launch, &cfg)) != QMK_OK) return st;
  LaunchTimer lt(ctx, QMK_KERNEL_MO, s);
  QMK_HIP(ctx, launch(cfg), "screened MO contraction");
  return QMK_OK;
}

}  // namespace qmk

extern "C" {

const char* qmk_status_string(qmk_status st) {
  switch (st) {
    case QMK_OK: return "QMK_OK";
    case QMK_INVALID_CONTEXT: return "QMK_INVALID_CONTEXT";
    case QMK_NOT_SET: return "QMK_NOT_SET";
    case QMK_SIZE: return "QMK_SIZE";
    case QMK_OUT_OF_MEMORY: return "QMK_OUT_OF_MEMORY";
    case QMK_HIP_ERROR: return "QMK_HIP_ERROR";
    case QMK_NONFINITE: return "QMK_NONFINITE";
    case QMK_UNSUPPORTED: return "QMK_UNSUPPORTED";
    default: break;
  }
  if (st > QMK_INVALID_ARG_BASE && st < QMK_INVALID_ARG_BASE + 100) return "QMK_INVALID_ARG";
  return "QMK_UNKNOWN_STATUS";
}

const char* qmk_last_error(qmk_ctx ctx) {
  if (ctx == nullptr) return g_create_error.c_str();
  if (!valid_ctx(ctx)) return "invalid context";
  return ctx->err.c_str();
}

qmk_status qmk_ctx_create(qmk_ctx* out, int32_t hip_device) {
  if (out == nullptr) {
    g_create_error = "argument 1: NULL output pointer";
    return QMK_INVALID_ARG_BASE + 1;
  }
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || hip_device < 0 || hip_device >= n) {
    g_create_error = std::string("argument 2: no HIP device ") + std::to_string(hip_device) +
                     (e != hipSuccess ? std::string(" (") + hipGetErrorString(e) + ")" : "");
    return e != hipSuccess ? QMK_HIP_ERROR : QMK_INVALID_ARG_BASE + 2;
  }
  qmk_ctx c = new (std::nothrow) qmk_ctx_s();
  if (!c) {
    g_create_error = "out of host memory";
    return QMK_OUT_OF_MEMORY;
  }
  c->device = hip_device;
  *out = c;
  return QMK_OK;
}

qmk_status qmk_ctx_destroy(qmk_ctx ctx) {
  QMK_CHECK_CTX(ctx);
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->magic = 0;
    delete ctx;
  }
  return QMK_OK;
}

qmk_status qmk_set_precision(qmk_ctx ctx, int32_t bits, int32_t mode) {
  QMK_CHECK_CTX(ctx);
  if (bits < 2 || bits > 53) return bad_arg(ctx, 2, "bits must be in 2..53");
  if (mode != QMK_FP64 && mode != QMK_MIXED_F32 && mode != QMK_MIXED_BF16X3)
    return bad_arg(ctx, 3, "unknown precision mode");
  ctx->bits = bits;
  ctx->mode = mode;
  ++ctx->date;
  ++ctx->geom_version;
  return QMK_OK;
}

qmk_status qmk_set_nucleus(qmk_ctx ctx, int64_t nucl_num, const double* coord) {
  QMK_CHECK_CTX(ctx);
  if (nucl_num < 1 || nucl_num > (1 << 24)) return bad_arg(ctx, 2, "nucl_num must be >= 1");
  if (!coord) return bad_arg(ctx, 3, "NULL coordinates");
  if (ctx->has_basis && nucl_num != ctx->nucl_num)
    return bad_arg(ctx, 2, "number of nuclei changed while a basis is set");
  for (int64_t i = 0; i < 3 * nucl_num; ++i)
    if (!std::isfinite(coord[i])) return fail(ctx, QMK_NONFINITE, "non-finite nuclear coordinate");
  ctx->nucl.assign(coord, coord + 3 * nucl_num);
  ctx->nucl_num = nucl_num;
  ctx->tables_dirty = true;
  ++ctx->date;
  ++ctx->geom_version;
  return QMK_OK;
}

qmk_status qmk_set_basis(qmk_ctx ctx, int64_t shell_num, int64_t prim_num,
                         const int64_t* shell_nucleus, const int32_t* shell_ang_mom,
                         const int64_t* shell_prim_offset, const double* exponent,
                         const double* coefficient, const double* prim_factor,
                         const double* shell_factor, const double* ao_factor) {
  QMK_CHECK_CTX(ctx);
  if (ctx->nucl_num <= 0) return fail(ctx, QMK_NOT_SET, "set the nuclei before the basis");
  if (shell_num < 1 || shell_num > (1 << 24)) return bad_arg(ctx, 2, "shell_num must be >= 1");
  if (prim_num < shell_num || prim_num > (1 << 26))
    return bad_arg(ctx, 3, "prim_num must be >= shell_num");
  if (!shell_nucleus) return bad_arg(ctx, 4, "NULL");
  if (!shell_ang_mom) return bad_arg(ctx, 5, "NULL");
  if (!shell_prim_offset) return bad_arg(ctx, 6, "NULL");
  if (!exponent) return bad_arg(ctx, 7, "NULL");
  if (!coefficient) return bad_arg(ctx, 8, "NULL");
  int64_t ao_num = 0;
  for (int64_t s = 0; s < shell_num; ++s) {
    if (shell_nucleus[s] < 0 || shell_nucleus[s] >= ctx->nucl_num)
      return bad_arg(ctx, 4, "shell " + std::to_string(s) + " refers to a missing nucleus");
    if (shell_ang_mom[s] < 0 || shell_ang_mom[s] > kMaxL)
      return bad_arg(ctx, 5, "angular momentum must be in 0..3");
    ao_num += n_cart(shell_ang_mom[s]);
  }
  if (shell_prim_offset[0] != 0 || shell_prim_offset[shell_num] != prim_num)
    return bad_arg(ctx, 6, "offsets must start at 0 and end at prim_num");
  for (int64_t s = 0; s < shell_num; ++s)
    if (shell_prim_offset[s + 1] <= shell_prim_offset[s])
      return bad_arg(ctx, 6, "every shell needs at least one primitive");
  for (int64_t k = 0; k < prim_num; ++k) {
    if (!std::isfinite(exponent[k]) || !std::isfinite(coefficient[k]))
      return fail(ctx, QMK_NONFINITE, "non-finite exponent or coefficient");
    if (!(exponent[k] > 0.0)) return bad_arg(ctx, 7, "exponents must be > 0");
    if (prim_factor && !std::isfinite(prim_factor[k]))
      return fail(ctx, QMK_NONFINITE, "non-finite primitive factor");
  }
  if (shell_factor)
    for (int64_t s = 0; s < shell_num; ++s)
      if (!std::isfinite(shell_factor[s])) return fail(ctx, QMK_NONFINITE, "non-finite shell factor");
  if (ao_factor)
    for (int64_t k = 0; k < ao_num; ++k)
      if (!std::isfinite(ao_factor[k])) return fail(ctx, QMK_NONFINITE, "non-finite AO factor");

  ctx->sh_nuc.assign(shell_nucleus, shell_nucleus + shell_num);
  ctx->sh_l.assign(shell_ang_mom, shell_ang_mom + shell_num);
  ctx->sh_off.assign(shell_prim_offset, shell_prim_offset + shell_num + 1);
  ctx->expo.assign(exponent, exponent + prim_num);
  ctx->coef.assign(coefficient, coefficient + prim_num);
  ctx->pf.resize(prim_num);
  ctx->sf.resize(shell_num);
  ctx->af.resize(ao_num);
  for (int64_t s = 0; s < shell_num; ++s) {
    const int l = shell_ang_mom[s];
    for (int64_t k = shell_prim_offset[s]; k < shell_prim_offset[s + 1]; ++k)
      ctx->pf[k] = prim_factor ? prim_factor[k] : 1.0 / std::sqrt(axis_norm2(l, 2.0 * exponent[k]));
    if (shell_factor) {
      ctx->sf[s] = shell_factor[s];
    } else {
      double ovl = 0.0;
      for (int64_t k = shell_prim_offset[s]; k < shell_prim_offset[s + 1]; ++k)
        for (int64_t q = shell_prim_offset[s]; q < shell_prim_offset[s + 1]; ++q)
          ovl += coefficient[k] * ctx->pf[k] * coefficient[q] * ctx->pf[q] *
                 axis_norm2(l, exponent[k] + exponent[q]);
      if (!(ovl > 0.0) || !std::isfinite(ovl))
        return bad_arg(ctx, 8, "shell " + std::to_string(s) + " has zero norm");
      ctx->sf[s] = 1.0 / std::sqrt(ovl);
    }
  }
  {
    int64_t k = 0;
    for (int64_t s = 0; s < shell_num; ++s) {
      const int l = shell_ang_mom[s];
      for (int a = l; a >= 0; --a)
        for (int b = l - a; b >= 0; --b, ++k) {
          const int c = l - a - b;
          ctx->af[k] = ao_factor ? ao_factor[k]
                                 : std::sqrt(moment(l, 1.0) * moment(0, 1.0) * moment(0, 1.0) /
                                             (moment(a, 1.0) * moment(b, 1.0) * moment(c, 1.0)));
        }
    }
  }
  ctx->shell_num = shell_num;
  ctx->prim_num = prim_num;
  ctx->ao_num = ao_num;
  ctx->has_basis = true;
  ctx->tables_dirty = true;
  ctx->coef_dirty = true;
  ++ctx->date;
  ++ctx->geom_version;
  return QMK_OK;
}

qmk_status qmk_set_mo_coef(qmk_ctx ctx, int64_t mo_num, int64_t ao_num, const double* coef) {
  QMK_CHECK_CTX(ctx);
  if (!ctx->has_basis) return fail(ctx, QMK_NOT_SET, "set the basis before the MO coefficients");
  if (mo_num < 1 || mo_num > (1 << 24)) return bad_arg(ctx, 2, "mo_num must be >= 1");
  if (ao_num != ctx->ao_num) return bad_arg(ctx, 3, "ao_num does not match the basis");
  if (!coef) return bad_arg(ctx, 4, "NULL");
  for (int64_t i = 0; i < mo_num * ao_num; ++i)
    if (!std::isfinite(coef[i])) return fail(ctx, QMK_NONFINITE, "non-finite MO coefficient");
  ctx->C.assign(coef, coef + mo_num * ao_num);
  ctx->mo_num = mo_num;
  ctx->has_coef = true;
  ctx->coef_dirty = true;
  ++ctx->coef_version;
  return QMK_OK;
}

qmk_status qmk_set_mo_cusp(qmk_ctx ctx, int64_t nucl_num, const double* charge,
                           const double* r_cusp) {
  QMK_CHECK_CTX(ctx);
  if (!r_cusp) {
    ctx->cusp_on = false;
    return QMK_OK;
  }
  if (ctx->nucl_num <= 0) return fail(ctx, QMK_NOT_SET, "set the nuclei before the cusp radii");
  if (nucl_num != ctx->nucl_num) return bad_arg(ctx, 2, "nucl_num does not match the nuclei");
  if (!charge) return bad_arg(ctx, 3, "NULL");
  for (int64_t a = 0; a < nucl_num; ++a) {
    if (!std::isfinite(charge[a]) || charge[a] < 0.0) return bad_arg(ctx, 3, "charges must be finite and >= 0");
    if (!std::isfinite(r_cusp[a]) || r_cusp[a] < 0.0) return bad_arg(ctx, 4, "radii must be finite and >= 0");
  }
  ctx->cusp_charge.assign(charge, charge + nucl_num);
  ctx->cusp_rc.assign(r_cusp, r_cusp + nucl_num);
  ctx->cusp_on = true;
  ++ctx->cusp_version;
  return QMK_OK;
}

qmk_status qmk_det_adj(qmk_ctx ctx, int64_t n, int64_t batch, const double* a, double* det, double* adj,
                       void* hip_stream) {
  QMK_CHECK_CTX(ctx);
  if (n < 1 || n > 32) return bad_arg(ctx, 2, "n must be in 1..32");
  if (batch < 0) return bad_arg(ctx, 3, "batch must be >= 0");
  if (batch == 0) return QMK_OK;  // nothing to do; the buffers may be NULL
  DeviceGuard g(ctx->device);
  qmk_status st;
  if ((st = check_dev_arg(ctx, 4, a)) != QMK_OK || (st = check_dev_arg(ctx, 5, det)) != QMK_OK ||
      (st = check_dev_arg(ctx, 6, adj)) != QMK_OK)
    return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  LaunchTimer lt(ctx, QMK_KERNEL_DET, s);
  QMK_HIP(ctx, launch_det_adj(static_cast<int>(n), batch, a, det, adj, s), "determinant / adjugate");
  return QMK_OK;
}

// Terms of the three-body Jastrow in coefficient order (Section 3.5):
// p = 2..nord, k = 0..p-1, l = 0..p-k-2 delta(k,0), each ascending, keeping
// p-k-l even.  Appends (k, m = (p-k-l)/2, e = (p-k+l)/2) per term to kme.
static int64_t een_term_list(int64_t nord, std::vector<int32_t>* kme) {
  int64_t n = 0;
  for (int64_t p = 2; p <= nord; ++p)
    for (int64_t k = 0; k < p; ++k)
      for (int64_t l = 0; l <= p - k - (k == 0 ? 2 : 0); ++l) {
        if ((p - k - l) % 2 != 0) continue;
        if (kme) kme->insert(kme->end(), {static_cast<int32_t>(k), static_cast<int32_t>((p - k - l) / 2),
                                          static_cast<int32_t>((p - k + l) / 2)});
        ++n;
      }
  return n;
}

qmk_status qmk_jastrow_een_terms(int64_t nord, int64_t* n_terms) {
  if (!n_terms) return QMK_INVALID_ARG_BASE + 2;
  if (nord < 2 || nord > 8) return QMK_INVALID_ARG_BASE + 1;
  *n_terms = een_term_list(nord, nullptr);
  return QMK_OK;
}

qmk_status qmk_jastrow_een(qmk_ctx ctx, int64_t nord, double kappa, int64_t n_terms, const double* c,
                           double* j_een, void* hip_stream) {
  QMK_CHECK_CTX(ctx);
  if (nord < 2 || nord > 8) return bad_arg(ctx, 2, "nord must be in 2..8");
  if (!std::isfinite(kappa) || kappa <= 0.0) return bad_arg(ctx, 3, "kappa must be finite and > 0");
  std::vector<int32_t> kme;
  if (n_terms != een_term_list(nord, &kme)) return bad_arg(ctx, 4, "n_terms does not match nord");
  if (!c) return bad_arg(ctx, 5, "NULL");
  DeviceGuard g(ctx->device);
  qmk_status st = check_dev_arg(ctx, 6, j_een);
  if (st != QMK_OK) return st;
  if (ctx->nucl_num <= 0) return fail(ctx, QMK_NOT_SET, "nuclei not set");
  if (!ctx->has_points) return fail(ctx, QMK_NOT_SET, "points not set");
  const int64_t nn = ctx->nucl_num, nw = ctx->walk_num, ne = ctx->elec_num, P = ctx->P();
  for (int64_t i = 0; i < n_terms * nn; ++i)
    if (!std::isfinite(c[i])) return fail(ctx, QMK_NONFINITE, "non-finite Jastrow coefficient");
  // m >= 1 needs k <= nord-2 and m <= nord/2 (the product's splits and
  // rows); m = 0 needs k >= 1 (handled per electron)
  const int nsplit = static_cast<int>(nord - 1), mh = static_cast<int>(nord / 2), deg = static_cast<int>(nord);
  const size_t nq = static_cast<size_t>(nsplit * mh * nn * kJasCoef);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (ctx->nuc_xyz_version != ctx->geom_version) {
    QMK_HIP(ctx, ctx->d_nuc_xyz.ensure(static_cast<size_t>(3 * nn) * 8), "alloc nuclei");
    QMK_HIP(ctx, hipMemcpy(ctx->d_nuc_xyz.p, ctx->nucl.data(), static_cast<size_t>(3 * nn) * 8,
                           hipMemcpyHostToDevice), "upload nuclei");
    ctx->nuc_xyz_version = ctx->geom_version;
  }
  const int64_t M = mh * nn;
  QMK_HIP(ctx, ctx->een_ra.ensure(static_cast<size_t>(P * M) * 8), "alloc rescaled e-n powers");
  QMK_HIP(ctx, ctx->een_x.ensure(static_cast<size_t>(P * nn) * 8), "alloc rescaled e-n distances");
  QMK_HIP(ctx, ctx->een_rt.ensure(static_cast<size_t>(nw * ne * ne) * 8), "alloc rescaled e-e distances");
  QMK_HIP(ctx, ctx->een_j0.ensure(static_cast<size_t>(P) * 8), "alloc per-electron parts");
  QMK_HIP(ctx, ctx->een_g0.ensure(static_cast<size_t>(P * 7) * 8), "alloc m = 0 weight sums");
  // the polynomial tables are uploaded only when the coefficients change
  // (a blocking copy; the usual caller keeps c fixed over many steps)
  std::vector<double> key(c, c + n_terms * nn);
  key.push_back(static_cast<double>(nord));
  if (key != ctx->een_key) {
    // Terms grouped by (k, m): the coefficient of x^e in the weight of
    // P^{k,m}_{ia} is c[t][a] of the one term with that (k, m, e).
    std::vector<double> q(nq, 0.0);
    std::vector<double> q0(static_cast<size_t>((nord - 1) * nn * (deg + 1)), 0.0);
    for (int64_t t = 0; t < n_terms; ++t) {
      const int k = kme[3 * t], m = kme[3 * t + 1], e = kme[3 * t + 2];
      for (int64_t a = 0; a < nn; ++a) {
        if (m == 0)
          q0[((k - 1) * nn + a) * (deg + 1) + e] = c[t * nn + a];
        else
          q[((static_cast<int64_t>(k) * mh + (m - 1)) * nn + a) * kJasCoef + e] = c[t * nn + a];
      }
    }
    // the previous call's kernels on this stream may still read the tables
    QMK_HIP(ctx, hipStreamSynchronize(s), "wait for the previous Jastrow call");
    QMK_HIP(ctx, ctx->een_q.ensure((q.size() + q0.size()) * 8), "alloc weight polynomials");
    QMK_HIP(ctx, hipMemcpy(ctx->een_q.p, q.data(), q.size() * 8, hipMemcpyHostToDevice), "upload weight polynomials");
    QMK_HIP(ctx, hipMemcpy(ctx->een_q.as<double>() + q.size(), q0.data(), q0.size() * 8, hipMemcpyHostToDevice),
            "upload weight polynomials");
    ctx->een_key = std::move(key);
  }
  double* const d_q = ctx->een_q.as<double>();
  double* const d_q0 = d_q + nq;
  // per-wave partial sums of the product: slots per (walker, k) for a tile
  auto slots_of = [&](int cfg) -> int64_t {
    const TileCfg t = gemm_tile(Prec::kF64, cfg);
    return (M + t.bm() - 1) / t.bm() * t.wgm * ((ne + t.bn() - 1) / t.bn() * t.wgn);
  };
  int64_t slots_max = 1;
  for (int cfg = 0; cfg < gemm_num_tiles(Prec::kF64); ++cfg) slots_max = std::max(slots_max, slots_of(cfg));
  QMK_HIP(ctx, ctx->een_part.ensure(static_cast<size_t>(nw * nsplit * slots_max) * 8), "alloc partial sums");
  {
    LaunchTimer lt(ctx, QMK_KERNEL_JASTROW, s);
    const PointArgs pa = point_args(ctx);
    QMK_HIP(ctx, launch_een_en(pa, ne, ctx->d_nuc_xyz.as<double>(), nn, kappa, mh, ctx->een_ra.as<double>(),
                               ctx->een_x.as<double>(), s),
            "Jastrow e-n distances");
    QMK_HIP(ctx, launch_een_ee(pa, ne, nn, kappa, static_cast<int>(nord), ctx->een_x.as<double>(), d_q0,
                               ctx->een_g0.as<double>(), ctx->een_rt.as<double>(), ctx->een_j0.as<double>(), s),
            "Jastrow e-e distances");
  }
  // part[w, k][slot] = weighted sums over the slot's outputs of
  //   P^{k,m}[(m-1) nn + a][i] = sum_j Ra[w][j][(m-1) nn + a] rt[w][j][i]^k
  //   (rt symmetric; the product takes the power as it stages rt)
  GemmArgs ga{};
  ga.A = ctx->een_ra.p;
  ga.sAi = 1;
  ga.sAl = M;
  ga.oAc = ne * M;
  ga.oAs = 0;
  ga.B = ctx->een_rt.p;
  ga.sBl = ne;
  ga.sBj = 1;
  ga.oBc = ne * ne;
  ga.oBs = 0;
  ga.D = ctx->een_part.p;
  ga.M = M;
  ga.N = ne;
  ga.L = nsplit * ne;  // split s = k runs over j in [0, ne) of rt, to the power k
  ga.Lchunk = ne;
  ga.nsplit = nsplit;
  ga.nbatch = static_cast<int32_t>(nw);
  ga.map_slab = 1;
  ga.jx = ctx->een_x.as<double>();
  ga.jq = d_q;
  ga.j_nn = nn;
  ga.j_mh = mh;
  auto enqueue = [&](int cfg) -> hipError_t {
    GemmArgs gc = ga;
    gc.oDz = slots_of(cfg);
    hipError_t e;
    {
      LaunchTimer lt(ctx, QMK_KERNEL_JASTROW_P, s);
      e = launch_gemm_jastrow(cfg, gc, s);
    }
    if (e != hipSuccess) return e;
    LaunchTimer lt(ctx, QMK_KERNEL_JASTROW, s);
    return launch_een_finish(ctx->een_part.as<double>(), nsplit * gc.oDz, ctx->een_j0.as<double>(), nw, ne,
                             j_een, s);
  };
  // tuning key: the product's size and its batch count (walkers x powers),
  // which decides how many tiles there are to spread over the CUs
  GemmProblem pb{GemmKind::kJastrow, Prec::kF64, 0, 0, M, ne, ne};
  pb.nbatch = static_cast<int>(std::min<int64_t>(nw * nsplit, 0x7fffffff));
  int cfg = 0;
  if ((st = pick_tile(ctx, pb, s, enqueue, &cfg)) != QMK_OK) return st;
  QMK_HIP(ctx, enqueue(cfg), "Jastrow product");
  return QMK_OK;
}

qmk_status qmk_set_ao_retention(qmk_ctx ctx, int32_t retain) {
  QMK_CHECK_CTX(ctx);
  if (retain != 0 && retain != 1) return bad_arg(ctx, 2, "retain must be 0 or 1");
  ctx->ao_retain = retain == 1;
  return QMK_OK;
}

qmk_status qmk_set_screening(qmk_ctx ctx, int32_t enable) {
  QMK_CHECK_CTX(ctx);
  if (enable != 0 && enable != 1) return bad_arg(ctx, 2, "enable must be 0 or 1");
  ctx->sparse = enable == 1;
  return QMK_OK;
}

qmk_status qmk_get_screening_density(qmk_ctx ctx, double* active_fraction) {
  QMK_CHECK_CTX(ctx);
  if (!active_fraction) return bad_arg(ctx, 2, "NULL");
  if (ctx->aos_date < 0 || !ctx->d_act.p) return fail(ctx, QMK_NOT_SET, "no screened AO evaluation yet");
  DeviceGuard g(ctx->device);
  const int64_t blocks = (ctx->P() + 63) / 64, nchunk = ctx->aos_Kp / kSparseChunk;
  std::vector<uint32_t> bits(static_cast<size_t>(blocks * ctx->act_words));
  QMK_HIP(ctx, hipDeviceSynchronize(), "wait for the AO stage");
  QMK_HIP(ctx, hipMemcpy(bits.data(), ctx->d_act.p, bits.size() * 4, hipMemcpyDeviceToHost), "download bitmap");
  int64_t on = 0;
  for (int64_t b = 0; b < blocks; ++b)
    for (int64_t c = 0; c < nchunk; ++c) on += (bits[b * ctx->act_words + (c >> 5)] >> (c & 31)) & 1u;
  *active_fraction = static_cast<double>(on) / static_cast<double>(std::max<int64_t>(1, blocks * nchunk));
  return QMK_OK;
}

qmk_status qmk_set_point(qmk_ctx ctx, char transp, int64_t walk_num, int64_t elec_num,
                         const double* coord, int32_t coord_on_device) {
  QMK_CHECK_CTX(ctx);
  if (transp != 'N' && transp != 'T') return bad_arg(ctx, 2, "transp must be 'N' or 'T'");
  if (walk_num < 1) return bad_arg(ctx, 3, "walk_num must be >= 1");
  if (elec_num < 1) return bad_arg(ctx, 4, "elec_num must be >= 1");
  if (walk_num * elec_num > (int64_t(1) << 31)) return bad_arg(ctx, 3, "too many points");
  if (!coord) return bad_arg(ctx, 5, "NULL");
  if (coord_on_device != 0 && coord_on_device != 1) return bad_arg(ctx, 6, "must be 0 or 1");
  const int64_t n = 3 * walk_num * elec_num;
  if (coord_on_device) {
    DeviceGuard g(ctx->device);
    qmk_status st = check_dev_arg(ctx, 5, coord);
    if (st != QMK_OK) return st;
    ctx->pts = coord;
  } else {
    for (int64_t i = 0; i < n; ++i)
      if (!std::isfinite(coord[i])) return fail(ctx, QMK_NONFINITE, "non-finite coordinate");
    DeviceGuard g(ctx->device);
    QMK_HIP(ctx, ctx->own_pts.ensure(static_cast<size_t>(n) * sizeof(double)), "alloc points");
    QMK_HIP(ctx, hipMemcpy(ctx->own_pts.p, coord, n * sizeof(double), hipMemcpyHostToDevice),
            "upload points");
    ctx->pts = ctx->own_pts.as<double>();
  }
  ctx->transp = transp;
  ctx->walk_num = walk_num;
  ctx->elec_num = elec_num;
  ctx->has_points = true;
  ++ctx->date;
  return QMK_OK;
}

qmk_status qmk_get_dims(qmk_ctx ctx, int64_t* nucl_num, int64_t* ao_num, int64_t* mo_num,
                        int64_t* walk_num, int64_t* elec_num) {
  QMK_CHECK_CTX(ctx);
  if (nucl_num) *nucl_num = ctx->nucl_num;
  if (ao_num) *ao_num = ctx->ao_num;
  if (mo_num) *mo_num = ctx->mo_num;
  if (walk_num) *walk_num = ctx->walk_num;
  if (elec_num) *elec_num = ctx->elec_num;
  return QMK_OK;
}

qmk_status qmk_get_launch_count(qmk_ctx ctx, int64_t* count) {
  QMK_CHECK_CTX(ctx);
  if (!count) return bad_arg(ctx, 2, "NULL");
  *count = ctx->launches;
  return QMK_OK;
}

qmk_status qmk_set_tile(qmk_ctx ctx, int32_t kernel_class, int32_t tile) {
  QMK_CHECK_CTX(ctx);
  int kind = -1;
  if (kernel_class == QMK_KERNEL_MO) kind = static_cast<int>(GemmKind::kForward);
  if (kernel_class == QMK_KERNEL_GBAR) kind = static_cast<int>(GemmKind::kGbar);
  if (kernel_class == QMK_KERNEL_DCOEF) kind = static_cast<int>(GemmKind::kDcoef);
  if (kernel_class == QMK_KERNEL_DENSITY) kind = static_cast<int>(GemmKind::kDensity);
  if (kernel_class == QMK_KERNEL_JASTROW_P) kind = static_cast<int>(GemmKind::kJastrow);
  if (kind < 0) return bad_arg(ctx, 2, "kernel class has no tile choice");
  const Prec prec = product_prec(ctx, static_cast<GemmKind>(kind));
  if (tile < -1 || tile >= gemm_num_tiles(prec)) return bad_arg(ctx, 3, "unknown tile for this product's precision");
  if (tile >= 0 && !tile_feasible(prec, tile)) return bad_arg(ctx, 3, "tile does not fit in LDS");
  ctx->forced_tile[kind] = tile;
  return QMK_OK;
}

qmk_status qmk_get_tile_count(qmk_ctx ctx, int32_t* count) {
  QMK_CHECK_CTX(ctx);
  if (!count) return bad_arg(ctx, 2, "NULL");
  *count = gemm_num_tiles(gemm_prec(ctx));
  return QMK_OK;
}

qmk_status qmk_set_timing(qmk_ctx ctx, int32_t enable) {
  QMK_CHECK_CTX(ctx);
  if (enable != 0 && enable != 1) return bad_arg(ctx, 2, "must be 0 or 1");
  DeviceGuard g(ctx->device);
  collect_timing(ctx);
  if (enable) {
    for (int k = 0; k < QMK_KERNEL_CLASSES; ++k) {
      ctx->t_ms[k] = 0.0;
      ctx->t_n[k] = 0;
    }
  }
  ctx->timing = enable != 0;
  return QMK_OK;
}

qmk_status qmk_get_timing(qmk_ctx ctx, int32_t kernel_class, double* total_ms, int64_t* launches) {
  QMK_CHECK_CTX(ctx);
  if (kernel_class < 0 || kernel_class >= QMK_KERNEL_CLASSES) return bad_arg(ctx, 2, "unknown kernel class");
  DeviceGuard g(ctx->device);
  collect_timing(ctx);
  if (total_ms) *total_ms = ctx->t_ms[kernel_class];
  if (launches) *launches = ctx->t_n[kernel_class];
  return QMK_OK;
}

qmk_status qmk_get_ao_vgl(qmk_ctx ctx, void* out, int64_t size_max, int32_t dtype,
                          void* hip_stream) {
  QMK_CHECK_CTX(ctx);
  {
    DeviceGuard dg(ctx->device);
    const qmk_status pst = check_dev_arg(ctx, 2, out);
    if (pst != QMK_OK) return pst;
  }
  if (dtype != QMK_F64 && dtype != QMK_F32) return bad_arg(ctx, 4, "dtype must be QMK_F64 or QMK_F32");
  qmk_status st = check_ready(ctx, false);
  if (st != QMK_OK) return st;
  const int64_t need = ctx->P() * 5 * ctx->ao_num;
  if (size_max < need)
    return fail(ctx, QMK_SIZE, "size_max " + std::to_string(size_max) + " < " + std::to_string(need));
  DeviceGuard g(ctx->device);
  st = ensure_tables(ctx);
  if (st != QMK_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  AoOut o{out, 1, ctx->ao_num, 5 * ctx->ao_num};
  LaunchTimer lt(ctx, QMK_KERNEL_AO, s);
  QMK_HIP(ctx, launch_ao_vgl(ctx->tab, point_args(ctx), o, dtype == QMK_F32, ctx->f32_storage(), s),
          "AO kernel");
  return QMK_OK;
}

qmk_status qmk_get_mo_vgl(qmk_ctx ctx, void* out, int64_t size_max, int32_t dtype,
                          void* hip_stream) {
  QMK_CHECK_CTX(ctx);
  {
    DeviceGuard dg(ctx->device);
    const qmk_status pst = check_dev_arg(ctx, 2, out);
    if (pst != QMK_OK) return pst;
  }
  if (dtype != QMK_F64 && dtype != QMK_F32) return bad_arg(ctx, 4, "dtype must be QMK_F64 or QMK_F32");
  qmk_status st = check_ready(ctx, true);
  if (st != QMK_OK) return st;
  const int64_t P = ctx->P(), N = ctx->mo_num, K = ctx->ao_num;
  if (size_max < P * 5 * N)
    return fail(ctx, QMK_SIZE, "size_max " + std::to_string(size_max) + " < " + std::to_string(P * 5 * N));
  DeviceGuard g(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((st = ensure_coef(ctx)) != QMK_OK) return st;
  if (ctx->sparse) {
    if ((st = get_mo_vgl_screened(ctx, out, dtype, s)) != QMK_OK) return st;
    return apply_cusp(ctx, out, dtype == QMK_F32, s);
  }
  if ((st = provide_ao(ctx, s)) != QMK_OK) return st;
  const int64_t Pp = ctx->ao_Pp;
  GemmArgs ga{};
  ga.A = ctx->ao.p;
  ga.sAi = 1;
  ga.sAl = 5 * Pp;
  ga.oAc = Pp;
  ga.pad_ok = 3;  // AO rows padded to Pp points, C^T rows to Np MOs
  if (ctx->mode == QMK_MIXED_BF16X3) {
    // AO array as bf16 hi / lo planes, C [n][k] split (reduction index contiguous)
    ga.A2 = static_cast<const uint16_t*>(ctx->ao.p) + ctx->ao_Kp * 5 * Pp;
    ga.B = ctx->d_Cb_hi.p;
    ga.B2 = ctx->d_Cb_lo.p;
    ga.sBl = 1;
    ga.sBj = ctx->Kp;
  } else {
    ga.B = ctx->d_Ct.p;
    ga.sBl = ctx->Np;
    ga.sBj = 1;
  }
  ga.D = out;
  ga.sDi = 5 * N;
  ga.sDj = 1;
  ga.oDz = N;
  ga.M = P;
  ga.N = N;
  ga.L = K;
  ga.Lchunk = K;
  ga.nsplit = 1;
  ga.nbatch = 5;
  const Prec prec = gemm_prec(ctx);
  const int o32 = dtype == QMK_F32;
  const GemmProblem pb{GemmKind::kForward, prec, 0, o32, P, N, K};
  int cfg = 0;
  if ((st = pick_tile(ctx, pb, s, [&](int c) {
         return launch_gemm_typed(GemmKind::kForward, prec, c, ga, 0, o32, s);
       }, &cfg)) != QMK_OK)
    return st;
  {
    LaunchTimer lt(ctx, QMK_KERNEL_MO, s);
    QMK_HIP(ctx, launch_gemm_typed(GemmKind::kForward, prec, cfg, ga, 0, o32, s), "MO contraction");
  }
  return apply_cusp(ctx, out, o32, s);
}

qmk_status qmk_get_mo_value(qmk_ctx ctx, void* out, int64_t size_max, int32_t dtype,
                            void* hip_stream) {
  QMK_CHECK_CTX(ctx);
  {
    DeviceGuard dg(ctx->device);
    const qmk_status pst = check_dev_arg(ctx, 2, out);
    if (pst != QMK_OK) return pst;
  }
  if (dtype != QMK_F64 && dtype != QMK_F32) return bad_arg(ctx, 4, "dtype must be QMK_F64 or QMK_F32");
  qmk_status st = check_ready(ctx, true);
  if (st != QMK_OK) return st;
  if (ctx->cusp_on) return fail(ctx, QMK_UNSUPPORTED, "MO values alone with the cusp correction on is not implemented");
  const int64_t P = ctx->P(), N = ctx->mo_num, K = ctx->ao_num;
  if (size_max < P * N)
    return fail(ctx, QMK_SIZE, "size_max " + std::to_string(size_max) + " < " + std::to_string(P * N));
  DeviceGuard g(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const Prec prec = ctx->mode == QMK_FP64 ? Prec::kF64 : Prec::kF32;
  if ((st = ensure_coef(ctx)) != QMK_OK) return st;
  const void* plane = nullptr;
  int64_t row = 0;
  if ((st = provide_ao_value(ctx, s, &plane, &row)) != QMK_OK) return st;
  GemmArgs ga{};
  ga.A = plane;
  ga.sAi = 1;
  ga.sAl = row;
  ga.pad_ok = 3;  // value rows padded to whole point blocks, C^T rows to Np MOs
  ga.B = ctx->d_Ct.p;
  ga.sBl = ctx->Np;
  ga.sBj = 1;
  ga.D = out;
  ga.sDi = N;
  ga.sDj = 1;
  ga.M = P;
  ga.N = N;
  ga.L = ga.Lchunk = K;
  ga.nsplit = 1;
  ga.nbatch = 1;
  const int o32 = dtype == QMK_F32;
  GemmProblem pb{GemmKind::kForward, prec, 0, o32, P, N, K};
  pb.nbatch = 1;
  int cfg = 0;
  if ((st = pick_tile(ctx, pb, s, [&](int c) {
         return launch_gemm_typed(GemmKind::kForward, prec, c, ga, 0, o32, s);
       }, &cfg)) != QMK_OK)
    return st;
  LaunchTimer lt(ctx, QMK_KERNEL_MO, s);
  QMK_HIP(ctx, launch_gemm_typed(GemmKind::kForward, prec, cfg, ga, 0, o32, s), "MO value product");
  return QMK_OK;
}

qmk_status qmk_get_density(qmk_ctx ctx, const double* occ, int64_t occ_num, double* rho,
                           int64_t size_max, void* hip_stream) {
  QMK_CHECK_CTX(ctx);
  if (!occ) return bad_arg(ctx, 2, "NULL");
  {
    DeviceGuard dg(ctx->device);
    const qmk_status pst = check_dev_arg(ctx, 4, rho);
    if (pst != QMK_OK) return pst;
  }
  qmk_status st = check_ready(ctx, true);
  if (st != QMK_OK) return st;
  if (ctx->cusp_on) return fail(ctx, QMK_UNSUPPORTED, "the density with the cusp correction on is not implemented");
  const int64_t P = ctx->P(), N = ctx->mo_num, K = ctx->ao_num;
  if (occ_num != N) return bad_arg(ctx, 3, "occ_num must equal mo_num");
  for (int64_t n = 0; n < N; ++n)
    if (!std::isfinite(occ[n])) return fail(ctx, QMK_NONFINITE, "non-finite occupation number");
  if (size_max < P)
    return fail(ctx, QMK_SIZE, "size_max " + std::to_string(size_max) + " < " + std::to_string(P));
  DeviceGuard g(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const Prec prec = ctx->mode == QMK_FP64 ? Prec::kF64 : Prec::kF32;
  const int f32 = prec == Prec::kF32 ? 1 : 0;

  // occupied MOs, compacted once per (occupations, coefficients, precision)
  std::vector<double> key(occ, occ + N);
  if (key != ctx->occ_key || ctx->occ_coef_version != ctx->coef_version || ctx->occ_f32 != f32) {
    std::vector<int64_t> rows;
    for (int64_t n = 0; n < N; ++n)
      if (occ[n] != 0.0) rows.push_back(n);
    const int64_t no = static_cast<int64_t>(rows.size());
    const int64_t Kp = round_up(K, kAoPad), Nop = std::max<int64_t>(round_up(no, kMoPad), kMoPad);
    std::vector<double> w(Nop, 0.0);
    std::vector<double> ct64;
    std::vector<float> ct32;
    if (f32) ct32.assign(static_cast<size_t>(Kp * Nop), 0.0f);
    else ct64.assign(static_cast<size_t>(Kp * Nop), 0.0);
    for (int64_t j = 0; j < no; ++j) {
      w[j] = occ[rows[j]];
      for (int64_t k = 0; k < K; ++k) {
        const double c = ctx->C[rows[j] * K + k];
        if (f32) ct32[k * Nop + j] = static_cast<float>(c);
        else ct64[k * Nop + j] = c;
      }
    }
    const size_t cb = static_cast<size_t>(Kp * Nop) * (f32 ? 4 : 8);
    QMK_HIP(ctx, ctx->d_Cocc_t.ensure(cb), "alloc occupied coefficients");
    QMK_HIP(ctx, hipMemcpy(ctx->d_Cocc_t.p, f32 ? static_cast<const void*>(ct32.data())
                                                 : static_cast<const void*>(ct64.data()),
                           cb, hipMemcpyHostToDevice),
            "upload occupied coefficients");
    QMK_HIP(ctx, ctx->d_occ.ensure(static_cast<size_t>(Nop) * 8), "alloc occupations");
    QMK_HIP(ctx, hipMemcpy(ctx->d_occ.p, w.data(), static_cast<size_t>(Nop) * 8, hipMemcpyHostToDevice),
            "upload occupations");
    ctx->occ_key = key;
    ctx->occ_coef_version = ctx->coef_version;
    ctx->occ_f32 = f32;
    ctx->n_occ = no;
    ctx->Nop = Nop;
  }
  if (ctx->n_occ == 0) {
    QMK_HIP(ctx, hipMemsetAsync(rho, 0, static_cast<size_t>(P) * 8, s), "clear density");
    return QMK_OK;
  }
  const void* plane = nullptr;
  int64_t row = 0;
  if ((st = provide_ao_value(ctx, s, &plane, &row)) != QMK_OK) return st;
  const int64_t Pp = round_up(P, kPointPad);
  // one partial row per (N tile, wave) of the widest tile on offer
  int64_t slots_max = 0;
  for (int c = 0; c < gemm_num_tiles(prec); ++c) {
    const TileCfg t = gemm_tile(prec, c);
    slots_max = std::max<int64_t>(slots_max, (ctx->n_occ + t.bn() - 1) / t.bn() * t.wgn);
  }
  QMK_HIP(ctx, ctx->ws_den.ensure(static_cast<size_t>(slots_max * Pp) * 8), "alloc density partials");
  GemmArgs ga{};
  ga.A = plane;
  ga.sAi = 1;
  ga.sAl = row;
  ga.pad_ok = 3;  // value rows padded to whole point blocks, occupied C^T rows to Nop MOs
  ga.B = ctx->d_Cocc_t.p;
  ga.sBl = ctx->Nop;
  ga.sBj = 1;
  ga.D = ctx->ws_den.p;
  ga.sDi = 1;
  ga.sDj = Pp;
  ga.M = P;
  ga.N = ctx->n_occ;
  ga.L = ga.Lchunk = K;
  ga.nsplit = 1;
  ga.nbatch = 1;
  ga.occ = ctx->d_occ.as<double>();
  auto enqueue = [&](int c) -> hipError_t {
    hipError_t e;
    {
      LaunchTimer lt(ctx, QMK_KERNEL_DENSITY, s);
      e = launch_gemm_density(prec, c, ga, s);
    }
    if (e != hipSuccess) return e;
    const TileCfg t = gemm_tile(prec, c);
    const int64_t slots = (ctx->n_occ + t.bn() - 1) / t.bn() * t.wgn;
    LaunchTimer lt(ctx, QMK_KERNEL_REDUCE, s);
    return launch_reduce_splits(ctx->ws_den.as<double>(), slots, 1, P, 0, Pp, rho, 0, s);
  };
  GemmProblem pb{GemmKind::kDensity, prec, 0, 0, P, ctx->n_occ, K};
  pb.nbatch = 1;
  int cfg = 0;
  if ((st = pick_tile(ctx, pb, s, enqueue, &cfg)) != QMK_OK) return st;
  QMK_HIP(ctx, enqueue(cfg), "density product");
  return QMK_OK;
}

qmk_status qmk_mo_vgl_adjoint(qmk_ctx ctx, const void* w, int32_t w_dtype, double* d_coef,
                              double* d_elec, double* d_nucl, void* hip_stream) {
  QMK_CHECK_CTX(ctx);
  {
    DeviceGuard dg(ctx->device);
    qmk_status pst = check_dev_arg(ctx, 2, w);
    if (pst == QMK_OK && d_coef) pst = check_dev_arg(ctx, 4, d_coef);
    if (pst == QMK_OK && d_elec) pst = check_dev_arg(ctx, 5, d_elec);
    if (pst == QMK_OK && d_nucl) pst = check_dev_arg(ctx, 6, d_nucl);
    if (pst != QMK_OK) return pst;
  }
  if (w_dtype != QMK_F64 && w_dtype != QMK_F32) return bad_arg(ctx, 3, "dtype must be QMK_F64 or QMK_F32");
  qmk_status st = check_ready(ctx, true);
  if (st != QMK_OK) return st;
  if (ctx->cusp_on) return fail(ctx, QMK_UNSUPPORTED, "the adjoint with the cusp correction on is not implemented");
  DeviceGuard g(ctx->device);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if ((st = ensure_coef(ctx)) != QMK_OK) return st;
  // screened adjoint: every product in sorted point order (Section 3.2)
  const bool scr = ctx->sparse;
  // dC reads the AO values: by default the forward pass's array of the same
  // points (memoised, as the provide scheme keeps any value whose inputs are
  // unchanged); with retention off they are evaluated again here
  const bool again = !ctx->ao_retain;
  if ((st = scr ? provide_ao_sorted(ctx, s, again) : provide_ao(ctx, s, again)) != QMK_OK) return st;
  const int64_t P = ctx->P(), N = ctx->mo_num, K = ctx->ao_num;
  const int64_t Pp = scr ? ctx->aos_Pp : ctx->ao_Pp, Kp = ctx->Kp, Np = ctx->Np;
  const void* ao_arr = scr ? ctx->aos.p : ctx->ao.p;
  auto screen = [&](GemmArgs& ga) {
    ga.act = ctx->d_act.as<uint32_t>();
    ga.act_words = ctx->act_words;
  };
  int w32 = w_dtype == QMK_F32;
  const int f32 = ctx->f32_storage() ? 1 : 0;
  const Prec prec = gemm_prec(ctx);
  // row length of W as the products read it ([p][c][ldw]); the copies below
  // pad their rows with zeros
  int64_t ldw = N;
  int w_pad = 0;
  if (!w32 && ctx->mode == QMK_MIXED_F32) {
    // the FP32 products round W to FP32 as they load it; one streaming pass
    // does the same rounding and halves the bytes both products read
    ldw = round_up(N, 4);
    w_pad = 1;
    QMK_HIP(ctx, ctx->w_f32.ensure(static_cast<size_t>(P * 5 * ldw) * 4), "alloc FP32 W");
    LaunchTimer lt(ctx, QMK_KERNEL_CONVERT, s);
    QMK_HIP(ctx, launch_pad_rows(w, 0, ctx->w_f32.p, 1, P * 5, N, ldw, s), "convert W");
    w = ctx->w_f32.p;
    w32 = 1;
  } else if ((ctx->mode == QMK_FP64 && !w32) || (ctx->mode == QMK_MIXED_F32 && w32)) {
    // the products load W in 16-byte pieces when its rows start 16-byte
    // aligned; other row lengths (or a misaligned W) get a padded copy
    const int64_t e = w32 ? 4 : 2;
    if ((5 * N) % e != 0 || reinterpret_cast<uintptr_t>(w) % 16 != 0) {
      ldw = round_up(N, 4);
      w_pad = 1;
      QMK_HIP(ctx, ctx->w_f32.ensure(static_cast<size_t>(P * 5 * ldw) * (w32 ? 4 : 8)), "alloc padded W");
      LaunchTimer lt(ctx, QMK_KERNEL_CONVERT, s);
      QMK_HIP(ctx, launch_pad_rows(w, w32, ctx->w_f32.p, w32, P * 5, N, ldw, s), "pad W");
      w = ctx->w_f32.p;
    }
  }
  // BF16x3 mode: W split once into bf16 hi / lo planes [Pp][5][Nw], read by
  // both products (the W C product along n, the W^T ao product along p)
  const bool planes = prec == Prec::kBF16P;
  const int64_t Nw = round_up(N, 32);
  const uint16_t *w_hi = nullptr, *w_lo = nullptr;
  if (planes) {
    const size_t plane = static_cast<size_t>(Pp) * 5 * static_cast<size_t>(Nw);
    QMK_HIP(ctx, ctx->w_split.ensure(plane * 4), "alloc split W");
    w_hi = ctx->w_split.as<uint16_t>();
    w_lo = w_hi + plane;
    LaunchTimer lt(ctx, QMK_KERNEL_CONVERT, s);
    // screened: the planes hold W in the sorted point order
    QMK_HIP(ctx, launch_split_w(w, w32, P, N, Pp, Nw, scr ? ctx->d_perm.as<int32_t>() : nullptr,
                                const_cast<uint16_t*>(w_hi), const_cast<uint16_t*>(w_lo), s),
            "split W");
  }
  if (scr && !planes) {
    // W in the sorted point order, once, so that both products read it with
    // their ordinary loaders
    const int64_t row_bytes = 5 * ldw * (w32 ? 4 : 8);
    QMK_HIP(ctx, ctx->w_sorted.ensure(static_cast<size_t>(P * row_bytes)), "alloc sorted W");
    LaunchTimer lt(ctx, QMK_KERNEL_SORT, s);
    QMK_HIP(ctx, launch_gather_rows(w, ctx->d_perm.as<int32_t>(), P, row_bytes, ctx->w_sorted.p, s),
            "sort W");
    w = ctx->w_sorted.p;
  }

  if (d_elec || d_nucl) {
    // Gbar[k][c][p] = sum_n W[p][c][n] C[n][k]
    if (ctx->gbar_Pp != Pp || ctx->gbar_Kp != Kp || ctx->gbar_f32 != f32 || !ctx->gbar.p) {
      ctx->gbar.release();
      QMK_HIP(ctx, ctx->gbar.ensure(static_cast<size_t>(Kp * 5 * Pp) * (f32 ? 4 : 8)), "alloc Gbar");
      ctx->gbar_Pp = Pp;
      ctx->gbar_Kp = Kp;
      ctx->gbar_f32 = f32;
    }
    GemmArgs ga = gbar_args(prec, planes ? static_cast<const void*>(w_hi) : w, w_lo, planes ? Nw : ldw, ctx->d_C.p,
                            ctx->d_Ctb_hi.p, ctx->d_Ctb_lo.p, ctx->gbar.p, P, Pp, K, Kp, N, Np);
    if (scr) screen(ga);
    GemmProblem pb{GemmKind::kGbar, prec, w32, f32, ga.M, ga.N, N};
    pb.sparse = scr ? 1 : 0;
    auto launch = [&](int c) {
      if (planes) return launch_gemm_bf16p(GemmKind::kGbar, c, ga, f32, scr ? 1 : 0, s);
      return scr ? launch_gemm_screened_adj(GemmKind::kGbar, prec, c, ga, w32, s)
                 : launch_gemm_typed(GemmKind::kGbar, prec, c, ga, w32, f32, s);
    };
    int cfg = 0;
    if ((st = pick_tile(ctx, pb, s, launch, &cfg)) != QMK_OK) return st;
    {
      LaunchTimer lt(ctx, QMK_KERNEL_GBAR, s);
      QMK_HIP(ctx, launch(cfg), "Gbar product");
    }

    const int64_t n_waves = (P + 255) / 256 * 4;
    QMK_HIP(ctx, ctx->ws_nuc.ensure(static_cast<size_t>(n_waves * ctx->nucl_dev * 3) * 8), "alloc nuc partials");
    double* elec_out = d_elec;
    int64_t gstride = 0;
    if (ctx->n_groups > 1 || !d_elec) {
      QMK_HIP(ctx, ctx->ws_elec.ensure(static_cast<size_t>(ctx->n_groups * P * 3) * 8), "alloc elec partials");
      elec_out = ctx->ws_elec.as<double>();
      gstride = P * 3;
    }
    int64_t nw = 0;
    {
      LaunchTimer lt(ctx, QMK_KERNEL_AO_ADJOINT, s);
      PointArgs pa = point_args(ctx);
      if (scr) pa.perm = ctx->d_perm.as<int32_t>();
      QMK_HIP(ctx, launch_ao_adjoint(ctx->tab, pa, ctx->gbar.p, f32, 5 * Pp, Pp, elec_out,
                                     gstride, ctx->ws_nuc.as<double>(), &nw, s),
              "AO adjoint kernel");
    }
    if (d_elec && elec_out != d_elec) {
      LaunchTimer lt(ctx, QMK_KERNEL_REDUCE, s);
      QMK_HIP(ctx, launch_reduce_splits(elec_out, ctx->n_groups, P, 3, 3, P * 3, d_elec, 3, s),
              "reduce electron gradient");
    }
    if (d_nucl) {
      LaunchTimer lt(ctx, QMK_KERNEL_REDUCE, s);
      QMK_HIP(ctx, launch_reduce_nuc(ctx->ws_nuc.as<double>(), nw, ctx->nucl_dev,
                                     ctx->d_devof.as<int32_t>(), static_cast<int32_t>(ctx->nucl_num),
                                     d_nucl, s),
              "reduce nuclear gradient");
    }
  }
  if (d_coef) {
    // dC[n][k] = sum_{c, p} W[p][c][n] ao[k][c][p], split over (c, point chunk).
    // Every workgroup of this grid does the same work, so the number of point
    // chunks is chosen for a whole number of rounds of resident workgroups:
    // the largest count that fills at most four rounds (a fifth, nearly
    // empty round would cost up to a fifth of the launch).
    int ncu = 0;
    QMK_HIP(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device),
            "query CU count");
    auto split_of = [&](int cfg, int64_t* chunk_out) {
      const TileCfg t = gemm_tile(prec, cfg);
      const int64_t tiles = ((N + t.bm() - 1) / t.bm()) * ((K + t.bn() - 1) / t.bn());
      const int64_t resident = static_cast<int64_t>(std::max(1, ncu)) *
                               gemm_persist_blocks_per_cu(GemmKind::kDcoef, prec, cfg, w32, 0);
      int64_t ns = std::max<int64_t>(1, 4 * resident / (tiles * 5));
      ns = std::min<int64_t>(ns, std::max<int64_t>(1, (P + 255) / 256));
      int64_t chunk = round_up((P + ns - 1) / ns, 32);
      if (planes && scr) {
        // screened BF16x3: whole 64-point blocks per split, at most
        // kSparseMaxStages K steps of 32 points each
        chunk = std::min<int64_t>(round_up(chunk, 64), static_cast<int64_t>(kSparseMaxStages) * 32);
      }
      *chunk_out = chunk;
      return (P + chunk - 1) / chunk;
    };
    int64_t nz_max = 0;
    for (int c = 0; c < gemm_num_tiles(prec); ++c) {
      int64_t ch = 0;
      if (tile_feasible(prec, c)) nz_max = std::max(nz_max, 5 * split_of(c, &ch));
    }
    QMK_HIP(ctx, ctx->ws_dc.ensure(static_cast<size_t>(nz_max * Np * Kp) * 8), "alloc dC partials");
    auto enqueue = [&](int cfg) -> hipError_t {
      int64_t chunk = 0;
      const int64_t nsplit = split_of(cfg, &chunk);
      GemmArgs ga{};
      ga.A = w;
      ga.sAi = 1;
      ga.sAl = 5 * ldw;
      ga.oAc = ldw;
      ga.oAs = chunk * 5 * ldw;
      ga.pad_ok = w_pad;  // the FP32 copy of W has rows padded to ldw MOs
      ga.B = ao_arr;
      ga.sBl = 1;
      ga.sBj = 5 * Pp;
      ga.oBc = Pp;
      ga.oBs = chunk;
      if (planes) {  // W and the AO array as bf16 hi / lo planes
        ga.A = w_hi;
        ga.A2 = w_lo;
        ga.sAl = 5 * Nw;
        ga.oAc = Nw;
        ga.oAs = chunk * 5 * Nw;
        ga.B2 = static_cast<const uint16_t*>(ao_arr) + Kp * 5 * Pp;
      }
      ga.D = ctx->ws_dc.p;
      ga.sDi = Kp;
      ga.sDj = 1;
      ga.oDz = Np * Kp;
      ga.M = N;
      ga.N = K;
      ga.L = P;
      ga.Lchunk = chunk;
      ga.nsplit = static_cast<int32_t>(nsplit);
      ga.nbatch = 5;
      ga.map_slab = 1;
      if (scr) screen(ga);
      hipError_t e;
      {
        LaunchTimer lt(ctx, QMK_KERNEL_DCOEF, s);
        e = planes ? launch_gemm_bf16p(GemmKind::kDcoef, cfg, ga, 0, scr ? 1 : 0, s)
            : scr  ? launch_gemm_screened_adj(GemmKind::kDcoef, prec, cfg, ga, w32, s)
                : launch_gemm_typed(GemmKind::kDcoef, prec, cfg, ga, w32, 0, s);
      }
      if (e != hipSuccess) return e;
      LaunchTimer lt(ctx, QMK_KERNEL_REDUCE, s);
      return launch_reduce_splits(ctx->ws_dc.as<double>(), 5 * nsplit, N, K, Kp, Np * Kp, d_coef, K, s);
    };
    GemmProblem pb{GemmKind::kDcoef, prec, w32, 0, N, K, P};
    pb.sparse = scr ? 1 : 0;
    int cfg = 0;
    if ((st = pick_tile(ctx, pb, s, enqueue, &cfg)) != QMK_OK) return st;
    QMK_HIP(ctx, enqueue(cfg), "dC product");
  }
  return QMK_OK;
}

}  // extern "C"
