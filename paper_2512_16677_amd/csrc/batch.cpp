// Batch executor: many independent contexts (molecules of uneven sizes, each
// with its own walkers) evaluated together.  The QMCkl paper runs several
// independent contexts side by side (Section 2.2) and parallelises over
// them with threads (Section 2.4); on one GPU the same independence becomes
// one launch per stage for the whole batch:
//   * every stage (AO values, the AO -> MO product and, with weights, the W C
//     product, the AO adjoint, the split W^T ao product and the reductions)
//     is a persistent kernel whose grid is sized to the GPU and walks a work
//     list of (molecule, tile) items, longest first;
//   * the stage sequence is captured once into a HIP graph and replayed with
//     a single hipGraphLaunch per run;
//   * the MFMA tile shape of each product is chosen for the batch as a whole
//     by timing every tile shape on the first run (cached like the
//     per-context choices);
//   * in the BF16x3 mode the AO stage writes bf16 hi / lo planes and one
//     element-wise launch splits every molecule's W into planes, so that
//     the three products run the pre-split MFMA kernel, as per context.
// Per-molecule arguments live in device job tables that are rewritten before
// every launch, so new coordinates (set_point) or new output buffers need no
// re-capture; a change of any dimension re-plans and re-captures.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "ctx_internal.h"

using namespace qmk;

namespace {

constexpr uint32_t kBatchMagic = 0x514d4b42u;  // "QMKB"
constexpr int64_t kDcoefChunk = 4096;          // points per split of the W^T ao product

struct MolPlan {
  int64_t P, K, N, Pp, Kp, Np, Nw, nucl_num;
  int32_t n_groups, nucl_dev;
  size_t ao_off, gbar_off;  // elements of the AO / Gbar arenas
  size_t dc_off;            // doubles of the dC partial arena
  size_t w_off;             // bf16 elements of the split-W arena (hi plane, then lo)
  // FP64 / FP32 modes: whether the products read a copy of W with rows padded
  // to ldw weights (the caller's rows of N do not allow 16-byte loads), and
  // its offset (elements of the padded-W arena)
  bool pad_w;
  int64_t ldw;
  size_t wp_off;
  int64_t nsplit, chunk;
  size_t nuc_off;           // doubles of the nucleus partial arena
  int64_t n_waves;
  size_t elec_off;          // doubles of the electron partial arena
  size_t scratch_coef, scratch_elec, scratch_nucl;  // doubles of the discard arena
};

template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v, hipStream_t s) {
  hipError_t e = b.ensure(std::max<size_t>(v.size() * sizeof(T), 16));
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

}  // namespace

struct qmk_batch_s {
  uint32_t magic = kBatchMagic;
  int device = 0;
  std::string err;
  std::vector<qmk_ctx> ctxs;
  int mode = QMK_FP64;
  Prec prec = Prec::kF64;
  int esz = 8;     // bytes per AO / Gbar element (bf16 planes: hi + lo)
  int ao_fmt = 0;  // AO stage output: 0 FP64, 1 FP32, 2 bf16 hi / lo planes

  std::vector<int64_t> dims_key;
  std::vector<MolPlan> plan;
  bool planned = false;
  DevBuf ao, gbar, ws_dc, ws_nuc, ws_elec, discard, wsplit, wpad;
  size_t max_smem = 0;
  int n_cu = 0;

  // work lists (fixed per plan) and job tables (rewritten every run)
  std::vector<WorkItem> ao_items;
  int tile[3] = {-1, -1, -1};
  int tile_w32 = -1, tile_o32 = -1;
  std::vector<WorkItem> g_items[3];
  std::vector<GemmArgs> g_jobs[3];  // host copies of the product job tables
  DevBuf d_ao_items, d_g_items[3];
  DevBuf d_ao_jobs, d_adj_jobs, d_g_jobs[3], d_red_jobs, d_red_prefix, d_nred_jobs,
      d_nred_prefix, d_split_jobs, d_split_prefix, d_pad_jobs, d_pad_prefix;
  int n_red = 0, n_nred = 0, n_split = 0, n_pad = 0;
  int64_t red_total = 0, nred_total = 0, split_total = 0, pad_total = 0;

  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_adj = -1, graph_o32 = -1, graph_w32 = -1;
  std::vector<const void*> graph_addrs;
  hipStream_t own_stream = nullptr;

  ~qmk_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (own_stream) (void)hipStreamDestroy(own_stream);
  }
};

namespace {

qmk_status bfail(qmk_batch b, qmk_status st, const std::string& m) {
  b->err = m;
  return st;
}
qmk_status bhip(qmk_batch b, hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return bfail(b, QMK_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
  return bfail(b, QMK_HIP_ERROR, std::string(what) + ": " + hipGetErrorString(e));
}
#define QMK_BHIP(b, expr, what)                      \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return bhip(b, e_, what);  \
  } while (0)

void drop_graph(qmk_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_adj = b->graph_o32 = b->graph_w32 = -1;
}

// Work list of one product for tile `cfg`: (molecule, M tile, N tile, z),
// longest reduction first.
std::vector<WorkItem> gemm_items(qmk_batch b, GemmKind kind, int cfg) {
  const TileCfg t = gemm_tile(b->prec, cfg);
  struct Key {
    int64_t cost;
    WorkItem it;
  };
  std::vector<Key> v;
  for (size_t m = 0; m < b->plan.size(); ++m) {
    const MolPlan& mp = b->plan[m];
    int64_t M, N, L, nz;
    if (kind == GemmKind::kForward) {
      M = mp.P; N = mp.N; L = mp.K; nz = 5;
    } else if (kind == GemmKind::kGbar) {
      M = mp.K; N = mp.P; L = mp.N; nz = 5;  // rows k, columns p (gbar_args)
    } else {
      M = mp.N; N = mp.K; L = mp.chunk; nz = 5 * mp.nsplit;
    }
    const int64_t nM = (M + t.bm() - 1) / t.bm(), nN = (N + t.bn() - 1) / t.bn();
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t i = 0; i < nM; ++i)
        for (int64_t j = 0; j < nN; ++j)
          v.push_back({L, WorkItem{static_cast<int32_t>(m), static_cast<int32_t>(i),
                                   static_cast<int32_t>(j), static_cast<int32_t>(z)}});
  }
  std::stable_sort(v.begin(), v.end(), [](const Key& a, const Key& c) { return a.cost > c.cost; });
  std::vector<WorkItem> out(v.size());
  for (size_t i = 0; i < v.size(); ++i) out[i] = v[i].it;
  return out;
}

qmk_status make_plan(qmk_batch b, hipStream_t s) {
  drop_graph(b);
  b->plan.clear();
  b->tile[0] = b->tile[1] = b->tile[2] = -1;
  size_t ao = 0, dc = 0, nuc = 0, elec = 0, dis = 0, wsp = 0, wpd = 0;
  const bool planes = b->prec == Prec::kBF16P;
  b->max_smem = 0;
  std::vector<std::pair<int64_t, WorkItem>> ao_items;
  for (size_t m = 0; m < b->ctxs.size(); ++m) {
    qmk_ctx c = b->ctxs[m];
    MolPlan mp{};
    mp.P = c->P();
    mp.K = c->ao_num;
    mp.N = c->mo_num;
    mp.Pp = round_up(mp.P, kPointPad);
    mp.Kp = c->Kp;
    mp.Np = c->Np;
    mp.Nw = round_up(mp.N, 32);
    mp.nucl_num = c->nucl_num;
    mp.n_groups = c->n_groups;
    mp.nucl_dev = c->nucl_dev;
    mp.ao_off = ao;
    mp.gbar_off = ao;
    ao += static_cast<size_t>(mp.Kp * 5 * mp.Pp);
    mp.chunk = std::min<int64_t>(kDcoefChunk, round_up(mp.P, 32));
    mp.nsplit = (mp.P + mp.chunk - 1) / mp.chunk;
    mp.dc_off = dc;
    dc += static_cast<size_t>(5 * mp.nsplit * mp.Np * mp.Kp);
    mp.w_off = wsp;
    if (planes) wsp += static_cast<size_t>(2 * mp.Pp * 5 * mp.Nw);
    // the products load W in 16-byte pieces: 2 FP64 or 4 FP32 weights
    mp.pad_w = !planes && (5 * mp.N) % (b->prec == Prec::kF64 ? 2 : 4) != 0;
    mp.ldw = mp.pad_w ? round_up(mp.N, 4) : mp.N;
    mp.wp_off = wpd;
    if (mp.pad_w) wpd += static_cast<size_t>(mp.P * 5 * mp.ldw);
    mp.n_waves = (mp.P + 255) / 256 * 4;
    mp.nuc_off = nuc;
    nuc += static_cast<size_t>(mp.n_waves * mp.nucl_dev * 3);
    mp.elec_off = elec;
    if (mp.n_groups > 1) elec += static_cast<size_t>(mp.n_groups * mp.P * 3);
    mp.scratch_coef = dis;
    dis += static_cast<size_t>(mp.N * mp.K);
    mp.scratch_elec = dis;
    dis += static_cast<size_t>(mp.P * 3);
    mp.scratch_nucl = dis;
    dis += static_cast<size_t>(mp.nucl_num * 3);
    b->max_smem = std::max(b->max_smem, static_cast<size_t>(c->tab.smem_bytes));
    const int64_t nb = (mp.P + 255) / 256;
    for (int64_t bx = 0; bx < nb; ++bx)
      for (int gy = 0; gy < mp.n_groups; ++gy)
        ao_items.push_back({mp.K, WorkItem{static_cast<int32_t>(m), static_cast<int32_t>(bx), gy, 0}});
    b->plan.push_back(mp);
  }
  std::stable_sort(ao_items.begin(), ao_items.end(),
                   [](const std::pair<int64_t, WorkItem>& a, const std::pair<int64_t, WorkItem>& c) {
                     return a.first > c.first;
                   });
  b->ao_items.resize(ao_items.size());
  for (size_t i = 0; i < ao_items.size(); ++i) b->ao_items[i] = ao_items[i].second;

  QMK_BHIP(b, b->ao.ensure(std::max<size_t>(ao, 1) * b->esz), "alloc batch AO arena");
  QMK_BHIP(b, hipMemsetAsync(b->ao.p, 0, std::max<size_t>(ao, 1) * b->esz, s), "clear AO arena");
  QMK_BHIP(b, b->gbar.ensure(std::max<size_t>(ao, 1) * b->esz), "alloc batch Gbar arena");
  QMK_BHIP(b, b->ws_dc.ensure(std::max<size_t>(dc, 1) * 8), "alloc batch dC partials");
  QMK_BHIP(b, b->ws_nuc.ensure(std::max<size_t>(nuc, 1) * 8), "alloc batch nucleus partials");
  QMK_BHIP(b, b->ws_elec.ensure(std::max<size_t>(elec, 1) * 8), "alloc batch electron partials");
  QMK_BHIP(b, b->discard.ensure(std::max<size_t>(dis, 1) * 8), "alloc batch discard arena");
  if (planes) QMK_BHIP(b, b->wsplit.ensure(std::max<size_t>(wsp, 1) * 2), "alloc batch split W");
  if (wpd) QMK_BHIP(b, b->wpad.ensure(wpd * 8), "alloc batch padded W");
  QMK_BHIP(b, upload(b->d_ao_items, b->ao_items, s), "upload AO work list");
  b->planned = true;
  return QMK_OK;
}

// Per-molecule GEMM arguments, as the single-context calls build them.
// w (FP64 / FP32 modes): rows of ldw weights; pad: rows padded with zeros.
GemmArgs gemm_job(qmk_batch b, size_t m, GemmKind kind, void* out, const void* w, int64_t ldw = 0,
                  int pad = 0) {
  qmk_ctx c = b->ctxs[m];
  const MolPlan& mp = b->plan[m];
  const bool planes = b->prec == Prec::kBF16P;
  const char* aop = static_cast<const char*>(b->ao.p) + mp.ao_off * b->esz;
  // bf16 planes: the AO array's lo plane follows its hi plane; W's planes
  // [Pp][5][Nw] sit in the split-W arena
  const uint16_t* ao_lo = reinterpret_cast<const uint16_t*>(aop) + mp.Kp * 5 * mp.Pp;
  const uint16_t* w_hi = b->wsplit.as<uint16_t>() + mp.w_off;
  const uint16_t* w_lo = w_hi + mp.Pp * 5 * mp.Nw;
  char* gbp = static_cast<char*>(b->gbar.p) + mp.gbar_off * b->esz;
  GemmArgs g{};
  g.nsplit = 1;
  g.nbatch = 5;
  if (kind == GemmKind::kForward) {
    g.A = aop;
    g.sAi = 1;
    g.sAl = 5 * mp.Pp;
    g.oAc = mp.Pp;
    g.pad_ok = 3;  // AO rows padded to Pp points, C^T rows to Np MOs
    if (planes) {
      g.A2 = ao_lo;
      g.B = c->d_Cb_hi.p;
      g.B2 = c->d_Cb_lo.p;
      g.sBl = 1;
      g.sBj = mp.Kp;
    } else {
      g.B = c->d_Ct.p;
      g.sBl = mp.Np;
      g.sBj = 1;
    }
    g.D = out;
    g.sDi = 5 * mp.N;
    g.sDj = 1;
    g.oDz = mp.N;
    g.M = mp.P;
    g.N = mp.N;
    g.L = g.Lchunk = mp.K;
  } else if (kind == GemmKind::kGbar) {
    g = gbar_args(b->prec, planes ? static_cast<const void*>(w_hi) : w, w_lo, planes ? mp.Nw : ldw, c->d_C.p,
                  c->d_Ctb_hi.p,
                  c->d_Ctb_lo.p, gbp, mp.P, mp.Pp, mp.K, mp.Kp, mp.N, mp.Np);
  } else {
    g.A = w;
    g.sAi = 1;
    g.sAl = 5 * ldw;
    g.oAc = ldw;
    g.oAs = mp.chunk * 5 * ldw;
    g.pad_ok = pad;
    g.B = aop;
    g.sBl = 1;
    g.sBj = 5 * mp.Pp;
    g.oBc = mp.Pp;
    g.oBs = mp.chunk;
    g.D = static_cast<double*>(b->ws_dc.p) + mp.dc_off;
    g.sDi = mp.Kp;
    g.sDj = 1;
    g.oDz = mp.Np * mp.Kp;
    g.M = mp.N;
    g.N = mp.K;
    g.L = mp.P;
    g.Lchunk = mp.chunk;
    g.nsplit = static_cast<int32_t>(mp.nsplit);
    if (planes) {
      g.A = w_hi;
      g.A2 = w_lo;
      g.sAl = 5 * mp.Nw;
      g.oAc = mp.Nw;
      g.oAs = mp.chunk * 5 * mp.Nw;
      g.B2 = ao_lo;
    }
  }
  return g;
}

int persist_grid(qmk_batch b, int per_cu, size_t n_items) {
  const int64_t g = static_cast<int64_t>(per_cu) * b->n_cu;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(g, static_cast<int64_t>(n_items))));
}

std::string batch_key(qmk_batch b, GemmKind kind) {
  std::ostringstream o;
  uint64_t h = 1469598103934665603ull;
  for (int64_t v : b->dims_key) {
    h ^= static_cast<uint64_t>(v);
    h *= 1099511628211ull;
  }
  o << device_arch(b->device) << "/batch/k" << static_cast<int>(kind) << "/p"
    << static_cast<int>(b->prec) << "/w" << b->tile_w32 << "/o" << b->tile_o32 << "/n"
    << b->ctxs.size() << "/h" << std::hex << h;
  return o.str();
}

// Picks (timing every feasible tile when tuning is on) the tile of one product
// for the whole batch and uploads its work list.  The job table of `kind`
// must already be on the device.
qmk_status choose_batch_tile(qmk_batch b, GemmKind kind, hipStream_t s) {
  const int k = static_cast<int>(kind);
  if (b->tile[k] >= 0) return QMK_OK;
  const std::string key = batch_key(b, kind);
  // the pre-split kernel addresses its tiles by 32-bit offsets: every job's
  // strides must fit the tile
  auto usable = [&](int cfg) {
    if (!tile_feasible(b->prec, cfg)) return false;
    if (b->prec != Prec::kBF16P) return true;
    for (const GemmArgs& g : b->g_jobs[k])
      if (!gemm_bf16p_args_ok(cfg, g)) return false;
    return true;
  };
  int best = tune_cache_get(key);
  if (best < 0 || best >= gemm_num_tiles(b->prec) || !usable(best)) {
    best = -1;
    float best_ms = -1.0f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QMK_BHIP(b, hipEventCreate(&e0), "event");
    QMK_BHIP(b, hipEventCreate(&e1), "event");
    for (int cfg = 0; cfg < gemm_num_tiles(b->prec); ++cfg) {
      if (!usable(cfg)) continue;
      if (best < 0) best = cfg;
      if (!tuning_on()) break;
      std::vector<WorkItem> items = gemm_items(b, kind, cfg);
      QMK_BHIP(b, upload(b->d_g_items[k], items, s), "upload work list");
      const int grid = persist_grid(
          b, gemm_persist_blocks_per_cu(kind, b->prec, cfg, b->tile_w32, b->tile_o32), items.size());
      auto run = [&]() {
        return launch_gemm_persist(kind, b->prec, cfg, b->d_g_jobs[k].as<GemmArgs>(),
                                   b->d_g_items[k].as<WorkItem>(), static_cast<int>(items.size()),
                                   grid, b->tile_w32, b->tile_o32, s);
      };
      QMK_BHIP(b, run(), "tile trial");
      QMK_BHIP(b, hipEventRecord(e0, s), "event");
      QMK_BHIP(b, run(), "tile trial");
      QMK_BHIP(b, hipEventRecord(e1, s), "event");
      QMK_BHIP(b, hipEventSynchronize(e1), "tile trial");
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (best_ms < 0.0f || ms < best_ms) {
        best_ms = ms;
        best = cfg;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best < 0) return bfail(b, QMK_UNSUPPORTED, "no tile fits in LDS and the operands' strides");
    tune_cache_put(key, best);
  }
  b->tile[k] = best;
  b->g_items[k] = gemm_items(b, kind, best);
  QMK_BHIP(b, upload(b->d_g_items[k], b->g_items[k], s), "upload work list");
  return QMK_OK;
}

// Enqueues the whole batch (forward, and the adjoint when with_adj).
qmk_status enqueue_all(qmk_batch b, bool with_adj, hipStream_t s) {
  const int f32 = b->esz == 4;  // Gbar in FP32 (both mixed modes)
  const int ao_grid = persist_grid(b, ao_persist_blocks_per_cu(b->ao_fmt, b->max_smem), b->ao_items.size());
  QMK_BHIP(b, launch_ao_vgl_persist(b->d_ao_jobs.as<AoJob>(), b->d_ao_items.as<WorkItem>(),
                                    static_cast<int>(b->ao_items.size()), ao_grid, b->max_smem, b->ao_fmt, s),
           "batch AO stage");
  auto gemm = [&](GemmKind kind) -> hipError_t {
    const int k = static_cast<int>(kind);
    const int cfg = b->tile[k];
    const int grid = persist_grid(
        b, gemm_persist_blocks_per_cu(kind, b->prec, cfg, b->tile_w32, b->tile_o32), b->g_items[k].size());
    return launch_gemm_persist(kind, b->prec, cfg, b->d_g_jobs[k].as<GemmArgs>(),
                               b->d_g_items[k].as<WorkItem>(),
                               static_cast<int>(b->g_items[k].size()), grid, b->tile_w32,
                               b->tile_o32, s);
  };
  QMK_BHIP(b, gemm(GemmKind::kForward), "batch contraction");
  if (!with_adj) return QMK_OK;
  if (b->n_pad)
    QMK_BHIP(b, launch_pad_rows_batch(b->d_pad_jobs.as<PadJob>(), b->d_pad_prefix.as<int64_t>(), b->n_pad,
                                      b->pad_total, b->tile_w32, s),
             "batch W padding");
  if (b->prec == Prec::kBF16P)
    QMK_BHIP(b, launch_split_w_batch(b->d_split_jobs.as<SplitJob>(), b->d_split_prefix.as<int64_t>(), b->n_split,
                                     b->split_total, b->tile_w32, s),
             "batch W split");
  QMK_BHIP(b, gemm(GemmKind::kGbar), "batch W C product");
  const int adj_grid = persist_grid(b, adj_persist_blocks_per_cu(f32, b->max_smem), b->ao_items.size());
  QMK_BHIP(b, launch_ao_adjoint_persist(b->d_adj_jobs.as<AdjJob>(), b->d_ao_items.as<WorkItem>(),
                                        static_cast<int>(b->ao_items.size()), adj_grid, b->max_smem,
                                        f32, s),
           "batch AO adjoint");
  QMK_BHIP(b, gemm(GemmKind::kDcoef), "batch W^T ao product");
  QMK_BHIP(b, launch_reduce_batch(b->d_red_jobs.as<RedJob>(), b->d_red_prefix.as<int64_t>(), b->n_red,
                                  b->red_total, s),
           "batch reductions");
  QMK_BHIP(b, launch_reduce_nuc_batch(b->d_nred_jobs.as<NucRedJob>(), b->d_nred_prefix.as<int64_t>(),
                                      b->n_nred, b->nred_total, s),
           "batch nucleus reductions");
  return QMK_OK;
}

}  // namespace

extern "C" {

qmk_status qmk_batch_create(qmk_batch* out, const qmk_ctx* ctxs, int64_t n) {
  if (!out) return QMK_INVALID_ARG_BASE + 1;
  if (!ctxs) return QMK_INVALID_ARG_BASE + 2;
  if (n < 1 || n > (1 << 20)) return QMK_INVALID_ARG_BASE + 3;
  for (int64_t i = 0; i < n; ++i)
    if (!valid_ctx(ctxs[i])) return QMK_INVALID_CONTEXT;
  for (int64_t i = 1; i < n; ++i)
    if (ctxs[i]->device != ctxs[0]->device) return QMK_INVALID_ARG_BASE + 2;
  qmk_batch b = new (std::nothrow) qmk_batch_s();
  if (!b) return QMK_OUT_OF_MEMORY;
  b->ctxs.assign(ctxs, ctxs + n);
  b->device = ctxs[0]->device;
  *out = b;
  return QMK_OK;
}

qmk_status qmk_batch_destroy(qmk_batch b) {
  if (!b || b->magic != kBatchMagic) return QMK_INVALID_CONTEXT;
  DeviceGuard g(b->device);
  (void)hipDeviceSynchronize();
  b->magic = 0;
  delete b;
  return QMK_OK;
}

const char* qmk_batch_last_error(qmk_batch b) {
  if (!b || b->magic != kBatchMagic) return "invalid batch";
  return b->err.c_str();
}

qmk_status qmk_batch_run(qmk_batch b, void* const* outs, int32_t dtype, const void* const* ws,
                         double* const* d_coefs, double* const* d_elecs, double* const* d_nucls,
                         void* hip_stream) {
  if (!b || b->magic != kBatchMagic) return QMK_INVALID_CONTEXT;
  if (!outs) return bfail(b, QMK_INVALID_ARG_BASE + 2, "argument 2: NULL outputs");
  if (dtype != QMK_F64 && dtype != QMK_F32) return bfail(b, QMK_INVALID_ARG_BASE + 3, "argument 3: dtype");
  const size_t n = b->ctxs.size();
  DeviceGuard guard(b->device);
  auto dev_ok = [&](const void* p) { return p && device_accessible(p, b->device); };
  for (size_t i = 0; i < n; ++i) {
    const std::string at = " " + std::to_string(i) + " (NULL or not memory the device can access)";
    if (!dev_ok(outs[i])) return bfail(b, QMK_INVALID_ARG_BASE + 2, "argument 2: output" + at);
    if (ws && !dev_ok(ws[i])) return bfail(b, QMK_INVALID_ARG_BASE + 4, "argument 4: weights" + at);
    if (ws && d_coefs && d_coefs[i] && !dev_ok(d_coefs[i]))
      return bfail(b, QMK_INVALID_ARG_BASE + 5, "argument 5: dL/dC" + at);
    if (ws && d_elecs && d_elecs[i] && !dev_ok(d_elecs[i]))
      return bfail(b, QMK_INVALID_ARG_BASE + 6, "argument 6: dL/dr" + at);
    if (ws && d_nucls && d_nucls[i] && !dev_ok(d_nucls[i]))
      return bfail(b, QMK_INVALID_ARG_BASE + 7, "argument 7: dL/dR" + at);
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const bool own = s == nullptr;
  if (own) {
    if (!b->own_stream) QMK_BHIP(b, hipStreamCreate(&b->own_stream), "stream");  // blocking: ordered after null-stream work
    s = b->own_stream;
  }
  const bool with_adj = ws != nullptr;

  // inputs of every context, and the dimensions they imply
  const int mode = b->ctxs[0]->mode;
  std::vector<int64_t> key;
  for (size_t i = 0; i < n; ++i) {
    qmk_ctx c = b->ctxs[i];
    if (!valid_ctx(c)) return bfail(b, QMK_INVALID_CONTEXT, "context " + std::to_string(i) + " destroyed");
    if (c->mode != mode) return bfail(b, QMK_INVALID_ARG_BASE + 1, "contexts use different precision modes");
    qmk_status st = check_ready(c, true);
    if (st != QMK_OK) return bfail(b, st, "context " + std::to_string(i) + ": " + c->err);
    if (c->cusp_on)
      return bfail(b, QMK_UNSUPPORTED, "context " + std::to_string(i) + " has the cusp correction on");
    if ((st = ensure_tables(c)) != QMK_OK) return bfail(b, st, c->err);
    if ((st = ensure_coef(c)) != QMK_OK) return bfail(b, st, c->err);
    key.insert(key.end(), {c->P(), c->ao_num, c->mo_num, c->nucl_num, c->n_groups, c->nucl_dev,
                           static_cast<int64_t>(c->tab.smem_bytes)});
  }
  key.push_back(mode);
  if (!b->planned || key != b->dims_key || b->mode != mode) {
    b->mode = mode;
    b->prec = mode == QMK_FP64 ? Prec::kF64 : (mode == QMK_MIXED_F32 ? Prec::kF32 : Prec::kBF16P);
    b->esz = mode == QMK_FP64 ? 8 : 4;
    b->ao_fmt = mode == QMK_FP64 ? 0 : (mode == QMK_MIXED_F32 ? 1 : 2);
    b->dims_key = key;
    int ncu = 0;
    QMK_BHIP(b, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, b->device), "attr");
    b->n_cu = ncu > 0 ? ncu : 1;
    qmk_status st = make_plan(b, s);
    if (st != QMK_OK) return st;
  }
  const int o32 = dtype == QMK_F32;
  const int w32 = o32;  // weights have the output's element type
  if (b->tile_o32 != o32 || b->tile_w32 != w32) {
    b->tile[0] = b->tile[1] = b->tile[2] = -1;
    b->tile_o32 = o32;
    b->tile_w32 = w32;
    drop_graph(b);
  }

  // job tables from the current state of every context
  std::vector<AoJob> ao_jobs(n);
  std::vector<AdjJob> adj_jobs(n);
  std::vector<GemmArgs> gj[3];
  std::vector<RedJob> red;
  std::vector<int64_t> red_prefix{0};
  std::vector<NucRedJob> nred;
  std::vector<int64_t> nred_prefix{0};
  std::vector<SplitJob> split;
  std::vector<int64_t> split_prefix{0};
  std::vector<PadJob> pads;
  std::vector<int64_t> pad_prefix{0};
  for (size_t i = 0; i < n; ++i) {
    qmk_ctx c = b->ctxs[i];
    const MolPlan& mp = b->plan[i];
    AoTables t = c->tab;
    t.T = (c->bits - 1) * std::log(2.0);
    const PointArgs pa = point_args(c);
    char* aop = static_cast<char*>(b->ao.p) + mp.ao_off * b->esz;
    ao_jobs[i] = AoJob{t, pa, AoOut{aop, 5 * mp.Pp, mp.Pp, 1}};
    ao_jobs[i].out.plane = mp.Kp * 5 * mp.Pp;  // bf16 planes: lo plane offset
    gj[0].push_back(gemm_job(b, i, GemmKind::kForward, outs[i], nullptr));
    if (with_adj) {
      double* de = (d_elecs && d_elecs[i]) ? d_elecs[i]
                                           : static_cast<double*>(b->discard.p) + mp.scratch_elec;
      double* dn = (d_nucls && d_nucls[i]) ? d_nucls[i]
                                           : static_cast<double*>(b->discard.p) + mp.scratch_nucl;
      double* dc = (d_coefs && d_coefs[i]) ? d_coefs[i]
                                           : static_cast<double*>(b->discard.p) + mp.scratch_coef;
      double* elec_out = de;
      int64_t gstride = 0;
      if (mp.n_groups > 1) {
        elec_out = static_cast<double*>(b->ws_elec.p) + mp.elec_off;
        gstride = mp.P * 3;
        red.push_back(RedJob{elec_out, mp.n_groups, mp.P, 3, 3, mp.P * 3, de, 3});
        red_prefix.push_back(red_prefix.back() + mp.P * 3);
      }
      adj_jobs[i] = AdjJob{t, pa, static_cast<char*>(b->gbar.p) + mp.gbar_off * b->esz, 5 * mp.Pp,
                           mp.Pp, elec_out, gstride,
                           static_cast<double*>(b->ws_nuc.p) + mp.nuc_off};
      if (b->prec == Prec::kBF16P) {
        uint16_t* hi = b->wsplit.as<uint16_t>() + mp.w_off;
        const size_t esz_w = w32 ? 4 : 8;
        // vector loads need every group of eight weights to start 16-byte aligned
        const int vec = reinterpret_cast<uintptr_t>(ws[i]) % 16 == 0 && (mp.N * esz_w) % 16 == 0;
        split.push_back(SplitJob{ws[i], mp.P, mp.N, mp.Pp, mp.Nw, vec, hi, hi + mp.Pp * 5 * mp.Nw});
        const int64_t nj = mp.Pp * 5 * (mp.Nw / 8);
        if (nj > 0xffffffffLL) return bfail(b, QMK_SIZE, "context " + std::to_string(i) + ": W too large to split");
        split_prefix.push_back(split_prefix.back() + nj);
      }
      // FP64 / FP32 products on weights of their own type read a padded copy
      // where the caller's rows do not allow 16-byte loads
      const void* wj = ws[i];
      int64_t ldw = mp.N;
      int padded = 0;
      if (mp.pad_w && ((b->prec == Prec::kF64 && !w32) || (b->prec == Prec::kF32 && w32))) {
        char* dst = static_cast<char*>(b->wpad.p) + mp.wp_off * (w32 ? 4 : 8);
        pads.push_back(PadJob{ws[i], dst, 5 * mp.P, mp.N, mp.ldw});
        pad_prefix.push_back(pad_prefix.back() + 5 * mp.P * (mp.ldw / 4));
        wj = dst;
        ldw = mp.ldw;
        padded = 1;
      }
      gj[1].push_back(gemm_job(b, i, GemmKind::kGbar, nullptr, wj, ldw, padded));
      gj[2].push_back(gemm_job(b, i, GemmKind::kDcoef, nullptr, wj, ldw, padded));
      red.push_back(RedJob{static_cast<double*>(b->ws_dc.p) + mp.dc_off, 5 * mp.nsplit, mp.N, mp.K,
                           mp.Kp, mp.Np * mp.Kp, dc, mp.K});
      red_prefix.push_back(red_prefix.back() + mp.N * mp.K);
      nred.push_back(NucRedJob{static_cast<double*>(b->ws_nuc.p) + mp.nuc_off, mp.n_waves,
                               mp.nucl_dev, static_cast<int32_t>(mp.nucl_num),
                               c->d_devof.as<int32_t>(), dn});
      nred_prefix.push_back(nred_prefix.back() + mp.nucl_num * 3);
    }
  }
  QMK_BHIP(b, upload(b->d_ao_jobs, ao_jobs, s), "upload jobs");
  QMK_BHIP(b, upload(b->d_g_jobs[0], gj[0], s), "upload jobs");
  if (with_adj) {
    QMK_BHIP(b, upload(b->d_adj_jobs, adj_jobs, s), "upload jobs");
    QMK_BHIP(b, upload(b->d_g_jobs[1], gj[1], s), "upload jobs");
    QMK_BHIP(b, upload(b->d_g_jobs[2], gj[2], s), "upload jobs");
    QMK_BHIP(b, upload(b->d_red_jobs, red, s), "upload jobs");
    QMK_BHIP(b, upload(b->d_red_prefix, red_prefix, s), "upload jobs");
    QMK_BHIP(b, upload(b->d_nred_jobs, nred, s), "upload jobs");
    QMK_BHIP(b, upload(b->d_nred_prefix, nred_prefix, s), "upload jobs");
    QMK_BHIP(b, upload(b->d_split_jobs, split, s), "upload jobs");
    QMK_BHIP(b, upload(b->d_split_prefix, split_prefix, s), "upload jobs");
    b->n_split = static_cast<int>(split.size());
    b->split_total = split_prefix.back();
    QMK_BHIP(b, upload(b->d_pad_jobs, pads, s), "upload jobs");
    QMK_BHIP(b, upload(b->d_pad_prefix, pad_prefix, s), "upload jobs");
    b->n_pad = static_cast<int>(pads.size());
    b->pad_total = pad_prefix.back();
    b->n_red = static_cast<int>(red.size());
    b->red_total = red_prefix.back();
    b->n_nred = static_cast<int>(nred.size());
    b->nred_total = nred_prefix.back();
  }

  for (int k = 0; k < 3; ++k) b->g_jobs[k] = gj[k];

  // tiles (timed once per batch shape), then one graph per (adjoint, dtype)
  qmk_status st;
  if ((st = choose_batch_tile(b, GemmKind::kForward, s)) != QMK_OK) return st;
  if (with_adj) {
    if ((st = choose_batch_tile(b, GemmKind::kGbar, s)) != QMK_OK) return st;
    if ((st = choose_batch_tile(b, GemmKind::kDcoef, s)) != QMK_OK) return st;
  }
  // the graph bakes in the addresses of the job tables and work lists
  std::vector<const void*> addrs = {b->d_ao_jobs.p, b->d_ao_items.p, b->d_adj_jobs.p,
                                    b->d_red_jobs.p, b->d_red_prefix.p, b->d_nred_jobs.p,
                                    b->d_nred_prefix.p, b->ao.p, b->gbar.p};
  addrs.push_back(b->d_split_jobs.p);
  addrs.push_back(b->d_split_prefix.p);
  addrs.push_back(b->wsplit.p);
  addrs.push_back(b->d_pad_jobs.p);
  addrs.push_back(b->d_pad_prefix.p);
  addrs.push_back(b->wpad.p);
  for (int k = 0; k < 3; ++k) {
    addrs.push_back(b->d_g_jobs[k].p);
    addrs.push_back(b->d_g_items[k].p);
  }
  if (addrs != b->graph_addrs) drop_graph(b);
  if (!b->exec || b->graph_adj != (with_adj ? 1 : 0) || b->graph_o32 != o32 || b->graph_w32 != w32) {
    drop_graph(b);
    QMK_BHIP(b, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "begin capture");
    st = enqueue_all(b, with_adj, s);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s, &graph);
    if (st != QMK_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (ec != hipSuccess) return bhip(b, ec, "end capture");
    b->graph = graph;
    QMK_BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate graph");
    b->graph_adj = with_adj ? 1 : 0;
    b->graph_o32 = o32;
    b->graph_w32 = w32;
    b->graph_addrs = addrs;
  }
  QMK_BHIP(b, hipGraphLaunch(b->exec, s), "graph launch");
  if (own) QMK_BHIP(b, hipStreamSynchronize(s), "synchronize");
  return QMK_OK;
}

}  // extern "C"
