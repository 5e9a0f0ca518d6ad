// qmk_get_mo_vgl_noalloc: the forward mo_vgl of qmk_get_mo_vgl without any
// device or host allocation in the call, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// allocation).
//
// The AO array, the only intermediate of the forward pass, is placed in a
// file-scope device array of fixed size instead of the context's own buffer.
// Each GPU holds its own copy of the array, at its own address, from the
// first call on that GPU until the process ends.  Host code never uses the
// array's name as an address: the address is taken once per device with
// hipGetSymbolAddress and kept in a per-device table.
#include <mutex>

#include "ctx_internal.h"

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current).
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// Zeroes the padding of an AO array [Kp][5][Pp] holding `rows` = 5 K real
// rows of P points: columns P .. Pp-1 of the real rows and all of the rows
// rows .. total_rows-1.  The AO kernel writes every real (row, point) entry
// and the products read the padding without bounds tests, so the padding
// must hold zeros; the array is shared by every call on the GPU and keeps
// the previous call's contents.
template <typename T>
__global__ __launch_bounds__(256) void clear_ao_padding(T* __restrict__ ao, int64_t rows, int64_t P,
                                                        int64_t Pp, int64_t total_rows) {
  const int64_t pad = Pp - P;
  const int64_t n1 = rows * pad;
  const int64_t n = n1 + (total_rows - rows) * Pp;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    if (i < n1)
      ao[(i / pad) * Pp + P + i % pad] = T(0);
    else
      ao[rows * Pp + (i - n1)] = T(0);
  }
}

}  // namespace

using namespace qmk;

extern "C" qmk_status qmk_get_mo_vgl_noalloc(qmk_ctx ctx, void* out, int64_t size_max, int32_t dtype,
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
  if (ctx->cusp_on)
    return fail(ctx, QMK_UNSUPPORTED, "the no-allocation forward pass has no cusp correction");
  const int want = ctx->mode == QMK_FP64 ? 0 : (ctx->mode == QMK_MIXED_F32 ? 1 : 2);
  if (ctx->tables_dirty || ctx->coef_dirty || ctx->coef_mode != want)
    return fail(ctx, QMK_NOT_SET,
                "the device copies of the basis tables and MO coefficients for this precision mode are "
                "not built: call qmk_get_mo_vgl once after the last set_nucleus, set_basis, set_mo_coef "
                "or set_precision (that call allocates them)");
  const int fmt = ctx->ao_format();  // 0 FP64, 1 FP32, 2 bf16 hi and lo planes
  const int64_t Pp = round_up(P, kPointPad), Kp = round_up(K, kAoPad);
  const size_t need = static_cast<size_t>(Kp) * 5 * static_cast<size_t>(Pp) * (fmt ? 4 : 8);
  if (need > kScratchBytes)
    return fail(ctx, QMK_SIZE,
                "the AO array of " + std::to_string(K) + " AOs at " + std::to_string(P) + " points needs " +
                    std::to_string(need) + " bytes; the no-allocation scratch holds " +
                    std::to_string(kScratchBytes) + " (use qmk_get_mo_vgl, or fewer points per call)");
  DeviceGuard g(ctx->device);
  if ((st = ensure_tables(ctx)) != QMK_OK) return st;  // tables are current: sets the cutoff only
  void* ao = nullptr;
  QMK_HIP(ctx, scratch_address(ctx->device, &ao), "no-allocation scratch address");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);

  const int64_t rows = 5 * K, total_rows = 5 * Kp;
  const int64_t n_pad = rows * (Pp - P) + (total_rows - rows) * Pp;
  if (n_pad > 0) {
    const int blocks = static_cast<int>(std::min<int64_t>((n_pad + 255) / 256, 2048));
    if (fmt == 2) {
      uint16_t* hi = static_cast<uint16_t*>(ao);
      for (uint16_t* plane : {hi, hi + total_rows * Pp})
        hipLaunchKernelGGL(clear_ao_padding<uint16_t>, dim3(blocks), dim3(256), 0, s, plane, rows, P, Pp,
                           total_rows);
    } else if (fmt == 1) {
      hipLaunchKernelGGL(clear_ao_padding<float>, dim3(blocks), dim3(256), 0, s, static_cast<float*>(ao), rows,
                         P, Pp, total_rows);
    } else {
      hipLaunchKernelGGL(clear_ao_padding<double>, dim3(blocks), dim3(256), 0, s, static_cast<double*>(ao),
                         rows, P, Pp, total_rows);
    }
    QMK_HIP(ctx, hipGetLastError(), "clear AO padding");
    ++ctx->launches;
  }
  AoOut o{ao, 5 * Pp, Pp, 1};
  o.plane = total_rows * Pp;
  QMK_HIP(ctx, launch_ao_vgl(ctx->tab, point_args(ctx), o, fmt, fmt, s), "AO kernel");
  ++ctx->launches;

  GemmArgs ga{};
  ga.A = ao;
  ga.sAi = 1;
  ga.sAl = 5 * Pp;
  ga.oAc = Pp;
  if (fmt == 2) {
    ga.A2 = static_cast<const uint16_t*>(ao) + total_rows * Pp;
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
  int cfg = ctx->forced_tile[static_cast<int>(GemmKind::kForward)];
  if (cfg >= 0) {
    if (cfg >= gemm_num_tiles(prec) || !tile_feasible(prec, cfg))
      return fail(ctx, QMK_INVALID_ARG_BASE + 3, "the forced tile does not exist for this product's precision");
  } else {
    cfg = cached_tile(pb, ctx->device);
  }
  QMK_HIP(ctx, launch_gemm_typed(GemmKind::kForward, prec, cfg, ga, 0, o32, s), "MO contraction");
  ++ctx->launches;
  return QMK_OK;
}
