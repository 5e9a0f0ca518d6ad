// GEMM tile autotuner.
//
// For every distinct product (kind, precision, operand types, M, N, L) the
// first call times each tile shape of the kernel's table on the caller's own
// operands (one warm-up launch, then the best of two timed launches with HIP
// events on the caller's stream) and remembers the fastest.  Later calls --
// including calls from other contexts -- reuse the choice.  The table of
// choices can be persisted: QMK_TUNE_CACHE=<file> loads it at first use and
// rewrites it after each new decision (a flat JSON object key -> tile id).
// QMK_TUNE_TABLE=<file> names a read-only table of earlier decisions loaded
// first (the Python binding points it at the table shipped with the
// package), so that runs of known shapes use the same tiles every time.
// QMK_TUNE=0 disables timing and picks the tile with the least padded work.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "qmk_internal.h"

namespace qmk {
namespace {

std::mutex g_mu;
std::map<std::string, int> g_cache;
bool g_loaded = false;

const char* cache_path() {
  const char* p = std::getenv("QMK_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

void load_file_locked(const char* path) {
  if (!path || !*path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    const size_t c = s.find(':', j);
    if (c == std::string::npos) break;
    g_cache[key] = std::atoi(s.c_str() + c + 1);
    i = s.find_first_of(",}", c);
    if (i == std::string::npos) break;
  }
}

void load_cache_locked() {
  if (g_loaded) return;
  g_loaded = true;
  load_file_locked(std::getenv("QMK_TUNE_TABLE"));
  load_file_locked(cache_path());
}

void save_cache_locked() {
  const char* path = cache_path();
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  std::ofstream f(tmp);
  if (!f) return;
  f << "{\n";
  size_t n = 0;
  for (const auto& kv : g_cache) f << "  \"" << kv.first << "\": " << kv.second << (++n < g_cache.size() ? ",\n" : "\n");
  f << "}\n";
  f.close();
  std::rename(tmp.c_str(), path);
}

std::string key_of(const GemmProblem& p, int device) {
  hipDeviceProp_t prop;
  std::string arch = "gfx?";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  std::ostringstream o;
  o << arch << "/k" << static_cast<int>(p.kind) << "/p" << static_cast<int>(p.prec) << "/w" << p.w32
    << "/o" << p.o32 << "/" << p.M << "x" << p.N << "x" << p.L;
  if (p.nbatch != 5) o << "/b" << p.nbatch;
  if (p.sparse) o << "/s";
  return o.str();
}

bool tuning_enabled() {
  const char* e = std::getenv("QMK_TUNE");
  return !(e && std::string(e) == "0");
}

}  // namespace

bool tile_feasible(Prec prec, int cfg) {
  // one workgroup must fit the 160 KiB of LDS of a CDNA4 compute unit
  return gemm_tile_lds_bytes(prec, cfg) <= 160u * 1024u;
}

int default_tile(const GemmProblem& p) {
  int best = -1;
  double best_cost = 0.0;
  for (int c = 0; c < gemm_num_tiles(p.prec); ++c) {
    if (!tile_feasible(p.prec, c)) continue;
    const TileCfg t = gemm_tile(p.prec, c);
    const double pm = static_cast<double>((p.M + t.bm() - 1) / t.bm() * t.bm());
    const double pn = static_cast<double>((p.N + t.bn() - 1) / t.bn() * t.bn());
    // padded work, then a mild preference for large tiles (fewer operand loads)
    const double cost = pm * pn * (1.0 + 8.0 / t.bm() + 8.0 / t.bn()) * (t.bk == 16 ? 1.0 : 1.01);
    if (best < 0 || cost < best_cost) {
      best = c;
      best_cost = cost;
    }
  }
  return best < 0 ? 0 : best;
}

int choose_tile(const GemmProblem& p, int device, hipStream_t s,
                const std::function<hipError_t(int)>& enqueue, hipError_t* err) {
  *err = hipSuccess;
  const std::string key = key_of(p, device);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_cache_locked();
    auto it = g_cache.find(key);
    if (it != g_cache.end() && it->second >= 0 && it->second < gemm_num_tiles(p.prec) &&
        tile_feasible(p.prec, it->second))
      return it->second;
  }
  int best = default_tile(p);
  if (tuning_enabled()) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      return best;
    }
    float best_ms = -1.0f;
    for (int c = 0; c < gemm_num_tiles(p.prec); ++c) {
      if (!tile_feasible(p.prec, c)) continue;
      hipError_t e = enqueue(c);  // warm-up
      if (e != hipSuccess) continue;
      float t_min = -1.0f;
      for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(a, s);
        e = enqueue(c);
        (void)hipEventRecord(b, s);
        if (e != hipSuccess) break;
        if ((e = hipEventSynchronize(b)) != hipSuccess) {
          *err = e;
          break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (t_min < 0.0f || ms < t_min) t_min = ms;
      }
      if (*err != hipSuccess) break;
      if (t_min >= 0.0f && (best_ms < 0.0f || t_min < best_ms)) {
        best_ms = t_min;
        best = c;
      }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (*err != hipSuccess) return best;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[key] = best;
  save_cache_locked();
  return best;
}

int cached_tile(const GemmProblem& p, int device) {
  const std::string key = key_of(p, device);
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  auto it = g_cache.find(key);
  if (it != g_cache.end() && it->second >= 0 && it->second < gemm_num_tiles(p.prec) &&
      tile_feasible(p.prec, it->second))
    return it->second;
  return default_tile(p);
}

int tune_cache_get(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  auto it = g_cache.find(key);
  return it == g_cache.end() ? -1 : it->second;
}

void tune_cache_put(const std::string& key, int cfg) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_cache_locked();
  g_cache[key] = cfg;
  save_cache_locked();
}

bool tuning_on() { return tuning_enabled(); }

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  std::string arch = "gfx?";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  return colon == std::string::npos ? arch : arch.substr(0, colon);
}

void forget_tuning() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache.clear();
}

}  // namespace qmk
