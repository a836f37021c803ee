// Autotuner for the launch shapes of the Wilson stencil and of the tall-skinny contractions.
//
// For one (device architecture, lattice extents, precision, batch size) the
// tuner times every (variant, block order) candidate of the stencil with HIP
// events on the context's stream -- a warm-up launch, then `reps` back-to-back
// launches on device fields -- and keeps the fastest.  The contractions
// (V^H W and X += V D over FP64, FP32 or BF16 bases, and the basis rebuild
// Y = V G) are tuned the same way per (architecture, kind, field length,
// vectors, columns): grid size, row tiles per matrix-core launch, outputs per
// block and block-to-XCD mapping.  Choices live in process-wide tables (so
// every operator of a process makes the same choice and results are
// reproducible within a run) and in a text cache file, one line per key:
//
//     <arch> <Lx>x<Ly>x<Lz>x<Lt> <prec> <nrhs> <variant> <order> <us>      (stencil)
//     K <arch> <kind> <n> <nv> <nw> <grid> <tile> <us>                     (contraction)
//
// The file is $DEFLAN_TUNE_CACHE, else $HOME/.cache/deflan/tune.txt.
// DEFLAN_AUTOTUNE=0 disables tuning (the default shapes are used).
#include "engine.hpp"
#include "tsk.hpp"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <sys/stat.h>

namespace dl {

namespace {

std::mutex g_mu;
std::map<std::string, std::pair<WilsonCfg, double>> g_table;
std::map<std::string, std::pair<TskCfg, double>> g_tsk;
bool g_loaded = false;

std::string cache_path() {
  const char* e = std::getenv("DEFLAN_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = std::getenv("HOME");
  return std::string(h && *h ? h : "/tmp") + "/.cache/deflan/tune.txt";
}

std::string arch_name(int device) {
  static std::map<int, std::string> names;  // callers hold g_mu
  auto it = names.find(device);
  if (it != names.end()) return it->second;
  hipDeviceProp_t p;
  std::string a = "unknown";
  if (hipGetDeviceProperties(&p, device) == hipSuccess) {
    a = p.gcnArchName;
    const size_t c = a.find(':');
    if (c != std::string::npos) a = a.substr(0, c);
  }
  names[device] = a;
  return a;
}

std::string make_key(const std::string& arch, const Lattice& lat, int prec, int nrhs) {
  std::ostringstream os;
  os << arch << ' ' << lat.L[0] << 'x' << lat.L[1] << 'x' << lat.L[2] << 'x' << lat.L[3] << ' ' << prec << ' ' << nrhs;
  return os.str();
}

void load_cache() {
  if (g_loaded) return;
  g_loaded = true;
  std::ifstream in(cache_path());
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream is(line);
    std::string arch, dims;
    if (line.compare(0, 2, "K ") == 0) {  // contraction line
      std::string tag;
      int kind, nv, nw, grid, tile;
      long n;
      double us;
      if (!(is >> tag >> arch >> kind >> n >> nv >> nw >> grid >> tile >> us)) continue;
      if (kind < 0 || kind >= TK_COUNT || grid < 1 || tile < 0) continue;
      std::ostringstream k;
      k << arch << ' ' << kind << ' ' << n << ' ' << nv << ' ' << nw;
      g_tsk[k.str()] = {TskCfg{grid, tile}, us};
      continue;
    }
    int prec, nrhs, v, o;
    double us;
    if (!(is >> arch >> dims >> prec >> nrhs >> v >> o >> us)) continue;
    if (v < 0 || v >= kWilsonVariants || o < 0 || o >= kWilsonOrders) continue;
    std::ostringstream k;
    k << arch << ' ' << dims << ' ' << prec << ' ' << nrhs;
    g_table[k.str()] = {WilsonCfg{v, o}, us};
  }
}

void append_line(const std::string& text) {
  const std::string path = cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    // create the directory chain (best effort; an unwritable cache only costs re-tuning)
    std::string dir = path.substr(0, slash);
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') mkdir(dir.substr(0, i).c_str(), 0755);
  }
  std::ofstream out(path, std::ios::app);
  if (out) out << text << '\n';
}

void append_cache(const std::string& key, const WilsonCfg& c, double us) {
  std::ostringstream os;
  os << key << ' ' << c.variant << ' ' << c.order << ' ' << us;
  append_line(os.str());
}

template <class R, class SV>
double time_cfg(dl_op* op, const cplx_t<R>* U, const SV* in, SV* out, int nrhs, WilsonCfg c, int reps,
                hipEvent_t a, hipEvent_t b) {
  hipStream_t s = op->ctx->stream;
  wilson_batched<R>(s, op->lat, U, op->kappa, 2, in, out, op->lat.nc, nrhs, 0, nullptr, nullptr, nullptr, c);
  DL_HIP(hipEventRecord(a, s));
  for (int i = 0; i < reps; ++i)
    wilson_batched<R>(s, op->lat, U, op->kappa, 2, in, out, op->lat.nc, nrhs, 0, nullptr, nullptr, nullptr, c);
  DL_HIP(hipEventRecord(b, s));
  DL_HIP(hipEventSynchronize(b));
  float ms = 0.f;
  DL_HIP(hipEventElapsedTime(&ms, a, b));
  return 1e3 * ms / reps;
}

}  // namespace

bool autotune_enabled() {
  const char* e = std::getenv("DEFLAN_AUTOTUNE");
  return !(e && e[0] == '0');
}

WilsonCfg tune_wilson(dl_op* op, int prec, int nrhs, int reps, double* best_us) {
  op->wcfg.erase(prec * 100000 + nrhs);
  if (op->lat.eo) {  // the even-odd operator has one launch shape
    eo_reserve(op->ctx->stream, (size_t)nrhs * op->lat.nc * (prec == DL_FP64 ? 16 : 8));
    if (best_us) *best_us = 0.0;
    return WilsonCfg{};
  }
  const Lattice& lat = op->lat;
  const long n = (long)nrhs * lat.nc;
  hipEvent_t a, b;
  DL_HIP(hipEventCreate(&a));
  DL_HIP(hipEventCreate(&b));
  WilsonCfg best;
  double best_t = 1e300;
  DBuf<double2> in, out;  // FP64: n double2 each; FP32 uses the first half as float2, BF16 a quarter
  in.alloc(prec == DL_FP64 ? n : (n + 1) / 2);
  out.alloc(prec == DL_FP64 ? n : (n + 1) / 2);
  zero(op->ctx->stream, (long)in.n, in.get());
  for (int v = 0; v < kWilsonVariants; ++v)
    for (int o = 0; o < kWilsonOrders; ++o) {
      if (nrhs == 1 && o == 1) continue;  // identical to order 0 for one rhs
      const WilsonCfg c{v, o};
      if (wilson_nbs(lat, c) > kMaxPartials) continue;  // the fused reductions need the partials
      double t;
      if (prec == DL_FP64)
        t = time_cfg<double>(op, op->U.get(), in.get(), out.get(), nrhs, c, reps, a, b);
      else if (prec == DL_FP32)
        t = time_cfg<float>(op, op_links32_public(op), reinterpret_cast<float2*>(in.get()),
                            reinterpret_cast<float2*>(out.get()), nrhs, c, reps, a, b);
      else
        t = time_cfg<float>(op, op_links32_public(op), reinterpret_cast<bf2*>(in.get()),
                            reinterpret_cast<bf2*>(out.get()), nrhs, c, reps, a, b);
      if (verbose()) {
        std::fprintf(stderr, "[deflan] tune %s nrhs %d variant %d order %d: %.1f us\n",
                     prec == DL_FP64 ? "fp64" : prec == DL_FP32 ? "fp32" : "bf16", nrhs, v, o, t);
        std::fflush(stderr);
      }
      if (t < best_t) {
        best_t = t;
        best = c;
      }
    }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (best_us) *best_us = best_t;
  op->wcfg[prec * 100000 + nrhs] = best;
  std::lock_guard<std::mutex> g(g_mu);
  const std::string key = make_key(arch_name(op->ctx->device), lat, prec, nrhs);
  g_table[key] = {best, best_t};
  append_cache(key, best, best_t);
  return best;
}

WilsonCfg wilson_cfg(dl_op* op, int prec, int nrhs) {
  if (op->lat.eo) {
    // one launch shape; its odd intermediate is sized here, before any graph capture
    eo_reserve(op->ctx->stream, (size_t)nrhs * op->lat.nc * (prec == DL_FP64 ? 16 : 8));
    return WilsonCfg{};
  }
  // DEFLAN_WILSON_VARIANT=v or v,o forces a launch shape (checked on every call)
  if (const char* e = std::getenv("DEFLAN_WILSON_VARIANT")) {
    int v = -1, o = 0;
    if (std::sscanf(e, "%d,%d", &v, &o) >= 1 && v >= 0 && v < kWilsonVariants && o >= 0 && o < kWilsonOrders)
      return WilsonCfg{v, o};
  }
  const int okey = prec * 100000 + nrhs;
  auto oc = op->wcfg.find(okey);
  if (oc != op->wcfg.end()) return oc->second;
  WilsonCfg c;
  bool found = false;
  {
    std::lock_guard<std::mutex> g(g_mu);
    const std::string key = make_key(arch_name(op->ctx->device), op->lat, prec, nrhs);
    load_cache();
    auto it = g_table.find(key);
    if (it != g_table.end()) {
      c = it->second.first;
      found = true;
    }
  }
  if (!found && autotune_enabled()) c = tune_wilson(op, prec, nrhs, 10, nullptr);
  op->wcfg[okey] = c;
  return c;
}

// ---- contraction launch shapes ---------------------------------------------------------
TskCfg tsk_choose(hipStream_t s, int kind, long n, int nv, int nw, const std::vector<TskCfg>& cands,
                  const std::function<void(const TskCfg&)>& launch, int reps, double* best_us) {
  // DEFLAN_TSK_SHAPE=grid,tile forces a shape for every contraction, grid,tile,kind for one kind
  // (checked on every call; the launcher clamps it to what the kernel and the caller's partial
  // buffers allow)
  if (reps <= 0)
    if (const char* e = std::getenv("DEFLAN_TSK_SHAPE")) {
      int g = 0, t = 0, k = -1;
      const int got = std::sscanf(e, "%d,%d,%d", &g, &t, &k);
      if (got == 2 || (got == 3 && k == kind)) return TskCfg{g, t};
    }
  int dev = 0;
  DL_HIP(hipGetDevice(&dev));
  std::string key;
  {
    std::lock_guard<std::mutex> g(g_mu);
    std::ostringstream k;
    k << arch_name(dev) << ' ' << kind << ' ' << n << ' ' << nv << ' ' << nw;
    key = k.str();
    if (reps <= 0) {
      load_cache();
      auto it = g_tsk.find(key);
      if (it != g_tsk.end()) return it->second.first;
    }
  }
  if (reps <= 0) {
    // first use: tune unless disabled or inside a graph capture (timing events cannot be
    // recorded there); the untuned default is then used and not remembered
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    DL_HIP(hipStreamIsCapturing(s, &cs));
    if (!autotune_enabled() || cs != hipStreamCaptureStatusNone) return cands.front();
    reps = 5;
  }
  hipEvent_t a, b;
  DL_HIP(hipEventCreate(&a));
  DL_HIP(hipEventCreate(&b));
  TskCfg best = cands.front();
  double best_t = 1e300;
  try {
    for (const TskCfg& c : cands) {
      launch(c);  // warm-up
      DL_HIP(hipEventRecord(a, s));
      for (int i = 0; i < reps; ++i) launch(c);
      DL_HIP(hipEventRecord(b, s));
      DL_HIP(hipEventSynchronize(b));
      float ms = 0.f;
      DL_HIP(hipEventElapsedTime(&ms, a, b));
      const double t = 1e3 * ms / reps;
      if (verbose()) {
        std::fprintf(stderr, "[deflan] tune contraction %d n %ld nv %d nw %d grid %d tile %d: %.1f us\n", kind, n, nv,
                     nw, c.grid, c.tile, t);
        std::fflush(stderr);
      }
      if (t < best_t) {
        best_t = t;
        best = c;
      }
    }
  } catch (...) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    throw;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (best_us) *best_us = best_t;
  std::lock_guard<std::mutex> g(g_mu);
  g_tsk[key] = {best, best_t};
  std::ostringstream os;
  os << "K " << key << ' ' << best.grid << ' ' << best.tile << ' ' << best_t;
  append_line(os.str());
  return best;
}

}  // namespace dl
