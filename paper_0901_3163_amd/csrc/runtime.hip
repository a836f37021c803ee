// Runtime support: errors, device memory, lattice geometry, kernel timers.
#include "internal.hpp"

#include <cstdio>
#include <stdexcept>

namespace dl {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
const std::string& last_error() { return g_last_error; }

[[noreturn]] void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  char buf[512];
  std::snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  fail(e == hipErrorOutOfMemory ? DL_E_NOMEM : DL_E_HIP, buf);
}

void* dmalloc(size_t bytes) {
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    fail(e == hipErrorOutOfMemory ? DL_E_NOMEM : DL_E_HIP, buf);
  }
  return p;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

Lattice make_lattice(const int dims[4]) {
  Lattice lat{};
  lat.V = 1;
  for (int i = 0; i < 4; ++i) {
    if (dims[i] < 2 || dims[i] > 4096) fail(DL_E_INVALID, "each lattice extent must be in [2, 4096]");
    lat.L[i] = dims[i];
    lat.V *= dims[i];
  }
  lat.ntiles = (lat.V + kTile - 1) / kTile;
  lat.nc = lat.ntiles * kTile * kSpin;
  lat.nl = lat.ntiles * kTile * kLinkC;
  return lat;
}

hipEvent_t Timers::take() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  DL_HIP(hipEventCreate(&e));
  return e;
}

void Timers::begin(hipStream_t s, int id, hipEvent_t* a) {
  (void)id;
  *a = take();
  DL_HIP(hipEventRecord(*a, s));
}

void Timers::end(hipStream_t s, int id, hipEvent_t a, double nbytes) {
  hipEvent_t b = take();
  DL_HIP(hipEventRecord(b, s));
  pending.push_back({a, b, id, nbytes});
  if (pending.size() > 4096) collect();
}

void Timers::collect() {
  for (auto& p : pending) {
    DL_HIP(hipEventSynchronize(p.b));
    float ms_ = 0.f;
    DL_HIP(hipEventElapsedTime(&ms_, p.a, p.b));
    launches[p.id] += 1;
    ms[p.id] += ms_;
    bytes[p.id] += p.bytes;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void Timers::reset() {
  collect();
  for (int i = 0; i < T_COUNT; ++i) {
    launches[i] = 0;
    ms[i] = 0.0;
    bytes[i] = 0.0;
  }
}

Timers::~Timers() {
  for (auto& p : pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace dl
