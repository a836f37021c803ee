// Runtime support: errors, device memory, lattice geometry, kernel timers.
#include "internal.hpp"

#include <cstdio>
#include <map>
#include <mutex>
#include <stdexcept>
#include <unordered_map>
#include <vector>

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

// Device memory is cached per device: a freed block goes to a free list keyed by its
// (rounded) size and is handed out again by the next request of that size, so repeated
// solves of one shape map no new memory.  Sizes round to 512 B, and to 2 MiB from 1 MiB up.
// A block is cached only after a device-wide synchronisation (what hipFree implies), so a
// block never changes hands while a kernel on any stream may still use it.  The cache holds
// at most an eighth of the device's memory; an allocation that fails releases the device's
// cache and tries once more; dmem_trim releases it on request (context destruction).
namespace {
struct Block {
  int dev;
  size_t bytes;
};
struct MemCache {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<void*>> free_list;
  std::unordered_map<void*, Block> live;
  std::map<int, size_t> cached, cap;
};
MemCache& mem_cache() {
  static MemCache* c = new MemCache;  // never destroyed: blocks may be returned during exit
  return *c;
}
size_t round_bytes(size_t b) {
  const size_t g = b >= (size_t(1) << 20) ? (size_t(1) << 21) : 512;
  return (b + g - 1) / g * g;
}
void trim_locked(MemCache& c, int dev) {
  for (auto it = c.free_list.begin(); it != c.free_list.end();) {
    if (it->first.first == dev) {
      for (void* p : it->second) (void)hipFree(p);
      it = c.free_list.erase(it);
    } else {
      ++it;
    }
  }
  c.cached[dev] = 0;
}
}  // namespace

void* dmalloc(size_t bytes) {
  int dev = 0;
  DL_HIP(hipGetDevice(&dev));
  const size_t rb = round_bytes(bytes);
  MemCache& c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.free_list.find({dev, rb});
  if (it != c.free_list.end() && !it->second.empty()) {
    void* p = it->second.back();
    it->second.pop_back();
    c.cached[dev] -= rb;
    c.live[p] = Block{dev, rb};
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, rb);
  if (e == hipErrorOutOfMemory && c.cached[dev] > 0) {
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
    trim_locked(c, dev);
    e = hipMalloc(&p, rb);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    char buf[256];
    std::snprintf(buf, sizeof buf, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    fail(e == hipErrorOutOfMemory ? DL_E_NOMEM : DL_E_HIP, buf);
  }
  c.live[p] = Block{dev, rb};
  return p;
}

void dfree(void* p) {
  if (!p) return;
  MemCache& c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.live.find(p);
  if (it == c.live.end()) {  // not ours
    (void)hipFree(p);
    return;
  }
  const Block b = it->second;
  c.live.erase(it);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != b.dev) (void)hipSetDevice(b.dev);
  if (!c.cap.count(b.dev)) {
    size_t fr = 0, tot = 0;
    c.cap[b.dev] = hipMemGetInfo(&fr, &tot) == hipSuccess ? tot / 8 : 0;
  }
  if (hipDeviceSynchronize() == hipSuccess && c.cached[b.dev] + b.bytes <= c.cap[b.dev]) {
    c.free_list[{b.dev, b.bytes}].push_back(p);
    c.cached[b.dev] += b.bytes;
  } else {
    (void)hipFree(p);
  }
  if (cur != b.dev) (void)hipSetDevice(cur);
}

void dmem_trim(int dev) {
  MemCache& c = mem_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != dev) (void)hipSetDevice(dev);
  (void)hipDeviceSynchronize();
  trim_locked(c, dev);
  if (cur != dev) (void)hipSetDevice(cur);
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

Lattice make_lattice_eo(const int dims[4]) {
  Lattice lat = make_lattice(dims);
  for (int i = 0; i < 4; ++i)
    if (dims[i] % 2) fail(DL_E_INVALID, "the even-odd operator needs every lattice extent even");
  lat.eo = 1;
  lat.V /= 2;
  lat.ntiles = (lat.V + kTile - 1) / kTile;
  lat.nc = lat.ntiles * kTile * kSpin;  // nl (the whole lattice's links) is kept
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
