// The projection c = V^H w (and w <- w - V c) for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
// kernels as dl_tsk_project, with the reduction partials in a fixed device array of this
// library instead of a buffer allocated per call.
//
// The array `scratch` below exists once per device the library runs on (every GPU holds its
// own copy from module load until the process ends).  Host code never passes the array's name
// to a kernel: on the host it is only a stand-in symbol, so its device address is looked up
// once per device with hipGetSymbolAddress when a context is created, and that address is what
// the kernels receive.
#include "internal.hpp"
#include "tsk.hpp"

#include <mutex>

namespace dl {

// Partials of the dots: 2 * nv * nblocks doubles (nblocks = n / 2048 rounded up), at most
// kNoAllocDoubles (8 MiB).  At 16^3 x 32 (n = 1572864, 768 blocks) that covers nv <= 512, at
// 24^3 x 48 (n = 7962624) nv <= 134.
constexpr long kNoAllocDoubles = 1L << 20;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {nullptr};
}  // namespace

// Looks up the device address of `scratch` on `device` (which must be current) once.
void noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) fail(DL_E_INVALID, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return;
  void* p = nullptr;
  DL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) fail(DL_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
  g_ptr[device] = static_cast<double*>(p);
}

static double* noalloc_ptr(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  double* p = (device >= 0 && device < kMaxDevices) ? g_ptr[device] : nullptr;
  if (!p) fail(DL_E_INVALID, "no scratch address for this device (context not created)");
  return p;
}

int tsk_project_noalloc(dl_ctx* ctx, long n, int nv, const double2* V, double2* w, double2* c, int subtract) {
  const long nb = (long)tsk_nblocks(n);
  if (2L * nv * nb > kNoAllocDoubles)
    fail(DL_E_INVALID, "n * nv too large for the fixed scratch array: 2 * nv * ceil(n / 2048) must be <= 1048576");
  double* part = noalloc_ptr(ctx->device);
  hipStream_t s = ctx->stream;
  const int np = tsk_dots(s, n, nv, V, n, nullptr, w, part);
  sum_partials(s, part, np, 2 * nv, reinterpret_cast<double*>(c));
  if (subtract) tsk_update(s, n, nv, V, n, nullptr, c, -1.0, w);
  DL_HIP(hipGetLastError());
  return DL_OK;
}

}  // namespace dl
