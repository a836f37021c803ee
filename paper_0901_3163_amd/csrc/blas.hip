// Layout conversion and BLAS-1 kernels with deterministic two-stage reductions.
//
// Reductions: each block of 256 threads reduces its grid-stride share with a
// wavefront shuffle tree and writes one partial per block; a second kernel sums
// the partials of each column in a fixed order.  The number of blocks depends
// only on the vector length, so results are bitwise reproducible.
#include "internal.hpp"
#include "cplx.hpp"

namespace dl {

// ---- layout ----------------------------------------------------------------
__global__ void k_pack_spinor(const double2* __restrict__ in, double2* __restrict__ out, long V, long nc) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long f = blockIdx.y;
  if (i >= V * kSpin) return;
  const long site = i / kSpin;
  const int c = (int)(i % kSpin);
  out[f * nc + ((site >> 6) * kSpin + c) * kTile + (site & 63)] = in[f * V * kSpin + i];
}

__global__ void k_unpack_spinor(const double2* __restrict__ in, double2* __restrict__ out, long V, long nc) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long f = blockIdx.y;
  if (i >= V * kSpin) return;
  const long site = i / kSpin;
  const int c = (int)(i % kSpin);
  out[f * V * kSpin + i] = in[f * nc + ((site >> 6) * kSpin + c) * kTile + (site & 63)];
}

__global__ void k_pack_links(const double2* __restrict__ in, double2* __restrict__ out, long V) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= V * kLinkC) return;
  const long site = i / kLinkC;
  const int c = (int)(i % kLinkC);
  out[((site >> 6) * kLinkC + c) * kTile + (site & 63)] = in[i];
}

void pack_spinor(hipStream_t s, const Lattice& lat, const double2* in, double2* out, int nfield) {
  if (nfield <= 0) return;
  const long n = lat.V * kSpin;
  hipLaunchKernelGGL(k_pack_spinor, dim3((n + 255) / 256, nfield), dim3(256), 0, s, in, out, lat.V, lat.nc);
  DL_HIP(hipGetLastError());
}

void unpack_spinor(hipStream_t s, const Lattice& lat, const double2* in, double2* out, int nfield) {
  if (nfield <= 0) return;
  const long n = lat.V * kSpin;
  hipLaunchKernelGGL(k_unpack_spinor, dim3((n + 255) / 256, nfield), dim3(256), 0, s, in, out, lat.V, lat.nc);
  DL_HIP(hipGetLastError());
}

void pack_links(hipStream_t s, const Lattice& lat, const double2* in, double2* out) {
  const long n = lat.V * kLinkC;
  hipLaunchKernelGGL(k_pack_links, dim3((n + 255) / 256), dim3(256), 0, s, in, out, lat.V);
  DL_HIP(hipGetLastError());
}

// ---- streaming reductions -----------------------------------------------------
int nblocks_for(long n) {
  long nb = (n + 4 * kBlock - 1) / (4 * kBlock);
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  return (int)nb;
}

__global__ void __launch_bounds__(kBlock)
k_dot_partials(long n, const double2* __restrict__ a, const double2* __restrict__ b, double* __restrict__ part) {
  double re = 0.0, im = 0.0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const double2 x = a[i], y = b[i];
    re = fma(x.x, y.x, re);
    re = fma(x.y, y.y, re);
    im = fma(x.x, y.y, im);
    im = fma(-x.y, y.x, im);
  }
  __shared__ double lds[kBlock / 64];
  const double sr = block_sum<kBlock>(re, lds);
  const double si = block_sum<kBlock>(im, lds);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sr;
    part[gridDim.x + blockIdx.x] = si;
  }
}

__global__ void __launch_bounds__(kBlock)
k_norm2_partials(long n, const double2* __restrict__ a, double* __restrict__ part) {
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const double2 x = a[i];
    acc = fma(x.x, x.x, acc);
    acc = fma(x.y, x.y, acc);
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

int dot_partials(hipStream_t s, long n, const double2* a, const double2* b, double* part) {
  const int nb = nblocks_for(n);
  hipLaunchKernelGGL(k_dot_partials, dim3(nb), dim3(kBlock), 0, s, n, a, b, part);
  DL_HIP(hipGetLastError());
  return nb;
}

int norm2_partials(hipStream_t s, long n, const double2* a, double* part) {
  const int nb = nblocks_for(n);
  hipLaunchKernelGGL(k_norm2_partials, dim3(nb), dim3(kBlock), 0, s, n, a, part);
  DL_HIP(hipGetLastError());
  return nb;
}

__global__ void __launch_bounds__(kBlock)
k_sum_partials(const double* __restrict__ part, int nparts, int width, double* __restrict__ out) {
  const int col = blockIdx.x;
  double acc = 0.0;
  const double* p = part + (long)col * nparts;
  for (int i = threadIdx.x; i < nparts; i += kBlock) acc += p[i];
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) out[col] = s;
}

void sum_partials(hipStream_t s, const double* part, int nparts, int width, double* out) {
  hipLaunchKernelGGL(k_sum_partials, dim3(width), dim3(kBlock), 0, s, part, nparts, width, out);
  DL_HIP(hipGetLastError());
}

// ---- elementwise -------------------------------------------------------------
__global__ void k_copy(long n, const double2* __restrict__ a, double2* __restrict__ b) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}
__global__ void k_zero(long n, double2* __restrict__ a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = make_double2(0.0, 0.0);
}

void copy(hipStream_t s, long n, const double2* a, double2* b) {
  hipLaunchKernelGGL(k_copy, dim3((n + 255) / 256), dim3(256), 0, s, n, a, b);
  DL_HIP(hipGetLastError());
}
void zero(hipStream_t s, long n, double2* a) {
  hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, s, n, a);
  DL_HIP(hipGetLastError());
}

__global__ void k_round_f32(long n, const double2* __restrict__ a, float2* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = make_float2((float)a[i].x, (float)a[i].y);
}
__global__ void k_widen_f64(long n, const float2* __restrict__ a, double2* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = make_double2(a[i].x, a[i].y);
}

__global__ void k_round_bf16(long n, const double2* __restrict__ a, bf2* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    sst(b + i, make_float2((float)a[i].x, (float)a[i].y));
}
__global__ void k_widen_bf16(long n, const bf2* __restrict__ a, double2* __restrict__ b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float2 v = sld(a + i);
    b[i] = make_double2(v.x, v.y);
  }
}
void round_bf16(hipStream_t s, long n, const double2* a, bf2* b) {
  hipLaunchKernelGGL(k_round_bf16, dim3(2048), dim3(256), 0, s, n, a, b);
  DL_HIP(hipGetLastError());
}
void widen_bf16(hipStream_t s, long n, const bf2* a, double2* b) {
  hipLaunchKernelGGL(k_widen_bf16, dim3(2048), dim3(256), 0, s, n, a, b);
  DL_HIP(hipGetLastError());
}

void round_f32(hipStream_t s, long n, const double2* a, float2* b) {
  hipLaunchKernelGGL(k_round_f32, dim3(2048), dim3(256), 0, s, n, a, b);
  DL_HIP(hipGetLastError());
}
void widen_f64(hipStream_t s, long n, const float2* a, double2* b) {
  hipLaunchKernelGGL(k_widen_f64, dim3(2048), dim3(256), 0, s, n, a, b);
  DL_HIP(hipGetLastError());
}

}  // namespace dl

namespace dl {

// splitmix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) as the per-element mixer
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) k_field_hash(long n, const double2* __restrict__ a, uint64_t* part) {
  uint64_t acc = 0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const double2 v = a[i];
    const uint64_t re = (uint64_t)__double_as_longlong(v.x), im = (uint64_t)__double_as_longlong(v.y);
    acc += mix64(re ^ mix64(2 * (uint64_t)i + 1)) + mix64(im ^ mix64(2 * (uint64_t)i + 2));
  }
  __shared__ uint64_t lds[256];
  lds[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

uint64_t field_hash(hipStream_t s, long n, const double2* a) {
  constexpr int kParts = 1024;
  DBuf<uint64_t> part(kParts);
  hipLaunchKernelGGL(k_field_hash, dim3(kParts), dim3(256), 0, s, n, a, part.get());
  DL_HIP(hipGetLastError());
  std::vector<uint64_t> h(kParts);
  DL_HIP(hipMemcpyAsync(h.data(), part.get(), kParts * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  DL_HIP(hipStreamSynchronize(s));
  uint64_t t = 0;
  for (uint64_t v : h) t += v;
  return t;
}

}  // namespace dl
