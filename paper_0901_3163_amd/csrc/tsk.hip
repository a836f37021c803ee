// Tall-skinny contractions of the Lanczos basis with vectors (FP64).
//
//   dots:    c = V^H w                (re-orthogonalisation, deflation projection)
//   update:  w <- w + sgn * V c       (complex coefficients from device memory)
//   combine: Y_l = sum_j G[j][l] V_j  (real G: Ritz / harmonic-Ritz rebuild, x += V d)
//
// V is a set of nv fields addressed as base + slot[j] * ld (slot == nullptr
// means slot[j] = j), so that a restart can rebuild the basis out of place and
// permute slots without moving data.  These kernels stream V once per call and
// are HBM-bound: V^H w reads nv+1 vectors and writes nothing but partials.
#include "internal.hpp"
#include "cplx.hpp"
#include "tsk.hpp"

namespace dl {

constexpr int kEPT = 8;        // elements of w cached per thread in the dots kernel
constexpr int kMaxNV = 512;    // basis vectors per call

int tsk_nblocks(long n) {
  long nb = (n + (long)kBlock * kEPT - 1) / ((long)kBlock * kEPT);
  if (nb < 1) nb = 1;
  if (nb > kMaxPartials) fail(DL_E_INVALID, "vector too long for the tall-skinny reduction");
  return (int)nb;
}

__device__ __forceinline__ const double2* vec_at(const double2* base, long ld, const int* slot, int j) {
  return base + (long)(slot ? slot[j] : j) * ld;
}

// part is column-major [2*nv][gridDim.x]: Re/Im of <V_j, w> partial of this block.
__global__ void __launch_bounds__(kBlock)
k_tsk_dots(long n, int nv, const double2* __restrict__ base, long ld, const int* __restrict__ slot,
           const double2* __restrict__ w, double* __restrict__ part) {
  __shared__ double2 lds[kBlock / 64][kMaxNV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const long stride = (long)gridDim.x * kBlock;
  const long i0 = (long)blockIdx.x * kBlock + threadIdx.x;
  double2 wr[kEPT];
#pragma unroll
  for (int r = 0; r < kEPT; ++r) {
    const long i = i0 + r * stride;
    wr[r] = i < n ? w[i] : make_double2(0.0, 0.0);
  }
  for (int j = 0; j < nv; ++j) {
    const double2* v = vec_at(base, ld, slot, j);
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int r = 0; r < kEPT; ++r) {
      const long i = i0 + r * stride;
      if (i < n) {
        const double2 x = v[i];
        re = fma(x.x, wr[r].x, re);
        re = fma(x.y, wr[r].y, re);
        im = fma(x.x, wr[r].y, im);
        im = fma(-x.y, wr[r].x, im);
      }
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) lds[wid][j] = make_double2(re, im);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nv; j += kBlock) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) {
      re += lds[q][j].x;
      im += lds[q][j].y;
    }
    part[(long)(2 * j) * gridDim.x + blockIdx.x] = re;
    part[(long)(2 * j + 1) * gridDim.x + blockIdx.x] = im;
  }
}

// w += sgn * sum_j c_j V_j ; c complex (interleaved) in device memory.
__global__ void __launch_bounds__(kBlock)
k_tsk_update(long n, int nv, const double2* __restrict__ base, long ld, const int* __restrict__ slot,
             const double2* __restrict__ c, double sgn, double2* __restrict__ w) {
  __shared__ double2 cs[kMaxNV];
  for (int j = threadIdx.x; j < nv; j += kBlock) cs[j] = make_double2(sgn * c[j].x, sgn * c[j].y);
  __syncthreads();
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double2 acc = w[i];
    for (int j = 0; j < nv; ++j) acc = c_fma(cs[j], vec_at(base, ld, slot, j)[i], acc);
    w[i] = acc;
  }
}

// Y_l (+)= sum_j G[j * ldg + l] V_j for l in [l0, l0 + kNY) ; G real.
constexpr int kNY = 8;
__global__ void __launch_bounds__(kBlock)
k_tsk_combine(long n, int nv, const double2* __restrict__ base, long ld, const int* __restrict__ slot,
              const double* __restrict__ G, int ldg, int ny, double2* __restrict__ obase, long old,
              const int* __restrict__ oslot, int accumulate) {
  const int l0 = blockIdx.y * kNY;
  const int nl = min(kNY, ny - l0);
  __shared__ double gs[kMaxNV][kNY];
  for (int t = threadIdx.x; t < nv * kNY; t += kBlock) {
    const int j = t / kNY, l = t % kNY;
    gs[j][l] = l < nl ? G[(long)j * ldg + l0 + l] : 0.0;
  }
  __syncthreads();
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double2 acc[kNY];
#pragma unroll
    for (int l = 0; l < kNY; ++l) acc[l] = make_double2(0.0, 0.0);
    for (int j = 0; j < nv; ++j) {
      const double2 x = vec_at(base, ld, slot, j)[i];
#pragma unroll
      for (int l = 0; l < kNY; ++l) acc[l] = c_axpy(gs[j][l], x, acc[l]);
    }
#pragma unroll
    for (int l = 0; l < kNY; ++l) {
      if (l < nl) {
        double2* y = obase + (long)(oslot ? oslot[l0 + l] : l0 + l) * old;
        y[i] = accumulate ? c_add(y[i], acc[l]) : acc[l];
      }
    }
  }
}

static int stream_blocks(long n) {
  long nb = (n + kBlock - 1) / kBlock;
  if (nb > 2048) nb = 2048;
  if (nb < 1) nb = 1;
  return (int)nb;
}

int tsk_dots(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
             const double2* w, double* part) {
  if (nv > kMaxNV) fail(DL_E_INVALID, "too many basis vectors (max 512)");
  const int nb = tsk_nblocks(n);
  if (nv > 0) {
    hipLaunchKernelGGL(k_tsk_dots, dim3(nb), dim3(kBlock), 0, s, n, nv, base, ld, slot, w, part);
    DL_HIP(hipGetLastError());
  }
  return nb;
}

void tsk_update(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                const double2* c, double sgn, double2* w) {
  if (nv > kMaxNV) fail(DL_E_INVALID, "too many basis vectors (max 512)");
  if (nv <= 0) return;
  hipLaunchKernelGGL(k_tsk_update, dim3(stream_blocks(n)), dim3(kBlock), 0, s, n, nv, base, ld, slot, c, sgn, w);
  DL_HIP(hipGetLastError());
}

void tsk_combine(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                 const double* G, int ldg, int ny, double2* obase, long old, const int* oslot,
                 int accumulate) {
  if (nv > kMaxNV) fail(DL_E_INVALID, "too many basis vectors (max 512)");
  if (nv <= 0 || ny <= 0) return;
  const dim3 grid(stream_blocks(n), (ny + kNY - 1) / kNY);
  hipLaunchKernelGGL(k_tsk_combine, grid, dim3(kBlock), 0, s, n, nv, base, ld, slot, G, ldg, ny, obase, old,
                     oslot, accumulate);
  DL_HIP(hipGetLastError());
}

}  // namespace dl
