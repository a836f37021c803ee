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

#include <algorithm>
#include <map>
#include <mutex>

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

// part is column-major [2*nv][gridDim.x]: Re/Im of <V_j, w> partial of this block; with_norm
// adds column 2*nv, the block's partial of ||w||^2 (w is in registers already).  gate: when
// non-null and *gate == 0, the pass is skipped and the block writes zero partials.
__global__ void __launch_bounds__(kBlock)
k_tsk_dots(long n, int nv, const double2* __restrict__ base, long ld, const int* __restrict__ slot,
           const double2* __restrict__ w, double* __restrict__ part, const double* __restrict__ gate,
           int with_norm) {
  __shared__ double2 lds[kBlock / 64][kMaxNV + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ncol = nv + (with_norm ? 1 : 0);
  if (gate && *gate == 0.0) {
    for (int j = threadIdx.x; j < 2 * ncol; j += kBlock) part[(long)j * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
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
  if (with_norm) {
    double nn = 0.0;
#pragma unroll
    for (int r = 0; r < kEPT; ++r) nn = fma(wr[r].x, wr[r].x, fma(wr[r].y, wr[r].y, nn));
    nn = wave_sum(nn);
    if (lane == 0) lds[wid][nv] = make_double2(nn, 0.0);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < ncol; j += kBlock) {
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
             const double2* __restrict__ c, double sgn, double2* __restrict__ w, const double* __restrict__ gate) {
  if (gate && *gate == 0.0) return;
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

// Y_l (+)= sum_j G[j * ldg + l] V_j for l in [l0, l0 + NY) ; G real.  Block (bx, by) covers
// rows bx, bx + nbx, ... of outputs [by * NY, by * NY + NY).  xcd = 0: a 2-D grid (bx, by);
// xcd = 1: a 1-D grid of nbx * nby blocks (nbx a multiple of 8) numbered so that the nby blocks
// of one row range are consecutive on one XCD (hardware places block L on XCD L % 8), where they
// read the same rows of V through that XCD's L2 instead of each from HBM.
template <int NY>
__global__ void __launch_bounds__(kBlock)
k_tsk_combine(long n, int nv, const double2* __restrict__ base, long ld, const int* __restrict__ slot,
              const double* __restrict__ G, int ldg, int ny, double2* __restrict__ obase, long old,
              const int* __restrict__ oslot, int accumulate, int nbx, int nby, int xcd) {
  int bx, by;
  if (xcd) {
    const int q = blockIdx.x >> 3;
    by = q % nby;
    bx = (q / nby) * 8 + (blockIdx.x & 7);
  } else {
    bx = blockIdx.x;
    by = blockIdx.y;
  }
  const int l0 = by * NY;
  const int nl = min(NY, ny - l0);
  __shared__ double gs[NY == 8 ? kMaxNV : kMaxNV / 2][NY];
  for (int t = threadIdx.x; t < nv * NY; t += kBlock) {
    const int j = t / NY, l = t % NY;
    gs[j][l] = l < nl ? G[(long)j * ldg + l0 + l] : 0.0;
  }
  __syncthreads();
  const long stride = (long)nbx * kBlock;
  for (long i = (long)bx * kBlock + threadIdx.x; i < n; i += stride) {
    double2 acc[NY];
#pragma unroll
    for (int l = 0; l < NY; ++l) acc[l] = make_double2(0.0, 0.0);
    for (int j = 0; j < nv; ++j) {
      const double2 x = vec_at(base, ld, slot, j)[i];
#pragma unroll
      for (int l = 0; l < NY; ++l) acc[l] = c_axpy(gs[j][l], x, acc[l]);
    }
#pragma unroll
    for (int l = 0; l < NY; ++l) {
      if (l < nl) {
        double2* y = obase + (long)(oslot ? oslot[l0 + l] : l0 + l) * old;
        y[i] = accumulate ? c_add(y[i], acc[l]) : acc[l];
      }
    }
  }
}

// ---- several right-hand sides at once: C = V^H W and X += V D ---------------------------
// W and X hold nw fields at stride ldw (nw <= NW).  V streams once for all nw columns.
constexpr int kMultiNV = 64; // basis vectors per multi-column dots call
constexpr int kLpMaxNV = 128; // basis vectors per low-precision dots call
constexpr int kMultiBlocks = 2048;

// C = V^H W as a tiled product: a block stages a 64-row tile of 32 basis vectors and of up
// to 16 columns in LDS (coalesced 1 KiB runs), then each thread accumulates a 4 x 4 block of
// (vector, column) products over 8 of the tile's rows; the 8 row groups are added in LDS at
// the end (fixed order).  Vectors [j0, j0 + nj) of nv, columns r < nw.  part is column-major
// [2*nw*nv][gridDim.x]: column (r*nv + j)*2 (+1) holds Re (Im) of the block's share of
// <V_j, W_r>, so the summed result is c[r*nv + j] (rhs-major).
constexpr int kTR = 64, kTJ = 32, kTW = 16;
__global__ void __launch_bounds__(kBlock)
k_tsk_dots_multi(long n, int nv, int j0, int nj, const double2* __restrict__ base, long ld,
                 const double2* __restrict__ W, long ldw, int nw, const int* __restrict__ active,
                 double* __restrict__ part) {
  // one buffer: the V tile (kTJ rows of kTR + 1), the W tile after it, and later the reduction
  __shared__ double2 sm[(kTJ + kTW) * (kTR + 1)];
  double2 (*vt)[kTR + 1] = reinterpret_cast<double2 (*)[kTR + 1]>(sm);
  double2 (*wt)[kTR + 1] = reinterpret_cast<double2 (*)[kTR + 1]>(sm + kTJ * (kTR + 1));
  const int tid = threadIdx.x;
  const int mt = tid & 31, rg = tid >> 5;   // micro tile (8 j-groups x 4 r-groups), row group 0..7
  const int jq = (mt & 7) * 4, rq = (mt >> 3) * 4;
  double2 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = make_double2(0.0, 0.0);
  const long ntiles = (n + kTR - 1) / kTR;
  for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long r0 = tile * kTR;
    __syncthreads();
    for (int e = tid; e < kTJ * kTR; e += kBlock) {
      const int j = e / kTR, row = e % kTR;
      const long i = r0 + row;
      vt[j][row] = (j < nj && i < n) ? base[(long)(j0 + j) * ld + i] : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < kTW * kTR; e += kBlock) {
      const int r = e / kTR, row = e % kTR;
      const long i = r0 + row;
      const bool on = r < nw && i < n && (!active || active[r]);
      wt[r][row] = on ? W[(long)r * ldw + i] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 2
    for (int row = rg; row < kTR; row += 8) {
      double2 v[4], w[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) v[a] = vt[jq + a][row];
#pragma unroll
      for (int b = 0; b < 4; ++b) w[b] = wt[rq + b][row];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          // conj(v) * w
          acc[a][b].x = fma(v[a].x, w[b].x, acc[a][b].x);
          acc[a][b].x = fma(v[a].y, w[b].y, acc[a][b].x);
          acc[a][b].y = fma(v[a].x, w[b].y, acc[a][b].y);
          acc[a][b].y = fma(-v[a].y, w[b].x, acc[a][b].y);
        }
    }
  }
  // add the 8 row groups in two halves of 16 vectors: each row group writes its sums for the
  // half to red[g][256], then 256 threads add the 8 groups (fixed order)
  double2* red = sm;
  static_assert((kTJ + kTW) * (kTR + 1) >= 8 * 256, "reduction buffer");
  for (int half = 0; half < 2; ++half) {
    __syncthreads();
    if ((jq >> 4) == half) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) red[rg * 256 + (jq - 16 * half + a) * 16 + rq + b] = acc[a][b];
    }
    __syncthreads();
    const int t = tid;  // 256 (j, r) sums of this half
    const int j = 16 * half + t / 16, r = t % 16;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      re += red[g * 256 + t].x;
      im += red[g * 256 + t].y;
    }
    if (j < nj && r < nw) {
      const long col = 2L * (r * nv + j0 + j);
      part[col * gridDim.x + blockIdx.x] = re;
      part[(col + 1) * gridDim.x + blockIdx.x] = im;
    }
  }
}

__device__ __forceinline__ double2 widen2(double2 a) { return a; }
__device__ __forceinline__ double2 widen2(float2 a) { return make_double2(a.x, a.y); }

// X_r += sum_j D[r*ldd + j] V_j for active r < nw (D complex, rhs-major, device memory).  The
// basis is FP64 or FP32 (VB); the products and sums are FP64 either way.
template <int NW, class VB>
__global__ void __launch_bounds__(kBlock)
k_tsk_update_multi(long n, int nv, const VB* __restrict__ base, long ld, const double2* __restrict__ D, int ldd,
                   int nw, const int* __restrict__ active, double2* __restrict__ X, long ldx) {
  __shared__ double2 ds[kMaxNV / 4][NW];  // nv <= 128
  for (int t = threadIdx.x; t < nv * NW; t += kBlock) {
    const int j = t / NW, r = t % NW;
    ds[j][r] = r < nw ? D[(long)r * ldd + j] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const long stride = (long)gridDim.x * kBlock;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    double2 acc[NW];
#pragma unroll
    for (int r = 0; r < NW; ++r) acc[r] = make_double2(0.0, 0.0);
    for (int j = 0; j < nv; ++j) {
      const double2 x = widen2(base[(long)j * ld + i]);
#pragma unroll
      for (int r = 0; r < NW; ++r) acc[r] = c_fma(ds[j][r], x, acc[r]);
    }
#pragma unroll
    for (int r = 0; r < NW; ++r)
      if (r < nw && (!active || active[r])) X[(long)r * ldx + i] = c_add(X[(long)r * ldx + i], acc[r]);
  }
}

// One thread per element up to 8192 blocks: the largest grid the grid-stride kernels are tuned over.
static int max_stream_blocks(long n) {
  long nb = (n + kBlock - 1) / kBlock;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  return (int)nb;
}

// tsk_tune's request to re-time the next key, and what the launcher chose.
namespace {
struct TuneReq {
  int reps = 0;
  double us = 0.0;
  TskCfg cfg;
};
thread_local TuneReq t_tune;
}  // namespace

static TskCfg choose(hipStream_t s, int kind, long n, int nv, int nw, const std::vector<TskCfg>& cands,
                     const std::function<void(const TskCfg&)>& launch) {
  const TskCfg c = tsk_choose(s, kind, n, nv, nw, cands, launch, t_tune.reps, &t_tune.us);
  t_tune.cfg = c;
  return c;
}

static int stream_blocks(long n) {
  long nb = (n + kBlock - 1) / kBlock;
  if (nb > 2048) nb = 2048;
  if (nb < 1) nb = 1;
  return (int)nb;
}

int tsk_dots(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
             const double2* w, double* part, const double* gate, int with_norm) {
  if (nv > kMaxNV) fail(DL_E_INVALID, "too many basis vectors (max 512)");
  const int nb = tsk_nblocks(n);
  if (nv > 0 || with_norm) {
    hipLaunchKernelGGL(k_tsk_dots, dim3(nb), dim3(kBlock), 0, s, n, nv, base, ld, slot, w, part, gate, with_norm);
    DL_HIP(hipGetLastError());
  }
  return nb;
}

void tsk_update(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                const double2* c, double sgn, double2* w, const double* gate) {
  if (nv > kMaxNV) fail(DL_E_INVALID, "too many basis vectors (max 512)");
  if (nv <= 0) return;
  hipLaunchKernelGGL(k_tsk_update, dim3(stream_blocks(n)), dim3(kBlock), 0, s, n, nv, base, ld, slot, c, sgn, w,
                     gate);
  DL_HIP(hipGetLastError());
}

// gate = 1 if the first Gram-Schmidt pass removed more than the DGKS share of w, that is
// ||c||^2 > (1 - eta^2) ||w||^2 with ||w - V c||^2 = ||w||^2 - ||c||^2 for orthonormal V, else 0.
__global__ void k_dgks_gate(const double* __restrict__ c, int nv, const double* __restrict__ wn2, double eta2,
                            double* __restrict__ gate) {
  double cc = 0.0;
  for (int j = threadIdx.x; j < 2 * nv; j += blockDim.x) cc = fma(c[j], c[j], cc);
  cc = wave_sum(cc);  // one wave
  if (threadIdx.x == 0) *gate = cc > (1.0 - eta2) * *wn2 ? 1.0 : 0.0;
}

void tsk_dgks_gate(hipStream_t s, const double* c, int nv, const double* wn2, double eta2, double* gate) {
  hipLaunchKernelGGL(k_dgks_gate, dim3(1), dim3(64), 0, s, c, nv, wn2, eta2, gate);
  DL_HIP(hipGetLastError());
}

// Zero-filled device doubles (at least ndouble) for timing read-modify-write launches with no
// effect (x + 0 = x): one buffer per device that only grows, kept until the process ends (filled
// and synchronised before first use; timing happens outside graph capture).
static const double2* zeros(hipStream_t s, size_t ndouble) {
  static std::mutex mu;
  static std::map<int, std::pair<double2*, size_t>> bufs;
  int dev = 0;
  DL_HIP(hipGetDevice(&dev));
  const size_t n2 = (ndouble + 1) / 2;
  std::lock_guard<std::mutex> g(mu);
  auto& b = bufs[dev];
  if (b.second < n2) {
    if (b.first) {
      DL_HIP(hipStreamSynchronize(s));
      DL_HIP(hipFree(b.first));
      b.first = nullptr;
      b.second = 0;
    }
    void* p = nullptr;
    DL_HIP(hipMalloc(&p, n2 * sizeof(double2)));
    b.first = static_cast<double2*>(p);
    b.second = n2;
    zero(s, (long)n2, b.first);
    DL_HIP(hipStreamSynchronize(s));
  }
  return b.first;
}

static void combine_launch(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                           const double* G, int ldg, int ny, double2* obase, long old, const int* oslot,
                           int accumulate, const TskCfg& c) {
  const int ny_per = (c.tile & 2) ? 16 : 8;
  const int xcd = c.tile & 1;
  const int nby = (ny + ny_per - 1) / ny_per;
  int nbx = c.grid;
  if (xcd) nbx = (nbx + 7) / 8 * 8;
  const dim3 grid = xcd ? dim3((unsigned)nbx * nby) : dim3(nbx, nby);
  if (ny_per == 16)
    hipLaunchKernelGGL(k_tsk_combine<16>, grid, dim3(kBlock), 0, s, n, nv, base, ld, slot, G, ldg, ny, obase, old,
                       oslot, accumulate, nbx, nby, xcd);
  else
    hipLaunchKernelGGL(k_tsk_combine<8>, grid, dim3(kBlock), 0, s, n, nv, base, ld, slot, G, ldg, ny, obase, old,
                       oslot, accumulate, nbx, nby, xcd);
  DL_HIP(hipGetLastError());
}

static TskCfg combine_shape(TskCfg c, long n, int nv) {
  const int full = max_stream_blocks(n);
  if (c.grid < 1) c.grid = stream_blocks(n);
  if (c.grid > full) c.grid = full;
  if (c.tile < 0 || c.tile > 3 || ((c.tile & 2) && nv > kMaxNV / 2)) c.tile = 0;
  return c;
}

void tsk_combine(hipStream_t s, long n, int nv, const double2* base, long ld, const int* slot,
                 const double* G, int ldg, int ny, double2* obase, long old, const int* oslot,
                 int accumulate) {
  if (nv > kMaxNV) fail(DL_E_INVALID, "too many basis vectors (max 512)");
  if (nv <= 0 || ny <= 0) return;
  std::vector<TskCfg> cands;
  for (int t = 0; t < 4; ++t) {
    if ((t & 2) && nv > kMaxNV / 2) continue;
    for (int g : {2048, 1024, 4096}) {
      const TskCfg c = combine_shape(TskCfg{g, t}, n, nv);
      bool dup = false;
      for (const auto& o : cands) dup |= o.grid == c.grid && o.tile == c.tile;
      if (!dup) cands.push_back(c);
    }
  }
  cands.insert(cands.begin(), combine_shape(TskCfg{}, n, nv));  // the default first
  // timed with zero coefficients: outputs get zeros (or + 0) until the real launch below
  const TskCfg c = combine_shape(
      choose(s, TK_COMBINE, n, nv, ny, cands,
                 [&](const TskCfg& t) {
                   const double* gz = reinterpret_cast<const double*>(zeros(s, (size_t)nv * ldg));
                   combine_launch(s, n, nv, base, ld, slot, gz, ldg, ny, obase, old, oslot, accumulate, t);
                 }),
      n, nv);
  combine_launch(s, n, nv, base, ld, slot, G, ldg, ny, obase, old, oslot, accumulate, c);
}

int tsk_multi_nblocks(long n) {
  long nb = (n + kTR - 1) / kTR;
  if (nb < 1) nb = 1;
  if (nb > kMultiBlocks) nb = kMultiBlocks;
  return (int)nb;
}

// Grid candidates of a partial-writing kernel: the default d, d/2, d/4 (at least 1).
static std::vector<TskCfg> grid_cands(int d, const std::vector<int>& tiles) {
  std::vector<TskCfg> c;
  for (int t : tiles)
    for (int g : {d, d / 2, d / 4})
      if (g >= 1) {
        bool dup = false;
        for (const auto& o : c) dup |= o.grid == g && o.tile == t;
        if (!dup) c.push_back(TskCfg{g, t});
      }
  return c;
}

int tsk_dots_multi(hipStream_t s, long n, int nv, const double2* base, long ld, const double2* W, long ldw, int nw,
                   const int* active, double* part) {
  if (nv > kMultiNV) fail(DL_E_INVALID, "too many basis vectors for one multi-column contraction (max 64)");
  if (nw < 1 || nw > kTW) fail(DL_E_INVALID, "multi-column contraction takes 1..16 columns");
  const int d = tsk_multi_nblocks(n);
  auto launch = [&](const TskCfg& c) {
    for (int j0 = 0; j0 < nv; j0 += kTJ) {
      const int nj = nv - j0 < kTJ ? nv - j0 : kTJ;
      hipLaunchKernelGGL(k_tsk_dots_multi, dim3(c.grid), dim3(kBlock), 0, s, n, nv, j0, nj, base, ld, W, ldw, nw,
                         active, part);
      DL_HIP(hipGetLastError());
    }
  };
  // timed into the caller's partials, which the launch below overwrites
  TskCfg c = choose(s, TK_DOTS64, n, nv, nw, grid_cands(d, {0}), launch);
  c.grid = std::max(1, std::min(c.grid, d));
  c.tile = 0;
  launch(c);
  return c.grid;
}

template <class VB>
static void update_launch(hipStream_t s, long n, int nv, const VB* base, long ld, const double2* D, int nw,
                          const int* active, double2* X, long ldx, int nb) {
  constexpr int kChunk = kMaxNV / 4;  // basis vectors per launch (LDS holds kChunk x NW coefficients)
  for (int j0 = 0; j0 < nv; j0 += kChunk) {
    const int nc = nv - j0 < kChunk ? nv - j0 : kChunk;
    const VB* b = base + (long)j0 * ld;
    const double2* d = D + j0;
    if (nw <= 4)
      hipLaunchKernelGGL((k_tsk_update_multi<4, VB>), dim3(nb), dim3(kBlock), 0, s, n, nc, b, ld, d, nv, nw, active,
                         X, ldx);
    else if (nw <= 8)
      hipLaunchKernelGGL((k_tsk_update_multi<8, VB>), dim3(nb), dim3(kBlock), 0, s, n, nc, b, ld, d, nv, nw, active,
                         X, ldx);
    else if (nw <= 12)  // the 12 spin-colour sources: no FP64 work on padding columns
      hipLaunchKernelGGL((k_tsk_update_multi<12, VB>), dim3(nb), dim3(kBlock), 0, s, n, nc, b, ld, d, nv, nw, active,
                         X, ldx);
    else
      hipLaunchKernelGGL((k_tsk_update_multi<16, VB>), dim3(nb), dim3(kBlock), 0, s, n, nc, b, ld, d, nv, nw, active,
                         X, ldx);
    DL_HIP(hipGetLastError());
  }
}

template <class VB>
static void update_multi(hipStream_t s, long n, int nv, const VB* base, long ld, const double2* D, int nw,
                         const int* active, double2* X, long ldx) {
  if (nw < 1 || nw > 16) fail(DL_E_INVALID, "multi-column contraction takes 1..16 columns");
  if (nv <= 0) return;
  const int full = max_stream_blocks(n);
  std::vector<TskCfg> cands{TskCfg{stream_blocks(n), 0}};
  for (int g : {512, 1024, 4096})
    if (g <= full && g != cands[0].grid) cands.push_back(TskCfg{g, 0});
  // timed with zero coefficients (X + 0 = X)
  TskCfg c = choose(s, sizeof(VB) == 16 ? TK_UPD64 : TK_UPD32, n, nv, nw, cands, [&](const TskCfg& t) {
    update_launch(s, n, nv, base, ld, zeros(s, (size_t)2 * nv * nw), nw, active, X, ldx, t.grid);
  });
  c.grid = std::max(1, std::min(c.grid, full));
  update_launch(s, n, nv, base, ld, D, nw, active, X, ldx, c.grid);
}

void tsk_update_multi(hipStream_t s, long n, int nv, const double2* base, long ld, const double2* D, int nw,
                      const int* active, double2* X, long ldx) {
  update_multi(s, n, nv, base, ld, D, nw, active, X, ldx);
}

void tsk_update_multi32(hipStream_t s, long n, int nv, const float2* base, long ld, const double2* D, int nw,
                        const int* active, double2* X, long ldx) {
  update_multi(s, n, nv, base, ld, D, nw, active, X, ldx);
}

// ---- matrix-core contraction C = V^H W over FP32- or BF16-stored fields -----------------
//
// Each complex field of n elements is read as a real vector of 2n entries (re, im
// interleaved).  Then Re C[j][r] = sum_p V_j[p] W_r[p] and Im C[j][r] = sum_p V_j[p] W'_r[p]
// with W' the interleaved form of -i W (each pair (a, b) becomes (b, -a)), so one real
// contraction against the 2*16 columns [W | W'] gives both parts.  Per wave, a step takes
// one 16-byte load per lane from each of 16 basis vectors (lane % 16 picks the vector,
// lane / 16 the 16-byte piece) and from 16 columns (lane % 16 picks the column), and feeds
//   BF16: v_mfma_f32_16x16x32_bf16 (8 bf16 = 4 complex per lane, K = 32 per instruction),
//   FP32: v_mfma_f32_16x16x4_f32 four times (4 floats = 2 complex per lane, K = 4 each).
// The K ordering is the same for the A and B operands, so the sum is over the same real
// positions whatever order the matrix core visits them in.  A wave walks pairs of steps
// (128 contiguous bytes of each vector) strided over the grid; FP32 accumulation inside a
// block, FP64 partials across blocks (summed in a fixed order by sum_partials).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kLpBlocks = 2048; // upper bound of partials per column
constexpr int kLpDefault = 512; // the untuned grid (at most)

template <class SV>
struct LpTraits;
template <>
struct LpTraits<bf2> {
  static constexpr int kCpl = 4;  // complex elements per 16-byte lane load
};
template <>
struct LpTraits<float2> {
  static constexpr int kCpl = 2;
};

// 16 bytes of a field starting at complex element e (zero past n; n need not be a multiple
// of the load width, but the field base must be 16-byte aligned).
template <class SV>
__device__ __forceinline__ u32x4_t lp_load(const SV* __restrict__ f, long e, long n) {
  constexpr int C = LpTraits<SV>::kCpl;
  if (e + C <= n) return *reinterpret_cast<const u32x4_t*>(f + e);
  u32x4_t v = {0u, 0u, 0u, 0u};
  const unsigned int* w = reinterpret_cast<const unsigned int*>(f + e);
  constexpr int kWords = sizeof(SV) / 4;  // 32-bit words per complex element
#pragma unroll
  for (int c = 0; c < C; ++c)
    if (e + c < n) {
#pragma unroll
      for (int q = 0; q < kWords; ++q) v[c * kWords + q] = w[c * kWords + q];
    }
  return v;
}

// -i * w on 16 bytes of interleaved complex numbers
__device__ __forceinline__ u32x4_t lp_rot(u32x4_t w, bf2*) {
  u32x4_t o;
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q] = ((w[q] >> 16) | (w[q] << 16)) ^ 0x80000000u;  // (a, b) -> (b, -a)
  return o;
}
__device__ __forceinline__ u32x4_t lp_rot(u32x4_t w, float2*) {
  u32x4_t o;
  o[0] = w[1];
  o[1] = w[0] ^ 0x80000000u;
  o[2] = w[3];
  o[3] = w[2] ^ 0x80000000u;
  return o;
}

__device__ __forceinline__ void lp_mfma(f32x4_t& acc, u32x4_t a, u32x4_t b, bf2*) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                acc, 0, 0, 0);
}
__device__ __forceinline__ void lp_mfma(f32x4_t& acc, u32x4_t a, u32x4_t b, float2*) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a[q]), __uint_as_float(b[q]), acc, 0, 0, 0);
}

// part[(2*(r*nv + j0 + j) + reim) * gridDim.x + blockIdx.x] for j < nj (<= 16 * kNT), r < nw (<= 16).
// kNT row tiles of 16 basis vectors per launch (2, 4 or 8; the autotuner picks it).
template <class SV, int kNT>
__global__ void __launch_bounds__(kBlock)
k_tsk_dots_mfma(long n, int nv, int j0, int nj, const SV* __restrict__ base, long ld, const SV* __restrict__ W,
                long ldw, int nw, const int* __restrict__ active, double* __restrict__ part) {
  constexpr int C = LpTraits<SV>::kCpl;
  constexpr int kStep = 4 * C;  // complex elements of each vector per step (4 lane groups)
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int li = lane & 15, grp = lane >> 4;
  const bool col_on = li < nw && (!active || active[li]);
  const SV* wcol = W + (long)li * ldw;
  const SV* vrow[kNT];
  bool row_on[kNT];
#pragma unroll
  for (int t = 0; t < kNT; ++t) {
    const int j = 16 * t + li;
    row_on[t] = j < nj;
    vrow[t] = base + (long)(j0 + (row_on[t] ? j : 0)) * ld;
  }
  f32x4_t acc[kNT][2];
#pragma unroll
  for (int t = 0; t < kNT; ++t) acc[t][0] = acc[t][1] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const long nsteps = (n + kStep - 1) / kStep;
  const long npairs = (nsteps + 1) / 2;
  const long nwaves = (long)gridDim.x * (kBlock / 64);
  const u32x4_t zero = {0u, 0u, 0u, 0u};
  for (long pr = (long)blockIdx.x * (kBlock / 64) + wid; pr < npairs; pr += nwaves) {
    u32x4_t a[2][kNT], b[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const long e = (2 * pr + u) * kStep + grp * C;
      const bool in = e < n;
      b[u] = (in && col_on) ? lp_load(wcol, e, n) : zero;
#pragma unroll
      for (int t = 0; t < kNT; ++t) a[u][t] = (in && row_on[t]) ? lp_load(vrow[t], e, n) : zero;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const u32x4_t bi = lp_rot(b[u], (SV*)nullptr);
#pragma unroll
      for (int t = 0; t < kNT; ++t) {
        lp_mfma(acc[t][0], a[u][t], b[u], (SV*)nullptr);
        lp_mfma(acc[t][1], a[u][t], bi, (SV*)nullptr);
      }
    }
  }
  // add the four waves' tiles in a fixed order, four row tiles at a time; acc[t][c][q] of lane l
  // is row 16t + 4*(l/16) + q, column l % 16 of the real (c = 0) or imaginary (c = 1) part
  constexpr int kTG = kNT < 4 ? kNT : 4;
  __shared__ float red[kBlock / 64][kTG * 2 * 4][64];
#pragma unroll
  for (int t0 = 0; t0 < kNT; t0 += kTG) {
    if (t0) __syncthreads();
#pragma unroll
    for (int t = 0; t < kTG; ++t)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[wid][(t * 2 + c) * 4 + q][lane] = acc[t0 + t][c][q];
    __syncthreads();
    for (int e = threadIdx.x; e < kTG * 2 * 4 * 64; e += kBlock) {
      const int slot = e / 64, l = e % 64;
      const int t = t0 + slot / 8, c = (slot / 4) % 2, q = slot % 4;
      const int j = 16 * t + 4 * (l / 16) + q, r = l % 16;
      if (j >= nj || r >= nw) continue;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) v += (double)red[w][slot][l];
      part[(2L * ((long)r * nv + j0 + j) + c) * gridDim.x + blockIdx.x] = v;
    }
  }
}

template <class SV, int kNT>
static void mfma_launch(hipStream_t s, long n, int nv, const SV* base, long ld, const SV* W, long ldw, int nw,
                        const int* active, double* part, int nb) {
  constexpr int kRowsPer = 16 * kNT;
  for (int j0 = 0; j0 < nv; j0 += kRowsPer) {
    const int nj = nv - j0 < kRowsPer ? nv - j0 : kRowsPer;
    hipLaunchKernelGGL((k_tsk_dots_mfma<SV, kNT>), dim3(nb), dim3(kBlock), 0, s, n, nv, j0, nj, base, ld, W, ldw, nw,
                       active, part);
    DL_HIP(hipGetLastError());
  }
}

template <class SV>
static int dots_mfma(hipStream_t s, long n, int nv, const SV* base, long ld, const SV* W, long ldw, int nw,
                     const int* active, double* part) {
  if (nv < 1 || nv > kLpMaxNV) fail(DL_E_INVALID, "low-precision contraction takes 1..128 basis vectors");
  if (nw < 1 || nw > 16) fail(DL_E_INVALID, "low-precision contraction takes 1..16 columns");
  if (n < 1) fail(DL_E_INVALID, "empty fields");
  constexpr int C = LpTraits<SV>::kCpl;
  if ((reinterpret_cast<uintptr_t>(base) | reinterpret_cast<uintptr_t>(W)) % 16 != 0 || ld % C != 0 || ldw % C != 0)
    fail(DL_E_INVALID, "low-precision contraction needs 16-byte aligned fields");
  const int dmax = tsk_lowp_nblocks(n, sizeof(SV) == 4 ? DL_BF16 : DL_FP32);  // what part holds
  const int d = std::min(dmax, kLpDefault);
  auto launch = [&](const TskCfg& c) {
    if (c.tile == 2) mfma_launch<SV, 2>(s, n, nv, base, ld, W, ldw, nw, active, part, c.grid);
    else if (c.tile == 8) mfma_launch<SV, 8>(s, n, nv, base, ld, W, ldw, nw, active, part, c.grid);
    else mfma_launch<SV, 4>(s, n, nv, base, ld, W, ldw, nw, active, part, c.grid);
  };
  // the default (4 row tiles, d blocks) first; timed into the caller's partials
  std::vector<TskCfg> cands;
  for (int t : {4, 2, 8})
    for (int g : {d, 2 * d, 4 * d, d / 2, d / 4})
      if (g >= 1 && g <= dmax) {
        bool dup = false;
        for (const auto& o : cands) dup |= o.grid == g && o.tile == t;
        if (!dup) cands.push_back(TskCfg{g, t});
      }
  TskCfg c = choose(s, sizeof(SV) == 4 ? TK_DOTS16 : TK_DOTS32, n, nv, nw, cands, launch);
  c.grid = std::max(1, std::min(c.grid, dmax));
  if (c.tile != 2 && c.tile != 8) c.tile = 4;
  launch(c);
  return c.grid;
}

int tsk_lowp_nblocks(long n, int prec) {
  const long step = prec == DL_BF16 ? 16 : 8;  // complex elements per wave step
  long nb = (n + 8 * step - 1) / (8 * step);   // one pair of steps per wave, four waves per block
  if (nb < 1) nb = 1;
  if (nb > kLpBlocks) nb = kLpBlocks;
  return (int)nb;
}

int tsk_dots_lowp(hipStream_t s, long n, int nv, const float2* base, long ld, const float2* W, long ldw, int nw,
                  const int* active, double* part) {
  return dots_mfma(s, n, nv, base, ld, W, ldw, nw, active, part);
}

int tsk_dots_lowp(hipStream_t s, long n, int nv, const bf2* base, long ld, const bf2* W, long ldw, int nw,
                  const int* active, double* part) {
  return dots_mfma(s, n, nv, base, ld, W, ldw, nw, active, part);
}

TskCfg tsk_tune(hipStream_t s, int kind, long n, int nv, int nw, int reps, double* best_us) {
  if (reps < 1) fail(DL_E_INVALID, "reps must be >= 1");
  if (n < 1) fail(DL_E_INVALID, "n must be >= 1");
  const int nvmax = kind == TK_DOTS64 ? kMultiNV : (kind == TK_DOTS32 || kind == TK_DOTS16) ? kLpMaxNV : kMaxNV;
  if (nv < 1 || nv > nvmax) fail(DL_E_INVALID, "nv out of range for this contraction");
  if (nw < 1 || nw > (kind == TK_COMBINE ? kMaxNV : 16)) fail(DL_E_INVALID, "nw out of range for this contraction");
  // fields of zeros (the kernels' time does not depend on the values)
  const long ld = (n + 3) / 4 * 4;
  DBuf<double2> V, W;
  DBuf<double> part;
  struct Reset {
    ~Reset() { t_tune = TuneReq(); }
  } reset;
  t_tune.reps = reps;
  switch (kind) {
    case TK_DOTS64:
      V.alloc((size_t)nv * n);
      W.alloc((size_t)nw * n);
      part.alloc((size_t)2 * nv * nw * tsk_multi_nblocks(n));
      zero(s, (long)V.n, V.get());
      zero(s, (long)W.n, W.get());
      tsk_dots_multi(s, n, nv, V.get(), n, W.get(), n, nw, nullptr, part.get());
      break;
    case TK_DOTS32:
    case TK_DOTS16: {
      const bool b16 = kind == TK_DOTS16;
      V.alloc(((size_t)nv * ld + 1) / 2);
      W.alloc(((size_t)nw * ld + 1) / 2);
      part.alloc((size_t)2 * nv * nw * tsk_lowp_nblocks(n, b16 ? DL_BF16 : DL_FP32));
      zero(s, (long)V.n, V.get());
      zero(s, (long)W.n, W.get());
      if (b16)
        tsk_dots_lowp(s, n, nv, reinterpret_cast<const bf2*>(V.get()), ld, reinterpret_cast<const bf2*>(W.get()), ld,
                      nw, nullptr, part.get());
      else
        tsk_dots_lowp(s, n, nv, reinterpret_cast<const float2*>(V.get()), ld, reinterpret_cast<const float2*>(W.get()),
                      ld, nw, nullptr, part.get());
      break;
    }
    case TK_UPD64:
    case TK_UPD32: {
      const bool f32 = kind == TK_UPD32;
      V.alloc(f32 ? ((size_t)nv * n + 1) / 2 : (size_t)nv * n);
      W.alloc((size_t)nw * n);
      DBuf<double2> D((size_t)nw * nv);
      zero(s, (long)V.n, V.get());
      zero(s, (long)W.n, W.get());
      zero(s, (long)D.n, D.get());
      if (f32)
        tsk_update_multi32(s, n, nv, reinterpret_cast<const float2*>(V.get()), n, D.get(), nw, nullptr, W.get(), n);
      else
        tsk_update_multi(s, n, nv, V.get(), n, D.get(), nw, nullptr, W.get(), n);
      DL_HIP(hipStreamSynchronize(s));
      break;
    }
    case TK_COMBINE: {
      V.alloc((size_t)nv * n);
      W.alloc((size_t)nw * n);
      DBuf<double2> G(((size_t)nv * nw + 1) / 2);
      zero(s, (long)V.n, V.get());
      zero(s, (long)G.n, G.get());
      tsk_combine(s, n, nv, V.get(), n, nullptr, reinterpret_cast<const double*>(G.get()), nw, nw, W.get(), n,
                  nullptr, 0);
      DL_HIP(hipStreamSynchronize(s));
      break;
    }
    default:
      fail(DL_E_INVALID, "unknown contraction kind");
  }
  DL_HIP(hipStreamSynchronize(s));
  if (best_us) *best_us = t_tune.us;
  return t_tune.cfg;
}

}  // namespace dl
