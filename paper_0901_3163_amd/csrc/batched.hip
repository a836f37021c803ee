// Batched, mixed-precision later right-hand sides: D-MinRes / D-CG for nrhs
// right-hand sides advanced together.
//
// Every stage is one launch over (site block, right-hand side) pairs, so the
// Wilson links are read from HBM once per site block for the whole batch and
// launch latency is paid once per stage instead of once per right-hand side.
// Right-hand sides that have converged are masked off (their blocks return at
// once).  Krylov vectors and the Wilson apply are FP32 or BF16 storage with FP32
// arithmetic (links FP32);
// the solution x, the residual r = b - M x and the Galerkin projection over
// the stored eigenvectors (Section 2: "projected ... at the beginning") are
// FP64.  Accuracy is won back by restarting the FP32 inner solve from the FP64
// true residual r64 = b - M x64 (defect correction) whenever the inner
// residual estimate has dropped by `inner_drop`, re-projecting over the
// eigenvectors at every restart.  The inner MinRes / CG runs on the
// correction e with A e = gamma5 r64 (MinRes) or M e = r64 (CG on the normal
// equations), and x64 += e closes each cycle.  The batched CG instead keeps its
// search direction across FP64 reliable updates (x64 += e, r = b - M x64).  The batched
// MinRes keeps a cycle's Lanczos vectors in a ring and adds their share of e once per
// window of iterations (graph replay runs the fused short-recurrence form instead).
//
// A batch may hold several operators (lattices of different sizes): field j of the
// batch then starts at offs[j] and has length lens[j] (Seg), the stencil runs as one
// work-list launch over all lattices (wilson_multi), and every other stage is one
// launch over (block, rhs) pairs whatever lattice the rhs belongs to.
#include "engine.hpp"
#include "ptc.hpp"
#include "cplx.hpp"
#include "small.hpp"
#include "tsk.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <type_traits>

namespace dl {

// per-rhs device state, st[r * NS + field]
enum {
  B_ALPHA = 0, B_BETA, B_BNEXT, B_COLD, B_SOLD, B_C, B_S, B_ETA, B_TAU, B_DELTA, B_EPS, B_GAMMA,
  B_INV, B_NRM, B_FLAG, B_SS, B_QQ, B_RR, B_CGA, B_CGB, B_NCUR, B_NPREV, B_WSTART, B_WCNT, NS
};

// Field layout of a batch: rhs r starts at off[r] and has len[r] complex elements (device
// tables); off == nullptr means uniform fields of length n at stride n.
struct Seg {
  const long* off;
  const long* len;
  long n;
};
__device__ __forceinline__ long seg_off(const Seg& g, int r) { return g.off ? g.off[r] : (long)r * g.n; }
__device__ __forceinline__ long seg_len(const Seg& g, int r) { return g.off ? g.len[r] : g.n; }

constexpr int kMaxWindow = 64;  // longest window of the windowed MinRes

static int bgrid(long n) {
  long nb = (n + kBlock - 1) / kBlock;
  return (int)std::max(1L, std::min(nb, 1024L));
}

__device__ __forceinline__ double b_fin_sum(const double* part, int np, double* lds) {
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += kBlock) a += part[i];
  return block_sum<kBlock>(a, lds);
}

// ---- FP64 <-> FP32 and residual kernels (grid: (G, nrhs)) -----------------------
// r = b - y (FP64; y == nullptr: r = b), partial ||r||^2 column-major [rhs][G]
__global__ void __launch_bounds__(kBlock)
k_b_resid(Seg g, const double2* b, const double2* y, double2* r, const int* __restrict__ active,
          double* __restrict__ part) {
  const int rhs = blockIdx.y;
  double acc = 0.0;
  if (!active || active[rhs]) {
    const long off = seg_off(g, rhs), n = seg_len(g, rhs);
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
      const double2 v = y ? c_sub(b[off + i], y[off + i]) : b[off + i];
      r[off + i] = v;
      acc = fma(v.x, v.x, fma(v.y, v.y, acc));
    }
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[(long)rhs * gridDim.x + blockIdx.x] = s;
}

// per-rhs sum of partials into st[r*NS + field] (and sqrt into B_NRM / B_INV if field == B_RR)
__global__ void __launch_bounds__(kBlock) k_b_fin_store(const double* part, int np, double* st, int field) {
  const int r = blockIdx.x;
  __shared__ double lds[kBlock / 64];
  const double s = b_fin_sum(part + (long)r * np, np, lds);
  if (threadIdx.x == 0) {
    st[r * NS + field] = s;
    if (field == B_RR) {
      const double nr = sqrt(s);
      st[r * NS + B_NRM] = nr;
      st[r * NS + B_INV] = nr > 0.0 ? 1.0 / nr : 0.0;
    }
  }
}

// MinRes inner start: v = gamma5 r64 * inv (FP32), vp = d1 = d2 = e = 0; state reset.
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_minres_start(Seg g, const double2* r64, SV* v, SV* vp, SV* d1, SV* d2, SV* e, double* st, double* invs,
                 const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const double inv = st[rhs * NS + B_INV];
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const int c = (int)((i >> 6) % kSpin);
    const double2 x = r64[off + i];
    const double sg = c >= 6 ? -inv : inv;
    sst(v + off + i, make_float2((float)(x.x * sg), (float)(x.y * sg)));
    const float2 z = make_float2(0.f, 0.f);
    sst(vp + off + i, z);
    sst(d1 + off + i, z);
    sst(d2 + off + i, z);
    sst(e + off + i, z);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* s = st + rhs * NS;
    s[B_ETA] = s[B_NRM];
    s[B_BETA] = 0.0;
    s[B_COLD] = 1.0;
    s[B_SOLD] = 0.0;
    s[B_C] = 1.0;
    s[B_S] = 0.0;
    s[B_FLAG] = 0.0;
    s[B_NCUR] = 1.0;   // the first Lanczos vector is stored normalised
    s[B_NPREV] = 1.0;
    // the update that the first fused step applies (of the iteration before the first) is
    // d = (vp - 0 - 0) / 1 = 0, e += 0
    s[B_TAU] = 0.0;
    s[B_DELTA] = 0.0;
    s[B_EPS] = 0.0;
    s[B_GAMMA] = 1.0;
    s[B_WSTART] = 0.0;  // windowed form: no rotation recorded yet
    s[B_WCNT] = 0.0;
    invs[rhs] = 1.0;
  }
}

// coef != nullptr (windowed MinRes): the rotation's (tau, delta, eps, gamma, n_j) is also
// recorded at slot B_WCNT of the rhs's window (W slots) and B_WCNT is advanced.
__global__ void __launch_bounds__(kBlock)
k_b_fin_rot(const double* part, int np, double* st, double* invs, const int* active, double* coef = nullptr,
            int W = 0) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  __shared__ double lds[kBlock / 64];
  const double ww = b_fin_sum(part + (long)r * np, np, lds);
  if (threadIdx.x == 0) {
    double* S = st + r * NS;
    const double bnext = sqrt(ww);
    const double beta = S[B_BETA], alpha = S[B_ALPHA];
    const double eps = S[B_SOLD] * beta;
    const double dt = S[B_COLD] * beta;
    const double delta = S[B_C] * dt + S[B_S] * alpha;
    const double gbar = -S[B_S] * dt + S[B_C] * alpha;
    const double gamma = hypot(gbar, bnext);
    const bool ok = gamma > 0.0 && isfinite(gamma) && isfinite(bnext) && S[B_FLAG] == 0.0;
    if (ok) {
      const double cn = gbar / gamma, sn = bnext / gamma;
      S[B_TAU] = cn * S[B_ETA];
      S[B_ETA] = -sn * S[B_ETA];
      S[B_EPS] = eps;
      S[B_DELTA] = delta;
      S[B_GAMMA] = gamma;
      S[B_COLD] = S[B_C];
      S[B_SOLD] = S[B_S];
      S[B_C] = cn;
      S[B_S] = sn;
      S[B_BNEXT] = bnext;
      S[B_BETA] = bnext;
      S[B_NPREV] = S[B_NCUR];
      S[B_NCUR] = bnext;
      invs[r] = bnext > 0.0 ? 1.0 / bnext : 0.0;
      if (!(bnext > 0.0)) S[B_FLAG] = 2.0;
    } else {
      S[B_TAU] = 0.0;
      S[B_EPS] = 0.0;
      S[B_DELTA] = 0.0;
      S[B_GAMMA] = 1.0;
      S[B_BNEXT] = 0.0;
      invs[r] = 0.0;
      if (S[B_FLAG] == 0.0) S[B_FLAG] = 1.0;
    }
    if (coef) {
      const int L = (int)S[B_WCNT];
      if (L < W) {
        double* c = coef + ((long)r * W + L) * 5;
        c[0] = S[B_TAU];
        c[1] = S[B_DELTA];
        c[2] = S[B_EPS];
        c[3] = S[B_GAMMA];
        c[4] = S[B_NPREV];
        S[B_WCNT] = L + 1;
      } else {
        S[B_FLAG] = 3.0;  // a window overran (the host flushes every W iterations)
      }
    }
  }
}

// d_new = (u_j / n_j - delta d1 - eps d2)/gamma -> dn ; e += tau d_new   (n_j = B_NPREV after the rotation)
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_minres_update(Seg g, const double* st, const SV* u, const SV* d1, const SV* d2, SV* dn, SV* e,
                  const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const double* S = st + rhs * NS;
  const float delta = (float)S[B_DELTA], eps = (float)S[B_EPS], ig = (float)(1.0 / S[B_GAMMA]);
  const float tau = (float)S[B_TAU];
  const float iu = (float)(1.0 / S[B_NPREV]);
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    float2 d = c_axpy(-delta, sld(d1 + off + i), c_scale(sld(u + off + i), iu));
    d = c_axpy(-eps, sld(d2 + off + i), d);
    d = c_scale(d, ig);
    sst(dn + off + i, d);
    sst(e + off + i, c_axpy(tau, d, sld(e + off + i)));
  }
}

// One pass for two steps of the batched MinRes.  Lanczos vectors are kept unnormalised,
// u_j = n_j v_j, and w = A v_{j+1} (the Wilson epilogue applied 1/n_{j+1}).  The Lanczos step
// of iteration j + 1: un = w - (alpha/n_{j+1}) u_{j+1} - (beta_{j+1}/n_j) u_j, written over
// u_j, partial ||un||^2.  The solution update of iteration j, delayed by one iteration: as
// k_b_minres_update on u_j with the rotation of iteration j, which the state holds until the
// rotation of j + 1 is formed after this pass.  u_j is read once for both; the per-element
// arithmetic and its order are those of the two steps done apart.
// alpha = <v_{j+1}, A v_{j+1}> is summed from the stencil's partials (apart, anp per rhs) by
// every block in the same fixed order; block 0 of each rhs stores it for the rotation.
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_lanczos_minres(Seg g, double* st, const SV* u, SV* up, const SV* w, const SV* d1, SV* d2, SV* e,
                   const int* __restrict__ active, const double* __restrict__ apart, int anp,
                   double* __restrict__ part) {
  const int rhs = blockIdx.y;
  double acc = 0.0;
  __shared__ double lds[kBlock / 64];
  if (!active || active[rhs]) {
    __shared__ double alpha_s;
    const double asum = b_fin_sum(apart + (long)rhs * anp, anp, lds);
    if (threadIdx.x == 0) {
      alpha_s = asum;
      if (blockIdx.x == 0) st[rhs * NS + B_ALPHA] = asum;
    }
    __syncthreads();
    const double* S = st + rhs * NS;
    // after an exact breakdown (n_{j+1} = 0) the rhs's vectors are zero until the host check
    // retires it: a = 0/0 would put NaN into the solution update
    const float a = S[B_NCUR] > 0.0 ? (float)(alpha_s / S[B_NCUR]) : 0.f;
    const float b = (float)(S[B_BETA] / S[B_NPREV]);
    const float delta = (float)S[B_DELTA], eps = (float)S[B_EPS], ig = (float)(1.0 / S[B_GAMMA]);
    const float tau = (float)S[B_TAU];
    const float iu = (float)(1.0 / S[B_NPREV]);
    const long off = seg_off(g, rhs), n = seg_len(g, rhs);
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
      const float2 uj = sld(up + off + i);
      float2 d = c_axpy(-delta, sld(d1 + off + i), c_scale(uj, iu));
      d = c_axpy(-eps, sld(d2 + off + i), d);
      d = c_scale(d, ig);
      sst(d2 + off + i, d);
      sst(e + off + i, c_axpy(tau, d, sld(e + off + i)));
      float2 t = c_axpy(-a, sld(u + off + i), sld(w + off + i));
      t = c_axpy(-b, uj, t);
      sst(up + off + i, t);
      acc = fma((double)t.x, (double)t.x, fma((double)t.y, (double)t.y, acc));
    }
  }
  __syncthreads();  // lds is reused
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[(long)rhs * gridDim.x + blockIdx.x] = s;
}

// ---- windowed MinRes ---------------------------------------------------------------
// The same iterates as the fused form above, with the solution kept apart from the Lanczos
// pass: the unnormalised Lanczos vectors u_j of the cycle go to a ring of R = W + 2 slots
// (u_j in slot j mod R, u_0 = 0), each rotation's coefficients are recorded, and every W
// iterations one pass forms the window's share of the solution update and the last two
// search directions from the stored vectors.  The per-iteration pass then reads three
// vectors and writes one instead of reading six and writing three.

// Lanczos step alone: un = w - (alpha/n_{j+1}) u - (beta_{j+1}/n_j) up, partial ||un||^2;
// alpha is summed from the stencil partials as in k_b_lanczos_minres.
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_lanczos_w(Seg g, double* st, const SV* u, const SV* up, const SV* w, SV* un, const int* __restrict__ active,
              const double* __restrict__ apart, int anp, double* __restrict__ part) {
  const int rhs = blockIdx.y;
  double acc = 0.0;
  __shared__ double lds[kBlock / 64];
  if (!active || active[rhs]) {
    __shared__ double alpha_s;
    const double asum = b_fin_sum(apart + (long)rhs * anp, anp, lds);
    if (threadIdx.x == 0) {
      alpha_s = asum;
      if (blockIdx.x == 0) st[rhs * NS + B_ALPHA] = asum;
    }
    __syncthreads();
    const double* S = st + rhs * NS;
    // after an exact breakdown (n_{j+1} = 0) the rhs's vectors are zero until the host check
    // retires it: a = 0/0 would put NaN into the ring and the window's update
    const float a = S[B_NCUR] > 0.0 ? (float)(alpha_s / S[B_NCUR]) : 0.f;
    const float b = (float)(S[B_BETA] / S[B_NPREV]);
    const long off = seg_off(g, rhs), n = seg_len(g, rhs);
    // four elements per thread and step (fields are whole 64-site tiles: n and off are
    // multiples of 768 elements), one 16-byte (BF16) or two (FP32) accesses per field
    const long n4 = n >> 2;
    for (long q = (long)blockIdx.x * kBlock + threadIdx.x; q < n4; q += (long)gridDim.x * kBlock) {
      float2 vu[4], vw[4], vp[4];
      sld4(u + off + 4 * q, vu);
      sld4(w + off + 4 * q, vw);
      sld4(up + off + 4 * q, vp);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        vw[k] = c_axpy(-b, vp[k], c_axpy(-a, vu[k], vw[k]));
        acc = fma((double)vw[k].x, (double)vw[k].x, fma((double)vw[k].y, (double)vw[k].y, acc));
      }
      sst4(un + off + 4 * q, vw);
    }
    for (long i = 4 * n4 + (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
      float2 t = c_axpy(-a, sld(u + off + i), sld(w + off + i));
      t = c_axpy(-b, sld(up + off + i), t);
      sst(un + off + i, t);
      acc = fma((double)t.x, (double)t.x, fma((double)t.y, (double)t.y, acc));
    }
  }
  __syncthreads();  // lds is reused
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[(long)rhs * gridDim.x + blockIdx.x] = s;
}

// Coefficients of a window, one block per rhs.  Over the basis B = (d_{J-1}, d_J, u_{J+1},
// ..., u_{J+L}) (J = B_WSTART, L = B_WCNT recorded rotations), the search directions
// d_j = (u_j / n_j - delta_j d_{j-1} - eps_j d_{j-2}) / gamma_j are carried as coefficient
// vectors in FP64, thread b holding component b.  Out, per rhs (stride 2 + 3 (W + 2)): J, L,
// then the coefficients of sum_j tau_j d_j, of d_{J+L} and of d_{J+L-1}.  The window is then
// closed: B_WSTART += L, B_WCNT = 0.
__global__ void __launch_bounds__(128)
k_b_wcoef(double* st, const double* coef, int W, double* out, const int* __restrict__ active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  double* S = st + r * NS;
  const int L = (int)S[B_WCNT];
  const double J = S[B_WSTART];
  __syncthreads();
  const int b = threadIdx.x;
  const long stride = 2 + 3L * (W + 2);
  double* o = out + r * stride;
  if (b < W + 2) {
    double dm2 = b == 0 ? 1.0 : 0.0, dm1 = b == 1 ? 1.0 : 0.0, cx = 0.0;
    for (int i = 1; i <= L; ++i) {
      const double* c = coef + ((long)r * W + i - 1) * 5;
      double d = (b == 1 + i ? 1.0 / c[4] : 0.0) - c[1] * dm1 - c[2] * dm2;
      d /= c[3];
      cx = fma(c[0], d, cx);
      dm2 = dm1;
      dm1 = d;
    }
    o[2 + b] = cx;
    o[2 + (W + 2) + b] = dm1;
    o[2 + 2 * (W + 2) + b] = dm2;
  }
  if (b == 0) {
    o[0] = J;
    o[1] = L;
    S[B_WSTART] = J + L;
    S[B_WCNT] = 0.0;
  }
}

// The window's pass: e += sum_j tau_j d_j, d1 = d_{J+L}, d2 = d_{J+L-1} over the basis of
// k_b_wcoef (d1, d2 hold d_J, d_{J-1} on entry; each element is read and written by one
// thread, so the update is in place).  ring: R slots of `stride` elements.
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_wflush(Seg g, const SV* ring, long stride, int R, const double* cf, int W, SV* d1, SV* d2, SV* e,
           const int* __restrict__ active) {
  constexpr int kMaxB = 130;
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const double* o = cf + rhs * (2 + 3L * (W + 2));
  const long J = (long)o[0];
  const int L = (int)o[1];
  if (L == 0) return;
  __shared__ float cx[kMaxB], c1[kMaxB], c2[kMaxB];
  __shared__ long so[kMaxB];
  for (int b = threadIdx.x; b < L + 2; b += kBlock) {
    cx[b] = (float)o[2 + b];
    c1[b] = (float)o[2 + (W + 2) + b];
    c2[b] = (float)o[2 + 2 * (W + 2) + b];
    so[b] = b >= 2 ? ((J + b - 1) % R) * stride : 0;
  }
  __syncthreads();
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const float2 p2 = sld(d2 + off + i), p1 = sld(d1 + off + i);
    float2 x = c_axpy(cx[1], p1, c_axpy(cx[0], p2, sld(e + off + i)));
    float2 n1 = c_axpy(c1[1], p1, c_scale(p2, c1[0]));
    float2 n2 = c_axpy(c2[1], p1, c_scale(p2, c2[0]));
#pragma unroll 4
    for (int b = 2; b < L + 2; ++b) {
      const float2 v = sld(ring + so[b] + off + i);
      x = c_axpy(cx[b], v, x);
      n1 = c_axpy(c1[b], v, n1);
      n2 = c_axpy(c2[b], v, n2);
    }
    sst(e + off + i, x);
    sst(d1 + off + i, n1);
    sst(d2 + off + i, n2);
  }
}

// x64 += e (FP32 correction)
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_accum(Seg g, double2* x, const SV* e, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const float2 d = sld(e + off + i);
    x[off + i] = make_double2(x[off + i].x + (double)d.x, x[off + i].y + (double)d.y);
  }
}

// x64 += e, then e = 0 and the rhs's state flag cleared: the CGLS reliable update whose
// residual the FP64 stencil stores straight into the low-precision r (k_b_cg_start's other work)
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_accum_clear(Seg g, double2* x, SV* e, double* st, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const float2 d = sld(e + off + i);
    x[off + i] = make_double2(x[off + i].x + (double)d.x, x[off + i].y + (double)d.y);
    sst(e + off + i, make_float2(0.f, 0.f));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st[rhs * NS + B_FLAG] = 0.0;
}

// gamma5 on FP64 fields (batched)
__global__ void __launch_bounds__(kBlock) k_b_gamma5(Seg g, const double2* in, double2* out, const int* active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const int c = (int)((i >> 6) % kSpin);
    const double2 v = in[off + i];
    out[off + i] = c >= 6 ? make_double2(-v.x, -v.y) : v;
  }
}

// ---- CG on the normal equations (CGLS), FP32 inner -----------------------------------
// start: r32 = r64 (FP32), e = 0 ; s and p are formed by the caller (s = M^dag r32, p = s).
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_cg_start(Seg g, const double2* r64, SV* r32, SV* e, double* st, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const double2 x = r64[off + i];
    sst(r32 + off + i, make_float2((float)x.x, (float)x.y));
    sst(e + off + i, make_float2(0.f, 0.f));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) st[rhs * NS + B_FLAG] = 0.0;
}

__global__ void __launch_bounds__(kBlock) k_b_cg_alpha(const double* part, int np, double* st, const int* active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  __shared__ double lds[kBlock / 64];
  const double qq = b_fin_sum(part + (long)r * np, np, lds);
  if (threadIdx.x == 0) {
    double* S = st + r * NS;
    const bool ok = qq > 0.0 && isfinite(qq) && S[B_FLAG] == 0.0;
    S[B_CGA] = ok ? S[B_SS] / qq : 0.0;
    if (!ok) S[B_FLAG] = 1.0;
  }
}

// (E: e += alpha p ;) r -= alpha q ; partial ||r||^2.  Without E the e update waits for
// k_b_cg_xpay of the same iteration, which reads p anyway (one field pass fewer per iteration,
// the same bits: p does not change in between).
template <class SV, bool E>
__global__ void __launch_bounds__(kBlock)
k_b_cg_xr(Seg g, const double* st, const SV* p, const SV* q, SV* e, SV* r, const int* __restrict__ active,
          double* __restrict__ part) {
  const int rhs = blockIdx.y;
  double acc = 0.0;
  if (!active || active[rhs]) {
    const float a = (float)st[rhs * NS + B_CGA];
    const long off = seg_off(g, rhs), n = seg_len(g, rhs);
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
      if (E) sst(e + off + i, c_axpy(a, sld(p + off + i), sld(e + off + i)));
      const float2 v = c_axpy(-a, sld(q + off + i), sld(r + off + i));
      sst(r + off + i, v);
      acc = fma((double)v.x, (double)v.x, fma((double)v.y, (double)v.y, acc));
    }
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[(long)rhs * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
k_b_cg_beta(const double* ps, int nps, const double* pr, int npr, double* st, const int* active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  __shared__ double lds[kBlock / 64];
  const double ss = b_fin_sum(ps + (long)r * nps, nps, lds);
  const double rr = b_fin_sum(pr + (long)r * npr, npr, lds);
  if (threadIdx.x == 0) {
    double* S = st + r * NS;
    const double old = S[B_SS];
    const bool ok = old > 0.0 && isfinite(ss) && S[B_FLAG] == 0.0;
    S[B_CGB] = ok ? ss / old : 0.0;
    if (ok) S[B_SS] = ss;
    else S[B_FLAG] = 1.0;
    S[B_RR] = rr;
  }
}

// (E: e += alpha p, the update k_b_cg_xr<SV, false> left ;) p = s + beta p
template <class SV, bool E>
__global__ void __launch_bounds__(kBlock)
k_b_cg_xpay(Seg g, const double* st, const SV* s, SV* p, SV* e, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const float b = (float)st[rhs * NS + B_CGB];
  const float a = E ? (float)st[rhs * NS + B_CGA] : 0.f;
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const float2 pv = sld(p + off + i);
    if (E) sst(e + off + i, c_axpy(a, pv, sld(e + off + i)));
    sst(p + off + i, c_axpy(b, pv, sld(s + off + i)));
  }
}

// partial ||a||^2 of low-precision fields, column-major [rhs][G]
template <class SV>
__global__ void __launch_bounds__(kBlock)
k_b_norm2_f32(Seg g, const SV* a, const int* __restrict__ active, double* __restrict__ part) {
  const int rhs = blockIdx.y;
  double acc = 0.0;
  if (!active || active[rhs]) {
    const long off = seg_off(g, rhs), n = seg_len(g, rhs);
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
      const float2 v = sld(a + off + i);
      acc = fma((double)v.x, (double)v.x, fma((double)v.y, (double)v.y, acc));
    }
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[(long)rhs * gridDim.x + blockIdx.x] = s;
}

template <class SV>
__global__ void k_b_copy_f32(Seg g, const SV* a, SV* b, const int* active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = seg_off(g, rhs), n = seg_len(g, rhs);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[off + i] = a[off + i];
}

// ---- host driver -------------------------------------------------------------
static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// One operator of a batch and its right-hand sides [r0, r0 + nr).
struct BItem {
  dl_op* op;
  const dl_eig* eig;
  int r0, nr;
  double tol;
};

struct Batch {
  std::vector<BItem> items;
  dl_ctx* ctx;
  int nr;
  hipStream_t s;
  std::vector<long> h_off, h_len;
  DBuf<long> d_off, d_len;
  long total = 0, nmax = 0;
  Seg seg{};
  DBuf<double> st, part, part2;
  DBuf<int> active;
  DBuf<double> invs;  // per-rhs 1/n_j, the Wilson epilogue scale of the unnormalised Lanczos vector
  std::vector<int> h_active;
  std::vector<double> h_st;
  std::vector<int> item_of;  // rhs -> item
  int G;
  // multi-lattice stencil work lists (FP32 and FP64 links)
  DBuf<WilsonItem> wl32, wl64;
  int ml_blocks = 0, ml_pstride = 0;
  // multi-lattice stencil form, chosen by timing at the batch's setup (ml_choose): -1 not yet,
  // 0 one work-list launch over all lattices, 1 one launch per lattice in its tuned shape (fused
  // reductions re-strided from ml_part to pw partials per rhs)
  int ml_mode = -1;
  int pw = 0;
  DBuf<double> ml_part;
  // projection over lowered eigenvectors (eig_prec DL_FP32 / DL_BF16): rA rounded for the
  // matrix-core contraction
  int eig_prec = DL_FP64;
  DBuf<float2> ra32;
  DBuf<bf2> ra16;

  explicit Batch(const std::vector<BItem>& its) : items(its), ctx(its[0].op->ctx), s(its[0].op->ctx->stream) {
    nr = 0;
    for (const auto& it : items) nr += it.nr;
    item_of.resize(nr);
    for (size_t i = 0; i < items.size(); ++i) {
      const BItem& it = items[i];
      for (int r = 0; r < it.nr; ++r) {
        item_of[it.r0 + r] = (int)i;
        h_off.push_back(total);
        h_len.push_back(it.op->lat.nc);
        total += it.op->lat.nc;
      }
      nmax = std::max(nmax, it.op->lat.nc);
    }
    if (single()) {
      seg = Seg{nullptr, nullptr, nmax};
    } else {
      d_off.alloc(nr);
      d_len.alloc(nr);
      DL_HIP(hipMemcpyAsync(d_off.get(), h_off.data(), nr * sizeof(long), hipMemcpyHostToDevice, s));
      DL_HIP(hipMemcpyAsync(d_len.get(), h_len.data(), nr * sizeof(long), hipMemcpyHostToDevice, s));
      seg = Seg{d_off.get(), d_len.get(), nmax};
      build_worklists();
    }
    st.alloc((size_t)nr * NS);
    G = bgrid(nmax);
    int pw = G;
    for (const auto& it : items) pw = std::max(pw, wilson_max_nbs(it.op->lat));
    pw = std::max(pw, ml_pstride);
    const size_t np = (size_t)nr * pw;
    this->pw = pw;
    part.alloc(np);
    part2.alloc(np);
    if (!single()) ml_part.alloc(np);
    active.alloc(nr);
    invs.alloc(nr);
    h_active.assign(nr, 1);
    h_st.resize((size_t)nr * NS);
    static_assert(NS % 2 == 0, "state rows are cleared as double2");
    zero(s, (long)nr * NS / 2, reinterpret_cast<double2*>(st.get()));
    DL_HIP(hipStreamSynchronize(s));
  }
  bool single() const { return items.size() == 1; }
  void build_worklists();
  void push_active() {
    DL_HIP(hipMemcpyAsync(active.get(), h_active.data(), nr * sizeof(int), hipMemcpyHostToDevice, s));
    DL_HIP(hipStreamSynchronize(s));
  }
  void pull_state() {
    DL_HIP(hipMemcpyAsync(h_st.data(), st.get(), h_st.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
  }
  void push_state() {
    DL_HIP(hipMemcpyAsync(st.get(), h_st.data(), h_st.size() * sizeof(double), hipMemcpyHostToDevice, s));
    DL_HIP(hipStreamSynchronize(s));
  }
  double get(int r, int f) const { return h_st[(size_t)r * NS + f]; }
  int n_active() const {
    int a = 0;
    for (int v : h_active) a += v;
    return a;
  }
  // algorithmic stencil bytes of the active rhs: links once per site and lattice, spinors per rhs
  double wilson_bytes(double link_b, double spinor_b) const {
    double b = 0.0;
    for (const auto& it : items) {
      int na = 0;
      for (int r = 0; r < it.nr; ++r) na += h_active[it.r0 + r];
      if (na) b += (double)it.op->lat.V * (link_b + spinor_b * na);
    }
    return b;
  }
};

__global__ void k_f64_to_f32(long n, const double2* a, float2* b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// FP32 copy of the links, made on first use and kept with the operator.
const float2* op_links32_public(dl_op* op) {
  if (!op->U32.get()) {
    op->U32.alloc(op->lat.nl);
    hipLaunchKernelGGL(k_f64_to_f32, dim3(2048), dim3(kBlock), 0, op->ctx->stream, op->lat.nl, op->U.get(),
                       op->U32.get());
    DL_HIP(hipGetLastError());
  }
  return op->U32.get();
}

void Batch::build_worklists() {
  std::vector<WilsonItem> w32, w64;
  int block0 = 0;
  for (const auto& it : items) {
    const Lattice& lat = it.op->lat;
    WilsonItem w{};
    w.kappa = it.op->kappa;
    for (int d = 0; d < 4; ++d) w.L[d] = lat.L[d];
    w.V = lat.V;
    w.Vpad = lat.ntiles * kTile;
    w.rhs0 = it.r0;
    w.nrhs = it.nr;
    w.nbs = (int)((lat.V + 255) / 256);
    w.block0 = block0;
    block0 += w.nbs * w.nrhs;
    ml_pstride = std::max(ml_pstride, w.nbs);
    w.U = op_links32_public(it.op);
    w32.push_back(w);
    w.U = it.op->U.get();
    w64.push_back(w);
  }
  if (ml_pstride > kMaxPartials) fail(DL_E_INVALID, "lattice too large for fused reduction");
  ml_blocks = block0;
  wl32.alloc(w32.size());
  wl64.alloc(w64.size());
  DL_HIP(hipMemcpyAsync(wl32.get(), w32.data(), w32.size() * sizeof(WilsonItem), hipMemcpyHostToDevice, s));
  DL_HIP(hipMemcpyAsync(wl64.get(), w64.data(), w64.size() * sizeof(WilsonItem), hipMemcpyHostToDevice, s));
  DL_HIP(hipStreamSynchronize(s));
}

// One lattice's fused-reduction partials (nbs per rhs, column-major) into the batch layout of
// pw partials per rhs, zero beyond nbs, so that one reduction serves every lattice.
__global__ void k_restride_partials(const double* __restrict__ src, int nbs, int nr, double* __restrict__ dst,
                                    int pw) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)nr * pw) return;
  const int r = (int)(i / pw), sb = (int)(i % pw);
  dst[i] = sb < nbs ? src[(long)r * nbs + sb] : 0.0;
}

// The multi-lattice stencil in form `mode` (0 work list, 1 per lattice in its tuned shape); the
// lattices' fields are consecutive in the batch, lattice i's rhs at [r0, r0 + nr).  Returns the
// partial stride per rhs of the fused reduction.
template <class R, class SV>
static int bwilson_multi(Batch& bt, int mode, int which, const SV* in, SV* out, int red, double* part,
                         const double* scale) {
  constexpr int prec = sizeof(R) == 8 ? DL_FP64 : sizeof(SV) == sizeof(float2) ? DL_FP32 : DL_BF16;
  if (mode == 0) {
    wilson_multi<R>(bt.s, sizeof(R) == 8 ? bt.wl64.get() : bt.wl32.get(), (int)bt.items.size(), bt.ml_blocks,
                    bt.ml_pstride, which, in, out, bt.d_off.get(), red, scale, bt.active.get(), part);
    return red ? bt.ml_pstride : 0;
  }
  for (const auto& it : bt.items) {
    dl_op* op = it.op;
    const long off = bt.h_off[it.r0];
    double* ip = red ? bt.ml_part.get() + (size_t)it.r0 * bt.pw : nullptr;
    const cplx_t<R>* U;
    if constexpr (sizeof(R) == 8) U = op->U.get();
    else U = op_links32_public(op);
    const int nbs = wilson_batched<R>(bt.s, op->lat, U, op->kappa, which, in + off, out + off, op->lat.nc, it.nr, red,
                                      scale ? scale + it.r0 : nullptr, bt.active.get() + it.r0, ip,
                                      wilson_cfg(op, prec, it.nr));
    if (red) {
      if (nbs > bt.pw) fail(DL_E_INVALID, "stencil partials exceed the batch's partial stride");
      const long n = (long)it.nr * bt.pw;
      hipLaunchKernelGGL(k_restride_partials, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, bt.s, ip, nbs, it.nr,
                         part + (size_t)it.r0 * bt.pw, bt.pw);
    }
  }
  return red ? bt.pw : 0;
}

// Chooses the multi-lattice stencil form at the batch's setup, outside any graph capture: the
// per-lattice shapes (storage precision and FP64) are settled first, so that no captured
// block tunes, then both forms of the M apply are timed on zeroed temporary fields (3 applies
// each after a warm-up) and the faster is kept for the batch's lifetime (so the partial
// stride a solve reads stays the same).  DEFLAN_MULTI_STENCIL=list or =lattice forces a form;
// with autotuning off the work list is taken.
template <class SV>
static int ml_choose(Batch& bt) {
  constexpr int prec = sizeof(SV) == sizeof(float2) ? DL_FP32 : DL_BF16;
  const char* e = std::getenv("DEFLAN_MULTI_STENCIL");
  if (e && std::strcmp(e, "list") == 0) return 0;
  for (const auto& it : bt.items) {
    (void)wilson_cfg(it.op, prec, it.nr);
    (void)wilson_cfg(it.op, DL_FP64, it.nr);
  }
  if (e && std::strcmp(e, "lattice") == 0) return 1;
  if (!autotune_enabled()) return 0;
  // two fields of bt.total SV elements, allocated as double2 (16 B) and zeroed
  const long nd = (long)((bt.total * (long)sizeof(SV) + 15) / 16);
  DBuf<double2> tin, tout;
  tin.alloc((size_t)nd);
  tout.alloc((size_t)nd);
  zero(bt.s, nd, tin.get());
  const SV* in = reinterpret_cast<const SV*>(tin.get());
  SV* out = reinterpret_cast<SV*>(tout.get());
  bt.push_active();
  hipEvent_t a, b;
  DL_HIP(hipEventCreate(&a));
  DL_HIP(hipEventCreate(&b));
  float ms[2] = {0.f, 0.f};
  for (int m = 0; m < 2; ++m) {
    bwilson_multi<float, SV>(bt, m, 0, in, out, 0, nullptr, nullptr);
    DL_HIP(hipEventRecord(a, bt.s));
    for (int rep = 0; rep < 3; ++rep) bwilson_multi<float, SV>(bt, m, 0, in, out, 0, nullptr, nullptr);
    DL_HIP(hipEventRecord(b, bt.s));
    DL_HIP(hipEventSynchronize(b));
    DL_HIP(hipEventElapsedTime(&ms[m], a, b));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  const int mode = ms[1] < ms[0] ? 1 : 0;
  if (verbose()) {
    std::fprintf(stderr, "[deflan] multi-lattice stencil (%d lattices, %d rhs): work list %.1f us, per-lattice tuned "
                 "launches %.1f us -> %s\n", (int)bt.items.size(), bt.nr, 1e3 * ms[0] / 3, 1e3 * ms[1] / 3,
                 mode ? "per lattice" : "work list");
    std::fflush(stderr);
  }
  return mode;
}

// Low-precision stencil over the whole batch (FP32 arithmetic and links; spinors stored as SV:
// float2 or bf2); returns the partial stride per rhs of the fused reduction.
template <class SV>
static int bwilson_lo(Batch& bt, int which, const SV* in, SV* out, int red, double* part,
                      const double* scale = nullptr) {
  constexpr int prec = sizeof(SV) == sizeof(float2) ? DL_FP32 : DL_BF16;
  TimeScope ts(bt.ctx, T_WILSON, bt.wilson_bytes(288.0, 2.0 * kSpin * sizeof(SV)));
  if (bt.single()) {
    dl_op* op = bt.items[0].op;
    const WilsonCfg cfg = wilson_cfg(op, prec, bt.nr);
    return wilson_batched<float>(bt.s, op->lat, op_links32_public(op), op->kappa, which, in, out, op->lat.nc, bt.nr,
                                 red, scale, bt.active.get(), part, cfg);
  }
  return bwilson_multi<float, SV>(bt, bt.ml_mode == 1 ? 1 : 0, which, in, out, red, part, scale);
}

static void bwilson64(Batch& bt, int which, const double2* in, double2* out) {
  TimeScope ts(bt.ctx, T_WILSON64, bt.wilson_bytes(576.0, 384.0));
  if (bt.single()) {
    dl_op* op = bt.items[0].op;
    const WilsonCfg cfg = wilson_cfg(op, DL_FP64, bt.nr);
    wilson_batched<double>(bt.s, op->lat, op->U.get(), op->kappa, which, in, out, op->lat.nc, bt.nr, 0, nullptr,
                           bt.active.get(), nullptr, cfg);
    return;
  }
  // the FP64 applies follow the form chosen at the batch's setup
  bwilson_multi<double, double2>(bt, bt.ml_mode == 1 ? 1 : 0, which, in, out, 0, nullptr, nullptr);
}

// r64 = b - M x64 for active rhs (x_zero: x64 = 0, r64 = b without the stencil); refreshes
// st[B_RR], st[B_NRM], st[B_INV].
static void true_residual(Batch& bt, const double2* B, const double2* X, double2* R, double2* T,
                          bool x_zero = false) {
  dl_op* op0 = bt.items[0].op;
  if (!x_zero && bt.single() && !op0->lat.eo) {
    // one whole-lattice operator: the FP64 stencil forms r = b - M x and ||r||^2 itself
    int nbs;
    {
      TimeScope ts(bt.ctx, T_WILSON64, bt.wilson_bytes(576.0, 576.0));  // reads x and b, writes r
      nbs = wilson_residual_f64(bt.s, op0->lat, op0->U.get(), op0->kappa, X, B, R, op0->lat.nc, bt.nr,
                                bt.active.get(), bt.part.get());
    }
    hipLaunchKernelGGL(k_b_fin_store, dim3(bt.nr), dim3(kBlock), 0, bt.s, bt.part.get(), nbs, bt.st.get(),
                       (int)B_RR);
    DL_HIP(hipGetLastError());
    return;
  }
  if (!x_zero) bwilson64(bt, 0, X, T);
  hipLaunchKernelGGL(k_b_resid, dim3(bt.G, bt.nr), dim3(kBlock), 0, bt.s, bt.seg, B, x_zero ? nullptr : T, R,
                     bt.active.get(), bt.part.get());
  hipLaunchKernelGGL(k_b_fin_store, dim3(bt.nr), dim3(kBlock), 0, bt.s, bt.part.get(), bt.G, bt.st.get(),
                     (int)B_RR);
  DL_HIP(hipGetLastError());
}

// The projection over lowered eigenvectors: rA (FP64, in T) is rounded to the contraction's
// storage, c = Yc^H rA on the matrix cores (Yc = Y16 for BF16, Y32 for FP32; FP32 accumulation,
// FP64 partials), d = H32^-1 c in FP64, and x += Y32 d in FP64 arithmetic.  The Galerkin basis
// is Y32 with its own Gram matrix, so the correction is the exact projection onto span(Y32);
// the contraction's rounding only perturbs c, by about eps * ||rA|| / sqrt(n) per entry.
static void project_batch_lowp(Batch& bt, double2* X, const double2* T, DBuf<double2>& cbuf, Scratch& S) {
  constexpr int kCols = 16, kRows = 128;
  const bool b16 = bt.eig_prec == DL_BF16;
  if (b16) {
    if (bt.ra16.n < (size_t)bt.total) bt.ra16.alloc(bt.total);
    round_bf16(bt.s, bt.total, T, bt.ra16.get());
  } else {
    if (bt.ra32.n < (size_t)bt.total) bt.ra32.alloc(bt.total);
    round_f32(bt.s, bt.total, T, bt.ra32.get());
  }
  S.ensure_part((size_t)2 * kRows * kCols * tsk_lowp_nblocks(bt.nmax, bt.eig_prec) + 64);
  for (const auto& it : bt.items) {
    if (!it.eig || it.eig->k == 0) continue;
    const dl_eig* e = it.eig;
    if (e->lo_prec == DL_FP64 || (b16 && e->lo_prec != DL_BF16))
      fail(DL_E_INVALID, "eigenvector handle not lowered to the requested storage");
    const int k = e->k;
    const long n = it.op->lat.nc;
    int nact = 0;
    for (int r = it.r0; r < it.r0 + it.nr; ++r) nact += bt.h_active[r];
    if (!nact) continue;
    for (int c0 = 0; c0 < it.nr; c0 += kCols) {
      const int nw = std::min(kCols, it.nr - c0);
      const int* act = bt.active.get() + it.r0 + c0;
      const long off = bt.h_off[it.r0 + c0];
      for (int j0 = 0; j0 < k; j0 += kRows) {
        const int nv = std::min(kRows, k - j0);
        int np;
        {
          TimeScope ts(bt.ctx, T_TSK_DOTS);
          np = b16 ? tsk_dots_lowp(bt.s, n, nv, e->Y16.get() + (long)j0 * n, n, bt.ra16.get() + off, n, nw, act,
                                   S.part.get())
                   : tsk_dots_lowp(bt.s, n, nv, e->Y32.get() + (long)j0 * n, n, bt.ra32.get() + off, n, nw, act,
                                   S.part.get());
        }
        for (int r = 0; r < nw; ++r)
          sum_partials(bt.s, S.part.get() + (size_t)2 * r * nv * np, np, 2 * nv,
                       reinterpret_cast<double*>(cbuf.get() + (long)(c0 + r) * k + j0));
      }
    }
    {
      TimeScope ts(bt.ctx, T_SMALL);
      proj_solve(bt.s, k, it.nr, e->Zr32.get(), e->lamr32.get(), cbuf.get(), cbuf.get() + (long)it.nr * k);
    }
    for (int c0 = 0; c0 < it.nr; c0 += kCols) {
      const int nw = std::min(kCols, it.nr - c0);
      TimeScope ts(bt.ctx, T_TSK_UPDATE);
      tsk_update_multi32(bt.s, n, k, e->Y32.get(), n, cbuf.get() + (long)it.nr * k + (long)c0 * k, nw,
                         bt.active.get() + it.r0 + c0, X + bt.h_off[it.r0 + c0], n);
    }
  }
}

// Galerkin projection over each item's eigenvectors for every active rhs: x += Y H^-1 Y^H rA,
// rA = gamma5 r (G5M) or M^dag r (MDAGM).  T: scratch (a batch of fields).
static void project_batch(Batch& bt, const double2* R, double2* X, double2* T, DBuf<double2>& cbuf, Scratch& S) {
  bool any = false;
  for (const auto& it : bt.items) any |= it.eig && it.eig->k > 0;
  if (!any) return;
  if (bt.items[0].op->kind == DL_G5M)
    hipLaunchKernelGGL(k_b_gamma5, dim3(bt.G, bt.nr), dim3(kBlock), 0, bt.s, bt.seg, R, T, bt.active.get());
  else
    bwilson64(bt, 1, R, T);
  // c = Y^H rA and x += Y d for up to 16 rhs per launch, so the eigenvectors stream once per
  // 16 rhs instead of once per rhs (the rhs of one item are contiguous at stride n)
  constexpr int kCols = 16, kRows = 64;
  if (bt.eig_prec != DL_FP64) {
    project_batch_lowp(bt, X, T, cbuf, S);
    return;
  }
  S.ensure_part((size_t)2 * kRows * kCols * tsk_multi_nblocks(bt.nmax) + 64);
  for (const auto& it : bt.items) {
    if (!it.eig || it.eig->k == 0) continue;
    dl_op* op = it.op;
    const int k = it.eig->k;
    const long n = op->lat.nc;
    int nact = 0;
    for (int r = it.r0; r < it.r0 + it.nr; ++r) nact += bt.h_active[r];
    if (!nact) continue;
    const double2* Y = it.eig->Y.get();
    for (int c0 = 0; c0 < it.nr; c0 += kCols) {
      const int nw = std::min(kCols, it.nr - c0);
      const int* act = bt.active.get() + it.r0 + c0;
      for (int j0 = 0; j0 < k; j0 += kRows) {
        const int nv = std::min(kRows, k - j0);
        int np;
        {
          TimeScope ts(bt.ctx, T_TSK_DOTS);
          np = tsk_dots_multi(bt.s, n, nv, Y + (long)j0 * n, n, T + bt.h_off[it.r0 + c0], n, nw, act, S.part.get());
        }
        for (int r = 0; r < nw; ++r)
          sum_partials(bt.s, S.part.get() + (size_t)2 * r * nv * np, np, 2 * nv,
                       reinterpret_cast<double*>(cbuf.get() + (long)(c0 + r) * k + j0));
      }
    }
    {
      TimeScope ts(bt.ctx, T_SMALL);
      proj_solve(bt.s, k, it.nr, it.eig->Zr.get(), it.eig->lamr.get(), cbuf.get(), cbuf.get() + (long)it.nr * k);
    }
    for (int c0 = 0; c0 < it.nr; c0 += kCols) {
      const int nw = std::min(kCols, it.nr - c0);
      TimeScope ts(bt.ctx, T_TSK_UPDATE);
      tsk_update_multi(bt.s, n, k, Y, n, cbuf.get() + (long)it.nr * k + (long)c0 * k, nw,
                       bt.active.get() + it.r0 + c0, X + bt.h_off[it.r0 + c0], n);
    }
  }
}

// Instantiated graphs of launch sequences, keyed by a small id; captured from the stream on
// first use and replayed after.  The captured sequences contain kernel launches only.
struct GraphCache {
  hipStream_t s;
  std::map<int, hipGraphExec_t> exec;
  std::map<int, hipGraph_t> graph;
  explicit GraphCache(hipStream_t st) : s(st) {}
  template <class F>
  void run(int id, F&& enqueue) {
    auto it = exec.find(id);
    if (it == exec.end()) {
      hipGraph_t gr = nullptr;
      DL_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      try {
        enqueue();
      } catch (...) {
        (void)hipStreamEndCapture(s, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      DL_HIP(hipStreamEndCapture(s, &gr));
      hipGraphExec_t ex = nullptr;
      const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(gr);
        DL_HIP(e);
      }
      graph[id] = gr;
      it = exec.emplace(id, ex).first;
    }
    DL_HIP(hipGraphLaunch(it->second, s));
  }
  void clear() {
    if (!exec.empty()) (void)hipStreamSynchronize(s);
    for (auto& kv : exec) (void)hipGraphExecDestroy(kv.second);
    for (auto& kv : graph) (void)hipGraphDestroy(kv.second);
    exec.clear();
    graph.clear();
  }
  ~GraphCache() { clear(); }
};

// The batched solve over a list of operators.  B, X: all fields of the batch, field r at
// h_off[r] (tiled FP64).  net: learned initial guess (single operator only).
static int solve_batch(const std::vector<BItem>& items, const double2* B, double2* X, const dl_next_opts& o,
                       dl_stats* st, History* hist) {
  const double t0 = now_s();
  Batch bt(items);
  const int nr = bt.nr;
  hipStream_t s = bt.s;
  bt.eig_prec = o.eig_storage;
  // On M^dag M the coefficients are divided by lambda(M^dag M) = sigma^2 while the M-residual
  // multiplies them back by sigma only, so the contraction's error reaches the residual
  // amplified by 1/sigma_min(M); BF16 is too coarse for that near criticality.
  if (bt.eig_prec == DL_BF16 && items[0].op->kind == DL_MDAGM)
    fail(DL_E_INVALID, "the BF16 contraction serves the gamma5 M form; use DL_FP32 eigenvectors with M^dag M");
  // a handle lowered to BF16 also holds the FP32 basis, so it serves both
  if (bt.eig_prec != DL_FP64)
    for (const auto& it : items)
      if (it.eig && it.eig->k > 0 && it.eig->lo_prec != bt.eig_prec &&
          !(bt.eig_prec == DL_FP32 && it.eig->lo_prec == DL_BF16))
        fail(DL_E_INVALID, "eigenvector handle not lowered to the requested storage (dl_eig_lower)");
  // everything a captured block could allocate or tune is settled first: the FP32 links and
  // the stencil launch shapes (tuning launches kernels and allocates)
  for (const auto& it : items) (void)op_links32_public(it.op);
  if (bt.single()) {
    (void)wilson_cfg(items[0].op, o.storage == DL_BF16 ? DL_BF16 : DL_FP32, nr);
    (void)wilson_cfg(items[0].op, DL_FP64, nr);
  } else {
    bt.ml_mode = o.storage == DL_BF16 ? ml_choose<bf2>(bt) : ml_choose<float2>(bt);
  }
  const bool mr = items[0].op->kind == DL_G5M;
  int kmax = 1;
  for (const auto& it : items) kmax = std::max(kmax, it.eig ? it.eig->k : 1);
  int nrmax = 1;
  for (const auto& it : items) nrmax = std::max(nrmax, it.nr);
  Scratch S;
  S.sc.alloc(256);
  S.ensure_part((size_t)2 * kmax * tsk_nblocks(bt.nmax) + 64);
  DBuf<double2> R64((size_t)bt.total), T64((size_t)bt.total);
  // low-precision Krylov vectors: FP32 or BF16 storage (FP32 arithmetic either way)
  bool bf16 = o.storage == DL_BF16;  // BF16 storage; a stalled BF16 cycle moves the batch to FP32
  DBuf<float2> f[6];
  DBuf<bf2> h[6];
  for (int q = 0; q < 6; ++q) {
    if (bf16) h[q].alloc((size_t)bt.total);
    else f[q].alloc((size_t)bt.total);
  }
  DBuf<double2> cbuf(2 * (size_t)nrmax * kmax + 2);
  // windowed MinRes (without graph capture): the ring of Lanczos vectors (W + 2 fields per
  // rhs; W from 64 down to 8 while the ring exceeds 24 GiB), the recorded rotations and the
  // window coefficients
  DBuf<float2> ring32;
  DBuf<bf2> ring16;
  DBuf<double> wrot((size_t)nr * kMaxWindow * 5), wcf((size_t)nr * (2 + 3 * (kMaxWindow + 2)));
  std::vector<long> iters(nr, 0), mvp(nr, 0);
  std::vector<double> bnorm(nr), rel(nr, 1.0), tol(nr);
  for (int r = 0; r < nr; ++r) tol[r] = items[bt.item_of[r]].tol;
  // ||b|| per right-hand side (FP64)
  {
    std::vector<double> h(nr);
    for (int r = 0; r < nr; ++r) {
      const int nb = norm2_partials(s, bt.h_len[r], B + bt.h_off[r], S.part.get());
      sum_partials(s, S.part.get(), nb, 1, S.sc.get() + r % 256);
      if (r % 256 == 255 || r == nr - 1) {
        const int cnt = r % 256 + 1;
        DL_HIP(hipMemcpyAsync(h.data() + (r - cnt + 1), S.sc.get(), cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        DL_HIP(hipStreamSynchronize(s));
      }
    }
    for (int r = 0; r < nr; ++r) {
      if (!std::isfinite(h[r])) fail(DL_E_NONFINITE, "right-hand side contains NaN or Inf");
      bnorm[r] = std::sqrt(h[r]);
    }
  }
  if (!o.x0_given) zero(s, bt.total, X);
  for (int r = 0; r < nr; ++r) {
    if (bnorm[r] == 0.0) {
      bt.h_active[r] = 0;
      zero(s, bt.h_len[r], X + bt.h_off[r]);
      rel[r] = 0.0;
    }
  }
  bt.push_active();
  // FP64 true residual, projection, FP64 true residual again (X in place, R: its residual)
  bool any_eig = false;
  for (const auto& it : items) any_eig |= it.eig && it.eig->k > 0;
  auto start = [&](double2* Xs, double2* Rs, bool x_zero) {
    true_residual(bt, B, Xs, Rs, T64.get(), x_zero);
    if (!x_zero)
      for (int r = 0; r < nr; ++r) mvp[r] += bt.h_active[r];
    project_batch(bt, Rs, Xs, T64.get(), cbuf, S);
    if (any_eig) {
      for (int r = 0; r < nr; ++r) mvp[r] += bt.h_active[r] * (mr ? 0 : 1);
      true_residual(bt, B, Xs, Rs, T64.get());
      for (int r = 0; r < nr; ++r) mvp[r] += bt.h_active[r];
    }
  };
  std::vector<int> used_net(nr, 0);
  bool started = false;
  if (o.net && bt.n_active() > 0) {
    // Learned initial guess: start from net(b) + projection or from the projection alone,
    // whichever has the smaller FP64 true residual.
    if (!bt.single()) fail(DL_E_INVALID, "the learned initial guess takes one operator per batch");
    dl_op* op = items[0].op;
    dl_net* net = o.net;
    if (net->ctx != op->ctx) fail(DL_E_INVALID, "network and operator belong to different contexts");
    start(X, R64.get(), !o.x0_given);
    bt.pull_state();
    std::vector<double> rp(nr);
    for (int r = 0; r < nr; ++r) rp[r] = bt.get(r, B_NRM);
    DBuf<double2> XN((size_t)bt.total), RN((size_t)bt.total);
    net_apply(net, op, nr, B, XN.get(), o.net_prec == DL_BF16);
    start(XN.get(), RN.get(), false);
    bt.pull_state();
    // keep the better start per rhs, with its residual and residual state
    for (int r = 0; r < nr; ++r) {
      if (!bt.h_active[r]) continue;
      if (bt.get(r, B_NRM) < rp[r]) {
        used_net[r] = 1;
        copy(s, bt.h_len[r], XN.get() + bt.h_off[r], X + bt.h_off[r]);
        copy(s, bt.h_len[r], RN.get() + bt.h_off[r], R64.get() + bt.h_off[r]);
      } else {
        bt.h_st[(size_t)r * NS + B_NRM] = rp[r];
        bt.h_st[(size_t)r * NS + B_RR] = rp[r] * rp[r];
        bt.h_st[(size_t)r * NS + B_INV] = rp[r] > 0.0 ? 1.0 / rp[r] : 0.0;
      }
    }
    bt.push_state();
    started = true;
    if (verbose()) {
      int cnt = 0;
      for (int r = 0; r < nr; ++r) cnt += used_net[r];
      std::fprintf(stderr, "[deflan] learned guess kept for %d/%d rhs (%.2fs)\n", cnt, nr, now_s() - t0);
      std::fflush(stderr);
    }
  }
  // Per-cycle residual drop and D-CG reliable-update interval; 0 in the options = the default
  // for the storage and solver.  BF16 rounding limits what a MinRes cycle can reach, so BF16
  // D-MinRes cycles end at 1e-2.  BF16 D-CG keeps its search direction through FP64 residual
  // replacements every 8 iterations and runs 1e-5 cycles from the projection-only start, 1e-3
  // cycles from a learned start.  On near-critical Wilson fields (min|lambda(gamma5 M)| = 1e-3,
  // M^dag M, tol 1e-10) 1e-5 cycles took 272 iterations per rhs on 16^3x32 (1e-3: 288), 400 on
  // 24^3x48 (1e-3: 408) and 8% less time on a batch of four lattices from 8^4 to 20^3x40; each
  // cycle start costs an FP64 residual and a projection and discards the Krylov space.  Longer
  // cycles lose: at 1e-6, or with no restarts, the 16^3x32 field needed 464-479 iterations, as
  // BF16 rounding brings the deflated low modes back and only the projection removes them
  // cheaply.  From the learned start on the same fields 1e-3 cycles took 264.6 iterations, 1e-4
  // 275, 3e-5 272 and 1e-5 280.  With 1e-2 cycles and updates every 50 the 24^3x48 field took
  // 1662.  A batch that falls back from BF16 to FP32 takes the FP32 defaults for the values the
  // caller left at 0 and keeps the ones it set.
  const bool drop_default = o.inner_drop == 0.0, rel_default = o.reliable_every == 0;
  const bool bf16_cg = o.storage == DL_BF16 && !mr;
  double inner_drop =
      drop_default ? (o.storage == DL_BF16 ? (bf16_cg ? (o.net ? 1e-3 : 1e-5) : 1e-2) : 1e-4) : o.inner_drop;
  int rel_opt = rel_default ? (bf16_cg ? 8 : 50) : o.reliable_every;
  bool stalled_any = false;
  const int check = 8;                 // iterations between host checks (even)
  const Seg g = bt.seg;
  // Graph replay of the `check`-iteration blocks: off while kernel timing is on (its events
  // would be captured) and on the legacy null stream (which cannot be captured).
  const bool use_graph = o.graph != 0 && !bt.ctx->timers.enabled && s != nullptr;
  GraphCache graphs(s);
  for (int cycle = 0; cycle < 40 && bt.n_active() > 0; ++cycle) {
    if (!(cycle == 0 && started)) start(X, R64.get(), cycle == 0 && !o.x0_given);
    bt.pull_state();
    for (int r = 0; r < nr; ++r) {
      if (!bt.h_active[r]) continue;
      rel[r] = bt.get(r, B_NRM) / bnorm[r];
      if (!std::isfinite(rel[r])) fail(DL_E_NONFINITE, "non-finite residual");
      if (hist) hist->add(r, (double)mvp[r], rel[r]);
      if (rel[r] <= tol[r] || mvp[r] >= o.max_mvp) bt.h_active[r] = 0;
    }
    bt.push_active();
    if (verbose()) {
      double worst_rel = 0.0;
      long itmax = 0;
      for (int r = 0; r < nr; ++r) {
        worst_rel = std::max(worst_rel, rel[r]);
        itmax = std::max(itmax, iters[r]);
      }
      std::fprintf(stderr, "[deflan] batched cycle %d: %d/%d rhs active, worst relres %.3e, max iters %ld (%.2fs)\n",
                   cycle, bt.n_active(), nr, worst_rel, itmax, now_s() - t0);
      std::fflush(stderr);
    }
    if (bt.n_active() == 0) break;
    // Inner target: a cycle ends after an inner_drop reduction of the residual estimate and the
    // next one restarts from the FP64 residual with a fresh projection over the eigenvectors.
    // Running the FP32 recurrence on to tol with reliable updates alone, without re-projection,
    // took 1.7x the iterations of this scheme on the 4^4 near-critical field: FP32 rounding
    // feeds the deflated low modes back in and only the projection removes them cheaply.
    // Within a cycle, CG replaces its residual by the FP64 one every reliable_every iterations
    // and keeps its search direction (a reliable update).
    const bool reliable = !mr && rel_opt > 0;
    std::vector<double> target(nr);
    for (int r = 0; r < nr; ++r) target[r] = std::max(inner_drop * bt.get(r, B_NRM), 0.5 * tol[r] * bnorm[r]);
    std::vector<int> inner_active = bt.h_active;
    const int G = bt.G;
    // the inner solve for storage SV (the pointers of the six vector buffers)
    auto inner = [&](auto* f0, auto* f1, auto* f2, auto* f3, auto* f4, auto* f5) {
    using SV = std::remove_pointer_t<decltype(f0)>;
    if (mr) {
      SV *u = f0, *up = f1, *w = f2, *d1 = f3, *d2 = f4, *e = f5;
      // Without graph capture the MinRes runs windowed (Lanczos vectors kept in a ring, the
      // solution formed every W iterations); graphs replay the fused form, whose launch
      // sequence repeats every two iterations.
      const bool windowed = !use_graph && o.minres_window >= 0;
      int W = o.minres_window > 0 ? std::min(o.minres_window, kMaxWindow) : kMaxWindow;
      SV* ring = nullptr;
      if (windowed) {
        if (o.minres_window == 0)
          while (W > 8 && (size_t)(W + 2) * bt.total * sizeof(SV) > (size_t(24) << 30)) W /= 2;
        const size_t need = (size_t)(W + 2) * bt.total;
        if constexpr (std::is_same_v<SV, bf2>) {
          if (ring16.n != need) ring16.alloc(need);
          ring = ring16.get();
        } else {
          if (ring32.n != need) ring32.alloc(need);
          ring = ring32.get();
        }
      }
      const int R = W + 2;
      auto slot = [&](long j) { return ring + (j % R) * (long)bt.total; };
      hipLaunchKernelGGL((k_b_minres_start<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, R64.get(),
                         windowed ? slot(1) : u, windowed ? slot(0) : up, d1, d2, e, bt.st.get(), bt.invs.get(),
                         bt.active.get());
      auto flush = [&]() {
        hipLaunchKernelGGL(k_b_wcoef, dim3(nr), dim3(128), 0, s, bt.st.get(), wrot.get(), W, wcf.get(),
                           bt.active.get());
        hipLaunchKernelGGL((k_b_wflush<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, ring, (long)bt.total, R,
                           wcf.get(), W, d1, d2, e, bt.active.get());
      };
      long wit = 0;  // iterations of this cycle (windowed form)
      auto iteration_w = [&]() {
        SV* uc = slot(wit + 1);
        const int nbs = bwilson_lo(bt, 2, uc, w, 2, bt.part.get(), bt.invs.get());
        hipLaunchKernelGGL((k_b_lanczos_w<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, bt.st.get(), uc, slot(wit), w,
                           slot(wit + 2), bt.active.get(), bt.part.get(), nbs, bt.part2.get());
        hipLaunchKernelGGL(k_b_fin_rot, dim3(nr), dim3(kBlock), 0, s, bt.part2.get(), G, bt.st.get(), bt.invs.get(),
                           bt.active.get(), wrot.get(), W);
        DL_HIP(hipGetLastError());
        if (++wit % W == 0) flush();
      };
      // one MinRes iteration; `check` (even) iterations return u, up, d1, d2 to their places,
      // so a block of them is the same launch sequence every time (replayed as a graph).  The
      // solution update of an iteration runs in the next iteration's Lanczos pass; an rhs stops
      // only at a check, after an even number of iterations, so its buffers keep their roles
      // and its last update is applied after the loop.
      auto iteration = [&]() {
        const int nbs = bwilson_lo(bt, 2, u, w, 2, bt.part.get(), bt.invs.get());
        hipLaunchKernelGGL((k_b_lanczos_minres<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, bt.st.get(), u, up, w, d1,
                           d2, e, bt.active.get(), bt.part.get(), nbs, bt.part2.get());
        hipLaunchKernelGGL(k_b_fin_rot, dim3(nr), dim3(kBlock), 0, s, bt.part2.get(), G, bt.st.get(), bt.invs.get(),
                           bt.active.get());
        DL_HIP(hipGetLastError());
        std::swap(d1, d2);
        std::swap(u, up);
      };
      // Host checks (a device-to-host copy and a wait) fall at multiples of `check`; the next
      // one is scheduled from each active rhs's residual decay since its previous check: at
      // 3/4 of the fewest iterations any of them needs to reach its target, between `check`
      // and 8 * `check` iterations ahead (and not past an MVP cap).
      std::vector<double> eta_prev(nr), mr_best(nr);
      std::vector<long> it_prev(nr, 0), mr_best_it(nr, 0);
      constexpr long kStallMR = 25L * check;
      for (int r = 0; r < nr; ++r) eta_prev[r] = mr_best[r] = bt.get(r, B_NRM);
      long next_check = check;
      for (int it = 0; it < 100000; ++it) {
        if (use_graph) {
          if (it % check == 0) graphs.run(0, [&] { for (int q = 0; q < check; ++q) iteration(); });
        } else if (windowed) {
          iteration_w();
        } else {
          iteration();
        }
        for (int r = 0; r < nr; ++r) {
          iters[r] += bt.h_active[r];
          mvp[r] += bt.h_active[r];
        }
        if (it + 1 == next_check) {
          bt.pull_state();
          bool changed = false;
          double kmin = 8.0 * check;
          for (int r = 0; r < nr; ++r) {
            if (!bt.h_active[r]) continue;
            const double eta = std::fabs(bt.get(r, B_ETA));
            if (hist) hist->add(r, (double)mvp[r], eta / bnorm[r]);
            // with BF16 storage a cycle also ends when eta has not reached a new low (by 10%)
            // for kStall iterations (the rounding can hold it above the cycle's target)
            if (eta < 0.9 * mr_best[r]) {
              mr_best[r] = eta;
              mr_best_it[r] = it + 1;
            }
            const bool stalled = bf16 && it + 1 - mr_best_it[r] >= kStallMR && eta > target[r];
            stalled_any |= stalled;
            if (eta <= target[r] || stalled || bt.get(r, B_FLAG) != 0.0 || mvp[r] >= o.max_mvp) {
              bt.h_active[r] = 0;
              changed = true;
              continue;
            }
            double k = check;
            if (eta < eta_prev[r] && eta_prev[r] > 0.0) {
              const double rate = std::log(eta / eta_prev[r]) / (double)(it + 1 - it_prev[r]);
              k = std::log(target[r] / eta) / rate;
            }
            k = std::min(k, (double)(o.max_mvp - mvp[r]));
            kmin = std::min(kmin, k);
            eta_prev[r] = eta;
            it_prev[r] = it + 1;
          }
          if (changed) bt.push_active();
          if (bt.n_active() == 0) break;
          const long ahead = (long)(0.75 * kmin) / check * check;
          next_check = it + 1 + std::max<long>(check, std::min<long>(ahead, 8L * check));
        }
      }
      bt.h_active = inner_active;
      bt.push_active();
      if (windowed) {
        flush();  // every rhs's open window (rhs that stopped early keep theirs in the ring)
      } else {
        // the last iteration's solution update (its rotation is still in the state)
        hipLaunchKernelGGL((k_b_minres_update<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, bt.st.get(), up, d1, d2, d2,
                           e, bt.active.get());
      }
      hipLaunchKernelGGL((k_b_accum<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, X, e, bt.active.get());
    } else {
      SV *r32 = f0, *sv = f1, *p = f2, *q = f3, *e = f4;
      (void)f5;
      hipLaunchKernelGGL((k_b_cg_start<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, R64.get(), r32, e, bt.st.get(),
                         bt.active.get());
      const int nbs = bwilson_lo(bt, 1, r32, sv, 1, bt.part.get());
      hipLaunchKernelGGL(k_b_fin_store, dim3(nr), dim3(kBlock), 0, s, bt.part.get(), nbs, bt.st.get(), (int)B_SS);
      hipLaunchKernelGGL((k_b_copy_f32<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, sv, p, bt.active.get());
      for (int r = 0; r < nr; ++r) mvp[r] += bt.h_active[r];
      // With graphs, reliable updates fall on the last iteration of every `rel_blocks`-th block.
      const int rel_every = !reliable ? 0
                            : use_graph ? check * std::max(1, (rel_opt + check / 2) / check)
                                        : rel_opt;
      auto iteration = [&](bool update) {
        bwilson_lo(bt, 0, p, q, 1, bt.part.get());
        hipLaunchKernelGGL(k_b_cg_alpha, dim3(nr), dim3(kBlock), 0, s, bt.part.get(), nbs, bt.st.get(),
                           bt.active.get());
        // e += alpha p goes with r -= alpha q before a reliable update (which reads e), else
        // with p = s + beta p below
        if (update)
          hipLaunchKernelGGL((k_b_cg_xr<SV, true>), dim3(G, nr), dim3(kBlock), 0, s, g, bt.st.get(), p, q, e, r32,
                             bt.active.get(), bt.part2.get());
        else
          hipLaunchKernelGGL((k_b_cg_xr<SV, false>), dim3(G, nr), dim3(kBlock), 0, s, g, bt.st.get(), p, q, e, r32,
                             bt.active.get(), bt.part2.get());
        int npr = G;  // partials per rhs of ||r||^2 in part2
        if (update) {
          // reliable update: x64 += e, r = b - M x64 in FP64, the low-precision residual restarts
          // from it and the search direction p is kept
          dl_op* op0 = bt.items[0].op;
          bool whole = true;  // no even-odd operator in the batch
          for (const auto& it : bt.items) whole = whole && !it.op->lat.eo;
          if (bt.single() && whole) {
            // the FP64 stencil stores b - M x64 straight into r32 (rounded) with its ||.||^2
            hipLaunchKernelGGL((k_b_accum_clear<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, X, e, bt.st.get(),
                               bt.active.get());
            TimeScope ts(bt.ctx, T_WILSON64, bt.wilson_bytes(576.0, 384.0 + kSpin * sizeof(SV)));
            npr = wilson_residual_f64(s, op0->lat, op0->U.get(), op0->kappa, X, B, nullptr, op0->lat.nc, nr,
                                      bt.active.get(), bt.part2.get(), r32, sizeof(SV) == 4 ? DL_BF16 : DL_FP32);
          } else if (bt.ml_mode == 1 && whole) {
            // the same per lattice of a multi-lattice batch, its partials re-strided to pw per rhs
            hipLaunchKernelGGL((k_b_accum_clear<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, X, e, bt.st.get(),
                               bt.active.get());
            TimeScope ts(bt.ctx, T_WILSON64, bt.wilson_bytes(576.0, 384.0 + kSpin * sizeof(SV)));
            for (const auto& it : bt.items) {
              dl_op* op = it.op;
              const long off = bt.h_off[it.r0];
              double* ip = bt.ml_part.get() + (size_t)it.r0 * bt.pw;
              const int nb = wilson_residual_f64(s, op->lat, op->U.get(), op->kappa, X + off, B + off, nullptr,
                                                 op->lat.nc, it.nr, bt.active.get() + it.r0, ip, r32 + off,
                                                 sizeof(SV) == 4 ? DL_BF16 : DL_FP32);
              if (nb > bt.pw) fail(DL_E_INVALID, "stencil partials exceed the batch's partial stride");
              const long n = (long)it.nr * bt.pw;
              hipLaunchKernelGGL(k_restride_partials, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ip, nb,
                                 it.nr, bt.part2.get() + (size_t)it.r0 * bt.pw, bt.pw);
            }
            npr = bt.pw;
          } else {
            hipLaunchKernelGGL((k_b_accum<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, X, e, bt.active.get());
            true_residual(bt, B, X, R64.get(), T64.get());
            hipLaunchKernelGGL((k_b_cg_start<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, R64.get(), r32, e,
                               bt.st.get(), bt.active.get());
            hipLaunchKernelGGL((k_b_norm2_f32<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, r32, bt.active.get(),
                               bt.part2.get());
          }
        }
        bwilson_lo(bt, 1, r32, sv, 1, bt.part.get());
        hipLaunchKernelGGL(k_b_cg_beta, dim3(nr), dim3(kBlock), 0, s, bt.part.get(), nbs, bt.part2.get(), npr,
                           bt.st.get(), bt.active.get());
        if (update)
          hipLaunchKernelGGL((k_b_cg_xpay<SV, false>), dim3(G, nr), dim3(kBlock), 0, s, g, bt.st.get(), sv, p, e,
                             bt.active.get());
        else
          hipLaunchKernelGGL((k_b_cg_xpay<SV, true>), dim3(G, nr), dim3(kBlock), 0, s, g, bt.st.get(), sv, p, e,
                             bt.active.get());
        DL_HIP(hipGetLastError());
      };
      constexpr long kStall = 25L * check;
      std::vector<double> best(nr);
      std::vector<long> best_it(nr, 0);
      for (int r = 0; r < nr; ++r) best[r] = bt.get(r, B_NRM);
      for (int it = 0; it < 100000; ++it) {
        const bool update = rel_every > 0 && (it + 1) % rel_every == 0;
        if (use_graph) {
          if (it % check == 0) {
            const bool upd_block = rel_every > 0 && (it + check) % rel_every == 0;
            graphs.run(upd_block ? 2 : 1, [&] {
              for (int q2 = 0; q2 < check; ++q2) iteration(upd_block && q2 == check - 1);
            });
          }
        } else {
          iteration(update);
        }
        if (update)
          for (int r = 0; r < nr; ++r) mvp[r] += bt.h_active[r];
        for (int r = 0; r < nr; ++r) {
          iters[r] += bt.h_active[r];
          mvp[r] += 2 * bt.h_active[r];
        }
        if ((it + 1) % check == 0) {
          bt.pull_state();
          bool changed = false;
          for (int r = 0; r < nr; ++r) {
            if (!bt.h_active[r]) continue;
            const double rn = std::sqrt(bt.get(r, B_RR));
            if (hist) hist->add(r, (double)mvp[r], rn / bnorm[r]);
            // with BF16 storage a cycle also ends when its residual has not reached a new low
            // (by 10%) for kStall iterations: the rounding can hold it above the cycle's target
            if (rn < 0.9 * best[r]) {
              best[r] = rn;
              best_it[r] = it + 1;
            }
            const bool stalled = bf16 && it + 1 - best_it[r] >= kStall && rn > target[r];
            stalled_any |= stalled;
            if (rn <= target[r] || stalled || bt.get(r, B_FLAG) != 0.0 || mvp[r] >= o.max_mvp) {
              bt.h_active[r] = 0;
              changed = true;
            }
          }
          if (changed) bt.push_active();
          if (bt.n_active() == 0) break;
        }
      }
      bt.h_active = inner_active;
      bt.push_active();
      hipLaunchKernelGGL((k_b_accum<SV>), dim3(G, nr), dim3(kBlock), 0, s, g, X, e, bt.active.get());
    }
    };
    if (bf16) inner(h[0].get(), h[1].get(), h[2].get(), h[3].get(), h[4].get(), h[5].get());
    else inner(f[0].get(), f[1].get(), f[2].get(), f[3].get(), f[4].get(), f[5].get());
    DL_HIP(hipGetLastError());
    if (bf16 && stalled_any) {
      // A BF16 cycle stalled above its target: the modes left in the residual are below what
      // BF16 vectors resolve (near-critical fields without enough deflation).  The batch goes
      // on with FP32 storage and the FP32 cycle settings; cycles restart from the FP64 state.
      for (int q = 0; q < 6; ++q) {
        h[q].release();
        f[q].alloc((size_t)bt.total);
      }
      ring16.release();
      if (bt.single()) (void)wilson_cfg(items[0].op, DL_FP32, nr);
      if (!bt.single() && bt.ml_mode == 1)
        for (const auto& it : items) (void)wilson_cfg(it.op, DL_FP32, it.nr);
      graphs.clear();  // captured blocks name the BF16 buffers
      bf16 = false;
      // defaulted settings give way to the FP32 defaults; values the caller set are kept
      if (drop_default) inner_drop = 1e-4;
      if (rel_default) rel_opt = 50;
      if (verbose()) {
        std::fprintf(stderr, "[deflan] batched: a BF16 cycle stalled, continuing with FP32 storage\n");
        std::fflush(stderr);
      }
    }
  }
  // final FP64 true residuals for every rhs
  std::fill(bt.h_active.begin(), bt.h_active.end(), 1);
  for (int r = 0; r < nr; ++r)
    if (bnorm[r] == 0.0) bt.h_active[r] = 0;
  bt.push_active();
  true_residual(bt, B, X, R64.get(), T64.get());
  bt.pull_state();
  int worst = DL_OK;
  const double t1 = now_s();
  for (int r = 0; r < nr; ++r) {
    dl_stats one{};
    one.relres = bnorm[r] == 0.0 ? 0.0 : bt.get(r, B_NRM) / bnorm[r];
    one.status = one.relres <= tol[r] ? DL_OK : DL_NOT_CONVERGED;
    one.iters = iters[r];
    one.mvp = mvp[r] + (bnorm[r] == 0.0 ? 0 : 1);
    one.guess = used_net[r];
    one.time_s = t1 - t0;
    if (one.status != DL_OK) worst = DL_NOT_CONVERGED;
    if (st) st[r] = one;
  }
  return worst;
}

int solve_next_batched(dl_op* op, const dl_eig* eig, int nrhs, const double2* B, double2* X, double tol,
                       const dl_next_opts& o, dl_stats* st, History* hist) {
  if (eig && (eig->fingerprint != op->fingerprint || eig->kind != op->kind))
    fail(DL_E_MISMATCH, "eigenvector handle was built for a different operator");
  return solve_batch({BItem{op, eig, 0, nrhs, tol}}, B, X, o, st, hist);
}

int solve_next_multi(const std::vector<MultiItem>& items, const double2* B, double2* X, const dl_next_opts& o,
                     dl_stats* st, History* hist) {
  std::vector<BItem> bi;
  int r0 = 0;
  for (const auto& m : items) {
    if (m.eig && (m.eig->fingerprint != m.op->fingerprint || m.eig->kind != m.op->kind))
      fail(DL_E_MISMATCH, "eigenvector handle was built for a different operator");
    bi.push_back(BItem{m.op, m.eig, r0, m.nrhs, m.tol});
    r0 += m.nrhs;
  }
  return solve_batch(bi, B, X, o, st, hist);
}

}  // namespace dl
