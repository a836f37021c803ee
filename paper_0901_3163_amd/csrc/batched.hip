// Batched, mixed-precision later right-hand sides: D-MinRes / D-CG for nrhs
// right-hand sides advanced together.
//
// Every stage is one launch over (site block, right-hand side) pairs, so the
// Wilson links are read from HBM once per site block for the whole batch and
// launch latency is paid once per stage instead of once per right-hand side.
// Right-hand sides that have converged are masked off (their blocks return at
// once).  Krylov vectors and the Wilson apply are FP32 (FP32 accumulation);
// the solution x, the residual r = b - M x and the Galerkin projection over
// the stored eigenvectors (Section 2: "projected ... at the beginning") are
// FP64.  Accuracy is won back by restarting the FP32 inner solve from the FP64
// true residual r64 = b - M x64 (defect correction) whenever the inner
// residual estimate has dropped by `inner_drop`, re-projecting over the
// eigenvectors at every restart.  The inner MinRes / CG runs on the
// correction e with A e = gamma5 r64 (MinRes) or M e = r64 (CG on the normal
// equations), and x64 += e closes each cycle.
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

namespace dl {

// per-rhs device state, st[r * NS + field]
enum {
  B_ALPHA = 0, B_BETA, B_BNEXT, B_COLD, B_SOLD, B_C, B_S, B_ETA, B_TAU, B_DELTA, B_EPS, B_GAMMA,
  B_INV, B_NRM, B_FLAG, B_SS, B_QQ, B_RR, B_CGA, B_CGB, B_NCUR, B_NPREV, NS
};

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
// r = b - y (FP64), partial ||r||^2 column-major [rhs][G]
__global__ void __launch_bounds__(kBlock)
k_b_resid(long n, const double2* b, const double2* y, double2* r, const int* __restrict__ active,
          double* __restrict__ part) {
  const int rhs = blockIdx.y;
  double acc = 0.0;
  if (!active || active[rhs]) {
    const long off = (long)rhs * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
      const double2 v = c_sub(b[off + i], y[off + i]);
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
__global__ void __launch_bounds__(kBlock)
k_b_minres_start(long n, const double2* r64, float2* v, float2* vp, float2* d1, float2* d2, float2* e, double* st,
                 double* invs, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const double inv = st[rhs * NS + B_INV];
  const long off = (long)rhs * n;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const int c = (int)((i >> 6) % kSpin);
    const double2 x = r64[off + i];
    const double sg = c >= 6 ? -inv : inv;
    v[off + i] = make_float2((float)(x.x * sg), (float)(x.y * sg));
    const float2 z = make_float2(0.f, 0.f);
    vp[off + i] = z;
    d1[off + i] = z;
    d2[off + i] = z;
    e[off + i] = z;
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
    invs[rhs] = 1.0;
  }
}

__global__ void __launch_bounds__(kBlock) k_b_fin_alpha(const double* part, int np, double* st, const int* active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  __shared__ double lds[kBlock / 64];
  const double s = b_fin_sum(part + (long)r * np, np, lds);
  if (threadIdx.x == 0) st[r * NS + B_ALPHA] = s;
}

// Lanczos vectors are kept unnormalised, u_j = n_j v_j, and w = A v_j (the
// Wilson epilogue applied 1/n_j).  un = w - (alpha/n_j) u_j - (beta_j/n_{j-1}) u_{j-1},
// written over u_{j-1}; partial ||un||^2.
__global__ void __launch_bounds__(kBlock)
k_b_lanczos3(long n, const double* st, const float2* u, float2* up, const float2* w, const int* __restrict__ active,
             double* __restrict__ part) {
  const int rhs = blockIdx.y;
  double acc = 0.0;
  if (!active || active[rhs]) {
    const double* S = st + rhs * NS;
    const float a = (float)(S[B_ALPHA] / S[B_NCUR]), b = (float)(S[B_BETA] / S[B_NPREV]);
    const long off = (long)rhs * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
      float2 t = c_axpy(-a, u[off + i], w[off + i]);
      t = c_axpy(-b, up[off + i], t);
      up[off + i] = t;
      acc = fma((double)t.x, (double)t.x, fma((double)t.y, (double)t.y, acc));
    }
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[(long)rhs * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock)
k_b_fin_rot(const double* part, int np, double* st, double* invs, const int* active) {
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
  }
}

// d_new = (u_j / n_j - delta d1 - eps d2)/gamma -> dn ; e += tau d_new   (n_j = B_NPREV after the rotation)
__global__ void __launch_bounds__(kBlock)
k_b_minres_update(long n, const double* st, const float2* u, const float2* d1, const float2* d2, float2* dn,
                  float2* e, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const double* S = st + rhs * NS;
  const float delta = (float)S[B_DELTA], eps = (float)S[B_EPS], ig = (float)(1.0 / S[B_GAMMA]);
  const float tau = (float)S[B_TAU];
  const float iu = (float)(1.0 / S[B_NPREV]);
  const long off = (long)rhs * n;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    float2 d = c_axpy(-delta, d1[off + i], c_scale(u[off + i], iu));
    d = c_axpy(-eps, d2[off + i], d);
    d = c_scale(d, ig);
    dn[off + i] = d;
    e[off + i] = c_axpy(tau, d, e[off + i]);
  }
}

// x64 += e (FP32 correction)
__global__ void __launch_bounds__(kBlock)
k_b_accum(long n, double2* x, const float2* e, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = (long)rhs * n;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const float2 d = e[off + i];
    x[off + i] = make_double2(x[off + i].x + (double)d.x, x[off + i].y + (double)d.y);
  }
}

// gamma5 on FP64 fields (batched)
__global__ void __launch_bounds__(kBlock) k_b_gamma5(long n, const double2* in, double2* out, const int* active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = (long)rhs * n;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const int c = (int)((i >> 6) % kSpin);
    const double2 v = in[off + i];
    out[off + i] = c >= 6 ? make_double2(-v.x, -v.y) : v;
  }
}

// ---- CG on the normal equations (CGLS), FP32 inner -----------------------------------
// start: r32 = r64 (FP32), e = 0 ; s and p are formed by the caller (s = M^dag r32, p = s).
__global__ void __launch_bounds__(kBlock)
k_b_cg_start(long n, const double2* r64, float2* r32, float2* e, double* st, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = (long)rhs * n;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const double2 x = r64[off + i];
    r32[off + i] = make_float2((float)x.x, (float)x.y);
    e[off + i] = make_float2(0.f, 0.f);
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

// e += alpha p ; r -= alpha q ; partial ||r||^2
__global__ void __launch_bounds__(kBlock)
k_b_cg_xr(long n, const double* st, const float2* p, const float2* q, float2* e, float2* r,
          const int* __restrict__ active, double* __restrict__ part) {
  const int rhs = blockIdx.y;
  double acc = 0.0;
  if (!active || active[rhs]) {
    const float a = (float)st[rhs * NS + B_CGA];
    const long off = (long)rhs * n;
    for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
      e[off + i] = c_axpy(a, p[off + i], e[off + i]);
      const float2 v = c_axpy(-a, q[off + i], r[off + i]);
      r[off + i] = v;
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

// p = s + beta p
__global__ void __launch_bounds__(kBlock)
k_b_cg_xpay(long n, const double* st, const float2* s, float2* p, const int* __restrict__ active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const float b = (float)st[rhs * NS + B_CGB];
  const long off = (long)rhs * n;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock)
    p[off + i] = c_axpy(b, p[off + i], s[off + i]);
}

__global__ void k_b_copy_f32(long n, const float2* a, float2* b, const int* active) {
  const int rhs = blockIdx.y;
  if (active && !active[rhs]) return;
  const long off = (long)rhs * n;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[off + i] = a[off + i];
}

// ---- host driver -------------------------------------------------------------
static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Batch {
  dl_op* op;
  int nr;
  long n;
  hipStream_t s;
  DBuf<double> st, part, part2;
  DBuf<int> active;
  DBuf<double> invs;  // per-rhs 1/n_j, the Wilson epilogue scale of the unnormalised Lanczos vector
  std::vector<int> h_active;
  std::vector<double> h_st;
  int G;
  Batch(dl_op* o, int nrhs) : op(o), nr(nrhs), n(o->lat.nc), s(o->ctx->stream) {
    st.alloc((size_t)nr * NS);
    G = bgrid(n);
    const size_t np = (size_t)nr * std::max(G, wilson_max_nbs(op->lat));
    part.alloc(np);
    part2.alloc(np);
    active.alloc(nr);
    invs.alloc(nr);
    h_active.assign(nr, 1);
    h_st.resize((size_t)nr * NS);
    static_assert(NS % 2 == 0, "state rows are cleared as double2");
    zero(s, (long)nr * NS / 2, reinterpret_cast<double2*>(st.get()));
  }
  void push_active() {
    DL_HIP(hipMemcpyAsync(active.get(), h_active.data(), nr * sizeof(int), hipMemcpyHostToDevice, s));
    DL_HIP(hipStreamSynchronize(s));
  }
  void pull_state() {
    DL_HIP(hipMemcpyAsync(h_st.data(), st.get(), h_st.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DL_HIP(hipStreamSynchronize(s));
  }
  double get(int r, int f) const { return h_st[(size_t)r * NS + f]; }
  int n_active() const {
    int a = 0;
    for (int v : h_active) a += v;
    return a;
  }
};

__global__ void k_f64_to_f32(long n, const double2* a, float2* b) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[i] = make_float2((float)a[i].x, (float)a[i].y);
}

// FP32 copy of the links, made on first use and kept with the operator.
const float2* op_links32_public(dl_op* op);
static const float2* op_links32(dl_op* op) { return op_links32_public(op); }
const float2* op_links32_public(dl_op* op) {
  if (!op->U32.get()) {
    op->U32.alloc(op->lat.nl);
    hipLaunchKernelGGL(k_f64_to_f32, dim3(2048), dim3(kBlock), 0, op->ctx->stream, op->lat.nl, op->U.get(),
                       op->U32.get());
    DL_HIP(hipGetLastError());
  }
  return op->U32.get();
}

static int wilson32(dl_op* op, int which, const float2* in, float2* out, int nr, int nact, int red, double* part,
                    const int* active, const double* scale = nullptr) {
  const WilsonCfg cfg = wilson_cfg(op, DL_FP32, nr);
  // algorithmic bytes: links once per site (288 B FP32) + input and output spinor per active rhs (192 B)
  TimeScope ts(op->ctx, T_WILSON, (double)op->lat.V * (288.0 + 192.0 * nact));
  return wilson_batched<float>(op->ctx->stream, op->lat, op_links32(op), op->kappa, which, in, out, op->lat.nc, nr,
                               red, scale, active, part, cfg);
}

static void wilson64b(dl_op* op, int which, const double2* in, double2* out, int nr, int nact, const int* active) {
  const WilsonCfg cfg = wilson_cfg(op, DL_FP64, nr);
  TimeScope ts(op->ctx, T_WILSON, (double)op->lat.V * (576.0 + 384.0 * nact));
  wilson_batched<double>(op->ctx->stream, op->lat, op->U.get(), op->kappa, which, in, out, op->lat.nc, nr, 0,
                         nullptr, active, nullptr, cfg);
}

// r64 = b - M x64 for active rhs; refreshes st[B_RR], st[B_NRM], st[B_INV].
static void true_residual(Batch& bt, const double2* B, const double2* X, double2* R, double2* T) {
  dl_op* op = bt.op;
  wilson64b(op, 0, X, T, bt.nr, bt.n_active(), bt.active.get());
  hipLaunchKernelGGL(k_b_resid, dim3(bt.G, bt.nr), dim3(kBlock), 0, bt.s, bt.n, B, T, R, bt.active.get(),
                     bt.part.get());
  hipLaunchKernelGGL(k_b_fin_store, dim3(bt.nr), dim3(kBlock), 0, bt.s, bt.part.get(), bt.G, bt.st.get(),
                     (int)B_RR);
  DL_HIP(hipGetLastError());
}

// Galerkin projection over the eigenvectors for every active rhs: x += Y H^-1 Y^H rA,
// rA = gamma5 r (G5M) or M^dag r (MDAGM).  T: scratch (nr fields).
static void project_batch(Batch& bt, const dl_eig* eig, const double2* R, double2* X, double2* T,
                          DBuf<double2>& cbuf, Scratch& S) {
  if (!eig || eig->k == 0) return;
  dl_op* op = bt.op;
  const int k = eig->k;
  if (op->kind == DL_G5M)
    hipLaunchKernelGGL(k_b_gamma5, dim3(bt.G, bt.nr), dim3(kBlock), 0, bt.s, bt.n, R, T, bt.active.get());
  else
    wilson64b(op, 1, R, T, bt.nr, bt.n_active(), bt.active.get());
  for (int r = 0; r < bt.nr; ++r) {
    if (!bt.h_active[r]) continue;
    int nb;
    {
      TimeScope ts(op->ctx, T_TSK_DOTS);
      nb = tsk_dots(bt.s, bt.n, k, eig->Y.get(), bt.n, nullptr, T + (long)r * bt.n, S.part.get());
    }
    sum_partials(bt.s, S.part.get(), nb, 2 * k, reinterpret_cast<double*>(cbuf.get() + (long)r * k));
  }
  {
    TimeScope ts(op->ctx, T_SMALL);
    proj_solve(bt.s, k, bt.nr, eig->Zr.get(), eig->lamr.get(), cbuf.get(), cbuf.get() + (long)bt.nr * k);
  }
  for (int r = 0; r < bt.nr; ++r) {
    if (!bt.h_active[r]) continue;
    TimeScope ts(op->ctx, T_TSK_UPDATE);
    tsk_update(bt.s, bt.n, k, eig->Y.get(), bt.n, nullptr, cbuf.get() + (long)bt.nr * k + (long)r * k, 1.0,
               X + (long)r * bt.n);
  }
}

int solve_next_batched(dl_op* op, const dl_eig* eig, int nrhs, const double2* B, double2* X, double tol,
                       const dl_next_opts& o, dl_stats* st) {
  const double t0 = now_s();
  if (eig && (eig->fingerprint != op->fingerprint || eig->kind != op->kind))
    fail(DL_E_MISMATCH, "eigenvector handle was built for a different operator");
  Batch bt(op, nrhs);
  const long n = bt.n;
  const int nr = nrhs;
  hipStream_t s = bt.s;
  const bool mr = op->kind == DL_G5M;
  Scratch S;
  S.sc.alloc(256);
  S.ensure_part((size_t)2 * std::max(eig ? eig->k : 1, 1) * tsk_nblocks(n) + 64);
  DBuf<double2> R64((size_t)nr * n), T64((size_t)nr * n);
  DBuf<float2> f[6];
  for (auto& b : f) b.alloc((size_t)nr * n);
  DBuf<double2> cbuf(2 * (size_t)nr * std::max(eig ? eig->k : 1, 1) + 2);
  std::vector<long> iters(nr, 0), mvp(nr, 0);
  std::vector<double> bnorm(nr), rel(nr, 1.0);
  // ||b|| per right-hand side (FP64)
  {
    std::vector<double> h(nr);
    for (int r = 0; r < nr; ++r) {
      const int nb = norm2_partials(s, n, B + (long)r * n, S.part.get());
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
  for (int r = 0; r < nr; ++r) {
    if (bnorm[r] == 0.0) {
      bt.h_active[r] = 0;
      zero(s, n, X + (long)r * n);
      rel[r] = 0.0;
    }
  }
  if (!o.x0_given) zero(s, (long)nr * n, X);
  bt.push_active();
  // FP64 true residual, projection, FP64 true residual again (X in place, R: its residual)
  auto start = [&](double2* Xs, double2* Rs) {
    true_residual(bt, B, Xs, Rs, T64.get());
    for (int r = 0; r < nr; ++r) mvp[r] += bt.h_active[r];
    project_batch(bt, eig, Rs, Xs, T64.get(), cbuf, S);
    if (eig && eig->k > 0) {
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
    dl_net* net = o.net;
    if (net->ctx != op->ctx) fail(DL_E_INVALID, "network and operator belong to different contexts");
    start(X, R64.get());
    bt.pull_state();
    std::vector<double> rp(nr);
    for (int r = 0; r < nr; ++r) rp[r] = bt.get(r, B_NRM);
    DBuf<double2> XN((size_t)nr * n), RN((size_t)nr * n);
    net_apply(net, op, nr, B, XN.get());
    start(XN.get(), RN.get());
    bt.pull_state();
    for (int r = 0; r < nr; ++r) {
      if (!bt.h_active[r]) continue;
      if (bt.get(r, B_NRM) < rp[r]) {
        used_net[r] = 1;
        copy(s, n, XN.get() + (long)r * n, X + (long)r * n);
      }
    }
    // residual state of the chosen starts
    true_residual(bt, B, X, R64.get(), T64.get());
    for (int r = 0; r < nr; ++r) mvp[r] += bt.h_active[r];
    started = true;
    if (verbose()) {
      int cnt = 0;
      for (int r = 0; r < nr; ++r) cnt += used_net[r];
      std::fprintf(stderr, "[deflan] learned guess kept for %d/%d rhs (%.2fs)\n", cnt, nr, now_s() - t0);
      std::fflush(stderr);
    }
  }
  const double inner_drop = 1e-4;      // reduction of the inner residual estimate per cycle
  const int check = 8;
  for (int cycle = 0; cycle < 40 && bt.n_active() > 0; ++cycle) {
    if (!(cycle == 0 && started)) start(X, R64.get());
    bt.pull_state();
    for (int r = 0; r < nr; ++r) {
      if (!bt.h_active[r]) continue;
      rel[r] = bt.get(r, B_NRM) / bnorm[r];
      if (!std::isfinite(rel[r])) fail(DL_E_NONFINITE, "non-finite residual");
      if (rel[r] <= tol || mvp[r] >= o.max_mvp) bt.h_active[r] = 0;
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
    std::vector<double> target(nr);
    for (int r = 0; r < nr; ++r) target[r] = std::max(inner_drop * bt.get(r, B_NRM), 0.5 * tol * bnorm[r]);
    std::vector<int> inner_active = bt.h_active;
    const int G = bt.G;
    if (mr) {
      float2 *u = f[0].get(), *up = f[1].get(), *w = f[2].get(), *d1 = f[3].get(), *d2 = f[4].get(),
             *e = f[5].get();
      hipLaunchKernelGGL(k_b_minres_start, dim3(G, nr), dim3(kBlock), 0, s, n, R64.get(), u, up, d1, d2, e,
                         bt.st.get(), bt.invs.get(), bt.active.get());
      for (int it = 0; it < 100000; ++it) {
        const int nbs = wilson32(op, 2, u, w, nr, bt.n_active(), 2, bt.part.get(), bt.active.get(), bt.invs.get());
        hipLaunchKernelGGL(k_b_fin_alpha, dim3(nr), dim3(kBlock), 0, s, bt.part.get(), nbs, bt.st.get(),
                           bt.active.get());
        hipLaunchKernelGGL(k_b_lanczos3, dim3(G, nr), dim3(kBlock), 0, s, n, bt.st.get(), u, up, w,
                           bt.active.get(), bt.part.get());
        hipLaunchKernelGGL(k_b_fin_rot, dim3(nr), dim3(kBlock), 0, s, bt.part.get(), G, bt.st.get(), bt.invs.get(),
                           bt.active.get());
        hipLaunchKernelGGL(k_b_minres_update, dim3(G, nr), dim3(kBlock), 0, s, n, bt.st.get(), u, d1, d2, d2, e,
                           bt.active.get());
        DL_HIP(hipGetLastError());
        std::swap(d1, d2);
        std::swap(u, up);
        for (int r = 0; r < nr; ++r) {
          iters[r] += bt.h_active[r];
          mvp[r] += bt.h_active[r];
        }
        if ((it + 1) % check == 0) {
          bt.pull_state();
          bool changed = false;
          for (int r = 0; r < nr; ++r) {
            if (!bt.h_active[r]) continue;
            const double eta = std::fabs(bt.get(r, B_ETA));
            if (eta <= target[r] || bt.get(r, B_FLAG) != 0.0 || mvp[r] >= o.max_mvp) {
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
      hipLaunchKernelGGL(k_b_accum, dim3(G, nr), dim3(kBlock), 0, s, n, X, e, bt.active.get());
    } else {
      float2 *r32 = f[0].get(), *sv = f[1].get(), *p = f[2].get(), *q = f[3].get(), *e = f[4].get();
      hipLaunchKernelGGL(k_b_cg_start, dim3(G, nr), dim3(kBlock), 0, s, n, R64.get(), r32, e, bt.st.get(),
                         bt.active.get());
      const int nbs = wilson32(op, 1, r32, sv, nr, bt.n_active(), 1, bt.part.get(), bt.active.get());
      hipLaunchKernelGGL(k_b_fin_store, dim3(nr), dim3(kBlock), 0, s, bt.part.get(), nbs, bt.st.get(), (int)B_SS);
      hipLaunchKernelGGL(k_b_copy_f32, dim3(G, nr), dim3(kBlock), 0, s, n, sv, p, bt.active.get());
      for (int r = 0; r < nr; ++r) mvp[r] += bt.h_active[r];
      for (int it = 0; it < 100000; ++it) {
        wilson32(op, 0, p, q, nr, bt.n_active(), 1, bt.part.get(), bt.active.get());
        hipLaunchKernelGGL(k_b_cg_alpha, dim3(nr), dim3(kBlock), 0, s, bt.part.get(), nbs, bt.st.get(),
                           bt.active.get());
        hipLaunchKernelGGL(k_b_cg_xr, dim3(G, nr), dim3(kBlock), 0, s, n, bt.st.get(), p, q, e, r32,
                           bt.active.get(), bt.part2.get());
        wilson32(op, 1, r32, sv, nr, bt.n_active(), 1, bt.part.get(), bt.active.get());
        hipLaunchKernelGGL(k_b_cg_beta, dim3(nr), dim3(kBlock), 0, s, bt.part.get(), nbs, bt.part2.get(), G,
                           bt.st.get(), bt.active.get());
        hipLaunchKernelGGL(k_b_cg_xpay, dim3(G, nr), dim3(kBlock), 0, s, n, bt.st.get(), sv, p, bt.active.get());
        DL_HIP(hipGetLastError());
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
            if (rn <= target[r] || bt.get(r, B_FLAG) != 0.0 || mvp[r] >= o.max_mvp) {
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
      hipLaunchKernelGGL(k_b_accum, dim3(G, nr), dim3(kBlock), 0, s, n, X, e, bt.active.get());
    }
    DL_HIP(hipGetLastError());
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
    one.status = one.relres <= tol ? DL_OK : DL_NOT_CONVERGED;
    one.iters = iters[r];
    one.mvp = mvp[r] + (bnorm[r] == 0.0 ? 0 : 1);
    one.guess = used_net[r];
    one.time_s = t1 - t0;
    if (one.status != DL_OK) worst = DL_NOT_CONVERGED;
    if (st) st[r] = one;
  }
  return worst;
}

}  // namespace dl
