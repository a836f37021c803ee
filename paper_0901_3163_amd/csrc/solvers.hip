// Host drivers of the deflated Hermitian Lanczos methods (FP64 path).
//
//  * solve_first: Lan-DR(m,k) on M^dag M, MinRes-DR(m,k) on gamma5 M (the
//    paper's first right-hand side, abstract and Section 1).  Each Lanczos
//    step applies A, re-orthogonalises against the whole basis by classical
//    Gram-Schmidt twice (tall-skinny V^H w / w - V c kernels), and writes
//    alpha_j, beta_j into the projected matrix on the device.  At the end of
//    a cycle one workgroup solves the small FP64 problem (small.hip), the
//    basis is rebuilt out of place (V Y kernel) and the true residual
//    ||b - M x||/||b|| is checked: the only host synchronisation per cycle.
//    Cycles continue past linear convergence to refine the eigenvectors
//    (Section 2, last paragraph).
//  * solve_next: D-CG / D-MinRes -- a Galerkin projection over the stored
//    eigenvectors at the beginning (Section 2), then CG on the normal
//    equations (two MVPs per iteration) or MinRes on gamma5 M (one MVP).
//    Scalars (alpha, beta, Givens rotations) live in device memory and are
//    produced by one-block finalisation kernels, so iterations are enqueued
//    back to back; the host polls the residual estimate every few iterations.
#include "engine.hpp"
#include "cplx.hpp"
#include "small.hpp"
#include "tsk.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace dl {

// DEFLAN_VERBOSE=1: one progress line per restart cycle / inner cycle on stderr.
bool verbose() {
  static const bool v = [] {
    const char* e = std::getenv("DEFLAN_VERBOSE");
    return e && *e && *e != '0';
  }();
  return v;
}

// ---- device scalar slots ----------------------------------------------------
enum {
  S_BN2 = 0,      // ||b||^2 of the user system
  S_BRKJ,         // Lanczos column of the first breakdown
  S_RN2,          // residual norm^2 (true or recurrence)
  S_FLAG,         // nonzero: breakdown / non-finite
  S_INV,          // 1 / norm
  S_NRM,          // norm
  // CGLS
  S_SS, S_QQ, S_ALPHA, S_BETA,
  // MinRes
  M_ALPHA, M_BETA, M_BNEXT, M_COLD, M_SOLD, M_C, M_S, M_ETA, M_TAU, M_DELTA, M_EPS, M_GAMMA,
  S_COUNT
};

// ---- finalisation kernels (one block) --------------------------------------
__device__ __forceinline__ double fin_sum(const double* part, int np, double* lds) {
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += kBlock) a += part[i];
  return block_sum<kBlock>(a, lds);
}

__global__ void __launch_bounds__(kBlock) k_fin_store(const double* part, int np, double* sc, int idx) {
  __shared__ double lds[kBlock / 64];
  const double s = fin_sum(part, np, lds);
  if (threadIdx.x == 0) sc[idx] = s;
}

// sc[S_NRM] = sqrt(sum), sc[S_INV] = 1/sqrt(sum) (0 if the sum is 0)
__global__ void __launch_bounds__(kBlock) k_fin_norm(const double* part, int np, double* sc) {
  __shared__ double lds[kBlock / 64];
  const double s = fin_sum(part, np, lds);
  if (threadIdx.x == 0) {
    const double nr = sqrt(s);
    sc[S_NRM] = nr;
    sc[S_INV] = nr > 0.0 ? 1.0 / nr : 0.0;
    if (!isfinite(s)) sc[S_FLAG] = 1.0;
  }
}

__global__ void __launch_bounds__(kBlock) k_fin_cgls_alpha(const double* part, int np, double* sc) {
  __shared__ double lds[kBlock / 64];
  const double qq = fin_sum(part, np, lds);
  if (threadIdx.x == 0) {
    sc[S_QQ] = qq;
    const bool ok = qq > 0.0 && isfinite(qq) && sc[S_FLAG] == 0.0;
    sc[S_ALPHA] = ok ? sc[S_SS] / qq : 0.0;
    if (!ok) sc[S_FLAG] = 1.0;
  }
}

__global__ void __launch_bounds__(kBlock)
k_fin_cgls_beta(const double* ps, int nps, const double* pr, int npr, double* sc) {
  __shared__ double lds[kBlock / 64];
  const double ss = fin_sum(ps, nps, lds);
  const double rr = fin_sum(pr, npr, lds);
  if (threadIdx.x == 0) {
    const double old = sc[S_SS];
    const bool ok = old > 0.0 && isfinite(ss) && sc[S_FLAG] == 0.0;
    sc[S_BETA] = ok ? ss / old : 0.0;
    if (ok) sc[S_SS] = ss;
    else sc[S_FLAG] = 1.0;
    sc[S_RN2] = rr;
  }
}

// CG on a Hermitian A (positive or not): alpha = ||r||^2 / Re(p^H A p); breakdown if p^H A p = 0.
__global__ void __launch_bounds__(kBlock) k_fin_cg_alpha(const double* part, int np, double* sc) {
  __shared__ double lds[kBlock / 64];
  const double pap = fin_sum(part, np, lds);
  if (threadIdx.x == 0) {
    sc[S_QQ] = pap;
    const bool ok = pap != 0.0 && isfinite(pap) && sc[S_FLAG] == 0.0;
    sc[S_ALPHA] = ok ? sc[S_RN2] / pap : 0.0;
    if (!ok) sc[S_FLAG] = 1.0;
  }
}

// beta = ||r_new||^2 / ||r||^2, S_RN2 <- ||r_new||^2
__global__ void __launch_bounds__(kBlock) k_fin_cg_beta(const double* part, int np, double* sc) {
  __shared__ double lds[kBlock / 64];
  const double rr = fin_sum(part, np, lds);
  if (threadIdx.x == 0) {
    const double old = sc[S_RN2];
    const bool ok = old > 0.0 && isfinite(rr) && sc[S_FLAG] == 0.0;
    sc[S_BETA] = ok ? rr / old : 0.0;
    sc[S_RN2] = rr;
    if (!ok) sc[S_FLAG] = 1.0;
  }
}

// MinRes: Givens QR of the new tridiagonal column (beta_j, alpha_j, beta_{j+1}).
__global__ void __launch_bounds__(kBlock) k_fin_minres_rot(const double* part, int np, double* sc) {
  __shared__ double lds[kBlock / 64];
  const double ww = fin_sum(part, np, lds);
  if (threadIdx.x == 0) {
    const double bnext = sqrt(ww);
    const double beta = sc[M_BETA], alpha = sc[M_ALPHA];
    const double c_old = sc[M_COLD], s_old = sc[M_SOLD], c = sc[M_C], s = sc[M_S];
    const double eps = s_old * beta;
    const double dt = c_old * beta;
    const double delta = c * dt + s * alpha;
    const double gbar = -s * dt + c * alpha;
    const double gamma = hypot(gbar, bnext);
    const bool ok = gamma > 0.0 && isfinite(gamma) && isfinite(bnext) && sc[S_FLAG] == 0.0;
    if (ok) {
      const double cn = gbar / gamma, sn = bnext / gamma;
      const double eta = sc[M_ETA];
      sc[M_TAU] = cn * eta;
      sc[M_ETA] = -sn * eta;
      sc[M_EPS] = eps;
      sc[M_DELTA] = delta;
      sc[M_GAMMA] = gamma;
      sc[M_COLD] = c;
      sc[M_SOLD] = s;
      sc[M_C] = cn;
      sc[M_S] = sn;
      sc[M_BNEXT] = bnext;
      sc[M_BETA] = bnext;
      if (!(bnext > 0.0)) sc[S_FLAG] = 2.0;  // invariant subspace: the solution is exact
    } else {
      sc[M_TAU] = 0.0;
      sc[M_EPS] = 0.0;
      sc[M_DELTA] = 0.0;
      sc[M_GAMMA] = 1.0;
      if (sc[S_FLAG] == 0.0) sc[S_FLAG] = 1.0;
    }
    sc[S_RN2] = sc[M_ETA] * sc[M_ETA];
  }
}

// Lanczos step bookkeeping: Tb[j][j] = Re(c1[j] + c2[j]); beta = sqrt(sum) -> Tb[j+1][j]; sc[S_INV] = 1/beta.
__global__ void __launch_bounds__(kBlock)
k_fin_lanczos(const double* part, int np, double* Tb, int m, int j, const double* c1, const double* c2, double* sc,
              double tiny) {
  __shared__ double lds[kBlock / 64];
  const double ww = fin_sum(part, np, lds);
  if (threadIdx.x == 0) {
    const double beta = sqrt(ww);
    Tb[(long)j * m + j] = c1[2 * j] + c2[2 * j];
    Tb[(long)(j + 1) * m + j] = beta;
    const bool brk = !(beta > tiny);
    sc[S_INV] = brk ? 0.0 : 1.0 / beta;
    sc[S_NRM] = beta;
    if (!isfinite(ww)) sc[S_FLAG] = 1.0;
    else if (brk && sc[S_FLAG] == 0.0) { sc[S_FLAG] = 2.0; sc[S_BRKJ] = (double)j; }
  }
}

// One residual-history point: out = (mvp, scale * sqrt(sc[idx])) or (mvp, scale * |sc[idx]|).
__global__ void k_hist_push(const double* sc, int idx, int squared, double scale, double mvp, double* out) {
  if (threadIdx.x == 0) {
    const double v = sc[idx];
    out[0] = mvp;
    out[1] = scale * (squared ? sqrt(v) : fabs(v));
  }
}

// ---- streaming kernels ------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_scale(long n, const double* sc, int idx, const double2* __restrict__ in, double2* __restrict__ out) {
  const double a = sc[idx];
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock)
    out[i] = c_scale(in[i], a);
}

// r = b - y, partial ||r||^2
__global__ void __launch_bounds__(kBlock)
k_resid(long n, const double2* b, const double2* y, double2* r, double* __restrict__ part) {
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const double2 v = c_sub(b[i], y[i]);
    r[i] = v;
    acc = fma(v.x, v.x, fma(v.y, v.y, acc));
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x += alpha p ; r -= alpha q ; partial ||r||^2
__global__ void __launch_bounds__(kBlock)
k_cgls_xr(long n, const double* sc, const double2* __restrict__ p, const double2* __restrict__ q,
          double2* __restrict__ x, double2* __restrict__ r, double* __restrict__ part) {
  const double a = sc[S_ALPHA];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    x[i] = c_axpy(a, p[i], x[i]);
    const double2 v = c_axpy(-a, q[i], r[i]);
    r[i] = v;
    acc = fma(v.x, v.x, fma(v.y, v.y, acc));
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = s + beta p
__global__ void __launch_bounds__(kBlock)
k_xpay(long n, const double* sc, int idx, const double2* __restrict__ s, double2* __restrict__ p) {
  const double b = sc[idx];
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock)
    p[i] = c_axpy(b, p[i], s[i]);
}

// w = w - alpha v - beta vprev ; partial ||w||^2
__global__ void __launch_bounds__(kBlock)
k_lanczos3(long n, const double* sc, const double2* __restrict__ v, const double2* __restrict__ vp,
           double2* __restrict__ w, double* __restrict__ part) {
  const double a = sc[M_ALPHA], b = sc[M_BETA];
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    double2 t = c_axpy(-a, v[i], w[i]);
    t = c_axpy(-b, vp[i], t);
    w[i] = t;
    acc = fma(t.x, t.x, fma(t.y, t.y, acc));
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// d_new = (v - delta d1 - eps d2)/gamma -> dn ; x += tau d_new ; vn = w / bnext
__global__ void __launch_bounds__(kBlock)
k_minres_update(long n, const double* sc, const double2* __restrict__ v, const double2* __restrict__ d1,
                const double2* d2, double2* dn, double2* __restrict__ x, const double2* __restrict__ w,
                double2* __restrict__ vn) {
  const double delta = sc[M_DELTA], eps = sc[M_EPS], ig = 1.0 / sc[M_GAMMA], tau = sc[M_TAU];
  const double bn = sc[M_BNEXT];
  const double ib = bn > 0.0 ? 1.0 / bn : 0.0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    double2 d = c_axpy(-delta, d1[i], v[i]);
    d = c_axpy(-eps, d2[i], d);
    d = c_scale(d, ig);
    dn[i] = d;
    x[i] = c_axpy(tau, d, x[i]);
    vn[i] = c_scale(w[i], ib);
  }
}

static int grid_for(long n) {
  long nb = (n + kBlock - 1) / kBlock;
  return (int)std::max(1L, std::min(nb, 2048L));
}

// ---- helpers -------------------------------------------------------------------
int apply_wilson(dl_op* op, int which, const double2* in, double2* out, int red, double* part) {
  const WilsonCfg cfg = wilson_cfg(op, DL_FP64, 1);
  // algorithmic bytes: input spinor, links and output spinor moved once (FP64: 960 B/site)
  TimeScope ts(op->ctx, T_WILSON64, 960.0 * (double)op->lat.V);
  return wilson_f64(op->ctx->stream, op->lat, op->U.get(), op->kappa, which, in, out, red, part, cfg);
}

int apply_A(dl_op* op, const double2* in, double2* out, double2* tmp) {
  if (op->kind == DL_MDAGM) {
    apply_wilson(op, 0, in, tmp);
    apply_wilson(op, 1, tmp, out);
    return 2;
  }
  apply_wilson(op, 2, in, out);
  return 1;
}

static void read_scalars(dl_ctx* ctx, const double* sc, int n, double* host) {
  DL_HIP(hipMemcpyAsync(ctx->pinned, sc, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  DL_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(host, ctx->pinned, n * sizeof(double));
}

static void write_scalars(dl_ctx* ctx, double* sc, int n, const double* host) {
  DL_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(ctx->pinned, host, n * sizeof(double));
  DL_HIP(hipMemcpyAsync(sc, ctx->pinned, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  DL_HIP(hipStreamSynchronize(ctx->stream));
}

// r = b - M x (tiled), returns ||r||^2 through sc[idx] (device), enqueued only.
static int enqueue_true_residual(dl_op* op, const double2* b, const double2* x, double2* r, double2* tmp,
                                 Scratch& S, int idx) {
  hipStream_t s = op->ctx->stream;
  const long n = op->lat.nc;
  apply_wilson(op, 0, x, tmp);
  const int nb = nblocks_for(n);
  hipLaunchKernelGGL(k_resid, dim3(nb), dim3(kBlock), 0, s, n, b, tmp, r, S.part.get());
  hipLaunchKernelGGL(k_fin_store, dim3(1), dim3(kBlock), 0, s, S.part.get(), nb, S.sc.get(), idx);
  DL_HIP(hipGetLastError());
  return 1;
}

static double host_norm2(dl_op* op, const double2* v, Scratch& S) {
  hipStream_t s = op->ctx->stream;
  const int nb = norm2_partials(s, op->lat.nc, v, S.part.get());
  hipLaunchKernelGGL(k_fin_store, dim3(1), dim3(kBlock), 0, s, S.part.get(), nb, S.sc.get(), (int)S_RN2);
  double h;
  read_scalars(op->ctx, S.sc.get() + S_RN2, 1, &h);
  return h;
}

static void init_scratch(Scratch& S, long nc, int maxvec) {
  S.sc.alloc(256);
  const size_t need = std::max<size_t>((size_t)2 * std::max(maxvec, 1) * tsk_nblocks(nc) + 64,
                                       (size_t)4 * kMaxPartials);
  S.ensure_part(need);
}

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Per-iteration residual history of one rhs of the FP64 later-rhs path, written on the device
// (no host synchronisation per point) and copied out when the rhs is done.
struct DevHist {
  DBuf<double> d;
  int cap = 0, n = 0;
  long mvp0 = 0;  // MVPs of the rhs before the current inner run
  void push(hipStream_t s, const double* sc, int idx, bool squared, double scale, long mvp) {
    if (n >= cap) return;
    hipLaunchKernelGGL(k_hist_push, dim3(1), dim3(64), 0, s, sc, idx, (int)squared, scale, (double)mvp,
                       d.get() + 2L * n);
    ++n;
  }
};

// ---- Krylov inner solvers -------------------------------------------------------
struct InnerResult {
  long iters = 0, mvp = 0;
  bool converged = false, breakdown = false;
};

// MinRes on gamma5 M from x: iterate until |eta|/||b|| <= tol (recurrence), FP64.
static InnerResult minres_run(dl_op* op, const double2* b, double2* x, double bnorm, double tol, long max_mvp,
                              Scratch& S, DBuf<double2>* w6, int check_every, DevHist* dh = nullptr) {
  hipStream_t s = op->ctx->stream;
  const long n = op->lat.nc;
  const int G = grid_for(n);
  double2 *v = w6[0].get(), *vp = w6[1].get(), *w = w6[2].get(), *d1 = w6[3].get(), *d2 = w6[4].get(),
          *tmp = w6[5].get();
  InnerResult res;
  // r0 = gamma5 (b - M x)
  apply_wilson(op, 2, x, tmp);
  res.mvp += 1;
  const int nb = nblocks_for(n);
  // w = gamma5 b - tmp  (gamma5 b formed in w first)
  gamma5_f64(s, op->lat, b, w);
  hipLaunchKernelGGL(k_resid, dim3(nb), dim3(kBlock), 0, s, n, w, tmp, w, S.part.get());
  hipLaunchKernelGGL(k_fin_norm, dim3(1), dim3(kBlock), 0, s, S.part.get(), nb, S.sc.get());
  hipLaunchKernelGGL(k_scale, dim3(G), dim3(kBlock), 0, s, n, S.sc.get(), (int)S_INV, w, v);
  zero(s, n, vp);
  zero(s, n, d1);
  zero(s, n, d2);
  double h[S_COUNT];
  read_scalars(op->ctx, S.sc.get(), S_COUNT, h);
  const double beta1 = h[S_NRM];
  if (dh) dh->push(s, S.sc.get(), (int)S_NRM, false, 1.0 / bnorm, dh->mvp0 + res.mvp);
  if (!(beta1 / bnorm > tol)) {
    res.converged = true;
    return res;
  }
  h[S_FLAG] = 0.0; h[M_BETA] = 0.0; h[M_COLD] = 1.0; h[M_SOLD] = 0.0; h[M_C] = 1.0; h[M_S] = 0.0;
  h[M_ETA] = beta1;
  write_scalars(op->ctx, S.sc.get(), S_COUNT, h);
  while (res.mvp < max_mvp) {
    const int nbw = apply_wilson(op, 2, v, w, 2, S.part.get());
    res.mvp += 1;
    hipLaunchKernelGGL(k_fin_store, dim3(1), dim3(kBlock), 0, s, S.part.get(), nbw, S.sc.get(), (int)M_ALPHA);
    hipLaunchKernelGGL(k_lanczos3, dim3(nb), dim3(kBlock), 0, s, n, S.sc.get(), v, vp, w, S.part.get());
    hipLaunchKernelGGL(k_fin_minres_rot, dim3(1), dim3(kBlock), 0, s, S.part.get(), nb, S.sc.get());
    // d_new into d2's buffer; v_next into vp's buffer
    hipLaunchKernelGGL(k_minres_update, dim3(G), dim3(kBlock), 0, s, n, S.sc.get(), v, d1, d2, d2, x, w, vp);
    DL_HIP(hipGetLastError());
    std::swap(w6[3], w6[4]);  // d1 <- d_new, d2 <- old d1
    std::swap(w6[0], w6[1]);  // v <- v_next, vp <- old v
    v = w6[0].get(); vp = w6[1].get(); d1 = w6[3].get(); d2 = w6[4].get();
    res.iters += 1;
    if (dh) dh->push(s, S.sc.get(), (int)M_ETA, false, 1.0 / bnorm, dh->mvp0 + res.mvp);
    if (res.iters % check_every == 0 || res.mvp >= max_mvp) {
      read_scalars(op->ctx, S.sc.get(), S_COUNT, h);
      if (h[S_FLAG] == 2.0) { res.converged = true; break; }
      if (h[S_FLAG] != 0.0) { res.breakdown = true; break; }
      if (std::fabs(h[M_ETA]) / bnorm <= tol) { res.converged = true; break; }
    }
  }
  return res;
}

// CG on the normal equations (CGLS) from x, tracking r = b - M x.
static InnerResult cgls_run(dl_op* op, const double2* b, double2* x, double bnorm, double tol, long max_mvp,
                            Scratch& S, DBuf<double2>* w6, int check_every, DevHist* dh = nullptr) {
  hipStream_t s = op->ctx->stream;
  const long n = op->lat.nc;
  const int G = grid_for(n);
  double2 *r = w6[0].get(), *sv = w6[1].get(), *p = w6[2].get(), *q = w6[3].get();
  InnerResult res;
  const int nb = nblocks_for(n);
  apply_wilson(op, 0, x, q);
  hipLaunchKernelGGL(k_resid, dim3(nb), dim3(kBlock), 0, s, n, b, q, r, S.part.get());
  hipLaunchKernelGGL(k_fin_store, dim3(1), dim3(kBlock), 0, s, S.part.get(), nb, S.sc.get(), (int)S_RN2);
  const int nbw = apply_wilson(op, 1, r, sv, 1, S.part.get());
  hipLaunchKernelGGL(k_fin_store, dim3(1), dim3(kBlock), 0, s, S.part.get(), nbw, S.sc.get(), (int)S_SS);
  copy(s, n, sv, p);
  res.mvp += 2;
  if (dh) dh->push(s, S.sc.get(), (int)S_RN2, true, 1.0 / bnorm, dh->mvp0 + res.mvp);
  double h[S_COUNT];
  read_scalars(op->ctx, S.sc.get(), S_COUNT, h);
  if (!(std::sqrt(h[S_RN2]) / bnorm > tol)) {
    res.converged = true;
    return res;
  }
  h[S_FLAG] = 0.0;
  write_scalars(op->ctx, S.sc.get(), S_COUNT, h);
  double* pq = S.part.get();
  double* pr = S.part.get() + kMaxPartials;
  double* ps = S.part.get() + 2 * kMaxPartials;
  while (res.mvp < max_mvp) {
    apply_wilson(op, 0, p, q, 1, pq);
    hipLaunchKernelGGL(k_fin_cgls_alpha, dim3(1), dim3(kBlock), 0, s, pq, nbw, S.sc.get());
    hipLaunchKernelGGL(k_cgls_xr, dim3(nb), dim3(kBlock), 0, s, n, S.sc.get(), p, q, x, r, pr);
    apply_wilson(op, 1, r, sv, 1, ps);
    hipLaunchKernelGGL(k_fin_cgls_beta, dim3(1), dim3(kBlock), 0, s, ps, nbw, pr, nb, S.sc.get());
    hipLaunchKernelGGL(k_xpay, dim3(G), dim3(kBlock), 0, s, n, S.sc.get(), (int)S_BETA, sv, p);
    DL_HIP(hipGetLastError());
    res.mvp += 2;
    res.iters += 1;
    if (dh) dh->push(s, S.sc.get(), (int)S_RN2, true, 1.0 / bnorm, dh->mvp0 + res.mvp);
    if (res.iters % check_every == 0 || res.mvp >= max_mvp) {
      read_scalars(op->ctx, S.sc.get(), S_COUNT, h);
      if (h[S_FLAG] != 0.0) {
        // alpha or beta undefined: the residual of the normal equations vanished
        res.breakdown = !(std::sqrt(h[S_RN2]) / bnorm <= tol);
        res.converged = !res.breakdown;
        break;
      }
      if (std::sqrt(h[S_RN2]) / bnorm <= tol) { res.converged = true; break; }
    }
  }
  return res;
}

// CG on gamma5 M x = gamma5 b from x (Hermitian, indefinite), tracking r = gamma5 (b - M x),
// whose norm is ||b - M x||.  The paper's counter-example to using CG on gamma5 M (Section 3).
static InnerResult cg_g5_run(dl_op* op, const double2* b, double2* x, double bnorm, double tol, long max_mvp,
                             Scratch& S, DBuf<double2>* w6, int check_every, DevHist* dh = nullptr) {
  hipStream_t s = op->ctx->stream;
  const long n = op->lat.nc;
  const int G = grid_for(n);
  double2 *r = w6[0].get(), *p = w6[2].get(), *q = w6[3].get();
  InnerResult res;
  const int nb = nblocks_for(n);
  apply_wilson(op, 0, x, q);
  res.mvp += 1;
  hipLaunchKernelGGL(k_resid, dim3(nb), dim3(kBlock), 0, s, n, b, q, q, S.part.get());
  hipLaunchKernelGGL(k_fin_store, dim3(1), dim3(kBlock), 0, s, S.part.get(), nb, S.sc.get(), (int)S_RN2);
  gamma5_f64(s, op->lat, q, r);
  copy(s, n, r, p);
  if (dh) dh->push(s, S.sc.get(), (int)S_RN2, true, 1.0 / bnorm, dh->mvp0 + res.mvp);
  double h[S_COUNT];
  read_scalars(op->ctx, S.sc.get(), S_COUNT, h);
  if (!(std::sqrt(h[S_RN2]) / bnorm > tol)) {
    res.converged = true;
    return res;
  }
  h[S_FLAG] = 0.0;
  write_scalars(op->ctx, S.sc.get(), S_COUNT, h);
  double* pq = S.part.get();
  double* pr = S.part.get() + kMaxPartials;
  while (res.mvp < max_mvp) {
    const int nbw = apply_wilson(op, 2, p, q, 2, pq);  // q = gamma5 M p, partials of Re(p^H q)
    hipLaunchKernelGGL(k_fin_cg_alpha, dim3(1), dim3(kBlock), 0, s, pq, nbw, S.sc.get());
    hipLaunchKernelGGL(k_cgls_xr, dim3(nb), dim3(kBlock), 0, s, n, S.sc.get(), p, q, x, r, pr);
    hipLaunchKernelGGL(k_fin_cg_beta, dim3(1), dim3(kBlock), 0, s, pr, nb, S.sc.get());
    hipLaunchKernelGGL(k_xpay, dim3(G), dim3(kBlock), 0, s, n, S.sc.get(), (int)S_BETA, r, p);
    DL_HIP(hipGetLastError());
    res.mvp += 1;
    res.iters += 1;
    if (dh) dh->push(s, S.sc.get(), (int)S_RN2, true, 1.0 / bnorm, dh->mvp0 + res.mvp);
    if (res.iters % check_every == 0 || res.mvp >= max_mvp) {
      read_scalars(op->ctx, S.sc.get(), S_COUNT, h);
      if (h[S_FLAG] != 0.0) {
        res.breakdown = !(std::sqrt(h[S_RN2]) / bnorm <= tol);
        res.converged = !res.breakdown;
        break;
      }
      if (std::sqrt(h[S_RN2]) / bnorm <= tol) { res.converged = true; break; }
    }
  }
  return res;
}

// ---- D-CG / D-MinRes --------------------------------------------------------------
static void project(dl_op* op, const dl_eig* eig, const double2* r, double2* x, Scratch& S, DBuf<double2>& cbuf) {
  if (!eig || eig->k == 0) return;
  hipStream_t s = op->ctx->stream;
  const long n = op->lat.nc;
  const int k = eig->k;
  int nb;
  {
    TimeScope ts(op->ctx, T_TSK_DOTS);
    nb = tsk_dots(s, n, k, eig->Y.get(), n, nullptr, r, S.part.get());
  }
  sum_partials(s, S.part.get(), nb, 2 * k, reinterpret_cast<double*>(cbuf.get()));
  {
    TimeScope ts(op->ctx, T_SMALL);
    proj_solve(s, k, 1, eig->Zr.get(), eig->lamr.get(), cbuf.get(), cbuf.get() + k);
  }
  TimeScope ts(op->ctx, T_TSK_UPDATE);
  tsk_update(s, n, k, eig->Y.get(), n, nullptr, cbuf.get() + k, 1.0, x);
}

int solve_next(dl_op* op, const dl_eig* eig, int nrhs, const double2* B, double2* X, double tol,
               const dl_next_opts& o, dl_stats* st, History* hist) {
  hipStream_t s = op->ctx->stream;
  const long n = op->lat.nc;
  if (eig && (eig->fingerprint != op->fingerprint || eig->kind != op->kind))
    fail(DL_E_MISMATCH, "eigenvector handle was built for a different operator");
  Scratch S;
  init_scratch(S, n, eig ? eig->k : 1);
  DBuf<double2> w6[6];
  for (auto& b : w6) b.alloc(n);
  DBuf<double2> cbuf(2 * (size_t)std::max(eig ? eig->k : 1, 1) + 2);
  int worst = DL_OK;
  for (int r = 0; r < nrhs; ++r) {
    const double t0 = now_s();
    const double2* b = B + (long)r * n;
    double2* x = X + (long)r * n;
    dl_stats one{};
    const double bn2 = host_norm2(op, b, S);
    if (!std::isfinite(bn2)) fail(DL_E_NONFINITE, "right-hand side contains NaN or Inf");
    if (bn2 == 0.0) {
      zero(s, n, x);
      one.status = DL_OK;
      one.relres = 0.0;
      if (st) st[r] = one;
      continue;
    }
    const double bnorm = std::sqrt(bn2);
    if (!o.x0_given) zero(s, n, x);
    // projection of the initial residual of the Hermitian system
    double2* rA = w6[0].get();
    double2* tmp = w6[1].get();
    long mvp = 0;
    if (eig && eig->k > 0) {
      if (op->kind == DL_G5M) {
        if (o.x0_given) {
          apply_wilson(op, 0, x, tmp);
          mvp += 1;
          const int nb = nblocks_for(n);
          hipLaunchKernelGGL(k_resid, dim3(nb), dim3(kBlock), 0, s, n, b, tmp, tmp, S.part.get());
          gamma5_f64(s, op->lat, tmp, rA);
        } else {
          gamma5_f64(s, op->lat, b, rA);
        }
      } else {
        if (o.x0_given) {
          apply_wilson(op, 0, x, tmp);
          mvp += 1;
          const int nb = nblocks_for(n);
          hipLaunchKernelGGL(k_resid, dim3(nb), dim3(kBlock), 0, s, n, b, tmp, tmp, S.part.get());
          apply_wilson(op, 1, tmp, rA);
        } else {
          apply_wilson(op, 1, b, rA);
        }
        mvp += 1;
      }
      project(op, eig, rA, x, S, cbuf);
    }
    const int check = 8;
    long iters = 0;
    bool conv = false;
    double relres = 1.0;
    DevHist dh;
    DevHist* dhp = nullptr;
    if (hist && hist->want(r)) {
      dh.cap = hist->cap[r];
      dh.d.alloc(2 * (size_t)dh.cap);
      dhp = &dh;
    }
    for (int attempt = 0; attempt < 6; ++attempt) {
      dh.mvp0 = mvp;
      InnerResult ir = op->kind != DL_G5M ? cgls_run(op, b, x, bnorm, tol, o.max_mvp - mvp, S, w6, check, dhp)
                       : o.method == DL_METHOD_CG ? cg_g5_run(op, b, x, bnorm, tol, o.max_mvp - mvp, S, w6, check, dhp)
                                                  : minres_run(op, b, x, bnorm, tol, o.max_mvp - mvp, S, w6, check, dhp);
      iters += ir.iters;
      mvp += ir.mvp;
      // true residual in FP64
      enqueue_true_residual(op, b, x, w6[0].get(), w6[1].get(), S, (int)S_RN2);
      mvp += 1;
      if (dhp) dh.push(s, S.sc.get(), (int)S_RN2, true, 1.0 / bnorm, mvp);
      double h;
      read_scalars(op->ctx, S.sc.get() + S_RN2, 1, &h);
      relres = std::sqrt(h) / bnorm;
      if (!std::isfinite(relres)) fail(DL_E_NONFINITE, "non-finite residual");
      if (relres <= tol) { conv = true; break; }
      if (mvp >= o.max_mvp) break;
    }
    if (dhp && dh.n > 0) {
      std::vector<double> hp(2 * (size_t)dh.n);
      DL_HIP(hipMemcpyAsync(hp.data(), dh.d.get(), hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      DL_HIP(hipStreamSynchronize(s));
      for (int i = 0; i < dh.n; ++i) hist->add(r, hp[2 * i], hp[2 * i + 1]);
    }
    one.status = conv ? DL_OK : DL_NOT_CONVERGED;
    one.iters = iters;
    one.mvp = mvp;
    one.relres = relres;
    one.time_s = now_s() - t0;
    if (verbose()) {
      std::fprintf(stderr, "[deflan] %s rhs %d: iters %ld relres %.3e (%.3fs)\n",
                   op->kind == DL_G5M ? (o.method == DL_METHOD_CG ? "D-CG on gamma5 M" : "D-MinRes") : "D-CG", r,
                   iters, relres, one.time_s);
      std::fflush(stderr);
    }
    if (!conv) worst = DL_NOT_CONVERGED;
    if (st) st[r] = one;
  }
  return worst;
}

// ---- eigenvector handle ---------------------------------------------------------
dl_eig* eig_build(dl_op* op, int k, DBuf<double2>&& Y, long* mvp) {
  hipStream_t s = op->ctx->stream;
  const long n = op->lat.nc;
  auto* e = new dl_eig();
  e->ctx = op->ctx;
  e->lat = op->lat;
  e->fingerprint = op->fingerprint;
  e->kappa = op->kappa;
  e->kind = op->kind;
  e->k = k;
  e->nc = n;
  e->Y = std::move(Y);
  if (k == 0) return e;
  Scratch S;
  init_scratch(S, n, k);
  DBuf<double2> ay(n), tmp(n);
  DBuf<double2> Hc((size_t)k * k);   // Hc[i*k + j] = <y_i, A y_j>
  DBuf<double> colbuf(2 * (size_t)k);
  DBuf<double> nrm((size_t)k);
  long used = 0;
  for (int j = 0; j < k; ++j) {
    double2* yj = e->Y.get() + (long)j * n;
    used += apply_A(op, yj, ay.get(), tmp.get());
    int nb;
    {
      TimeScope ts(op->ctx, T_TSK_DOTS);
      nb = tsk_dots(s, n, k, e->Y.get(), n, nullptr, ay.get(), S.part.get());
    }
    sum_partials(s, S.part.get(), nb, 2 * k, colbuf.get());
    // column j of H -> Hc[i*k + j]
    DL_HIP(hipMemcpy2DAsync(Hc.get() + j, k * sizeof(double2), colbuf.get(), sizeof(double2), sizeof(double2), k,
                            hipMemcpyDeviceToDevice, s));
    // residual ||A y_j - lambda_j y_j||, lambda_j = Re H_jj: ay -= lambda y via update with c = (lambda, 0)
    tsk_update(s, n, 1, yj, n, nullptr, reinterpret_cast<const double2*>(colbuf.get()) + j, -1.0, ay.get());
    const int nb2 = norm2_partials(s, n, ay.get(), S.part.get());
    sum_partials(s, S.part.get(), nb2, 1, nrm.get() + j);
  }
  // the update above used the complex H_jj; its imaginary part is rounding-level
  std::vector<double2> hH((size_t)k * k);
  std::vector<double> hn(k);
  DL_HIP(hipMemcpyAsync(hH.data(), Hc.get(), hH.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
  DL_HIP(hipMemcpyAsync(hn.data(), nrm.get(), k * sizeof(double), hipMemcpyDeviceToHost, s));
  e->Zr.alloc(4 * (size_t)k * k);
  e->lamr.alloc(2 * (size_t)k);
  DBuf<double> E(4 * (size_t)k * k), work(4 * (size_t)(k + 1) + 16);
  {
    TimeScope ts(op->ctx, T_SMALL);
    proj_setup(s, k, Hc.get(), E.get(), e->Zr.get(), e->lamr.get(), work.get());
  }
  DL_HIP(hipStreamSynchronize(s));
  e->evals.resize(k);
  e->resid.resize(k);
  for (int i = 0; i < k; ++i) {
    e->evals[i] = hH[(size_t)i * k + i].x;
    e->resid[i] = std::sqrt(hn[i]);
  }
  if (mvp) *mvp += used;
  return e;
}

long eig_lower(dl_op* op, dl_eig* e, int prec) {
  if (prec == DL_FP64) {
    e->Y32 = DBuf<float2>();
    e->Y16 = DBuf<bf2>();
    e->Zr32 = DBuf<double>();
    e->lamr32 = DBuf<double>();
    e->lo_prec = DL_FP64;
    return 0;
  }
  if (prec != DL_FP32 && prec != DL_BF16) fail(DL_E_INVALID, "eigenvector storage must be DL_FP64, DL_FP32 or DL_BF16");
  if (e->lo_prec == prec || e->k == 0) {
    e->lo_prec = prec;
    return 0;
  }
  hipStream_t s = op->ctx->stream;
  const long tot = (long)e->k * e->nc;
  long mvp = 0;
  if (e->lo_prec == DL_FP64) {
    // the Galerkin basis is the FP32 rounding for both storages: its Gram matrix in FP64
    e->Y32.alloc((size_t)tot);
    round_f32(s, tot, e->Y.get(), e->Y32.get());
    DBuf<double2> W((size_t)tot);
    widen_f64(s, tot, e->Y32.get(), W.get());
    dl_eig* g = eig_build(op, e->k, std::move(W), &mvp);
    e->Zr32 = std::move(g->Zr);
    e->lamr32 = std::move(g->lamr);
    delete g;
  }
  if (prec == DL_BF16) {
    e->Y16.alloc((size_t)tot);
    round_bf16(s, tot, e->Y.get(), e->Y16.get());
  } else {
    e->Y16 = DBuf<bf2>();
  }
  DL_HIP(hipStreamSynchronize(s));
  e->lo_prec = prec;
  return mvp;
}

// ---- first right-hand side: Lan-DR / MinRes-DR --------------------------------------
int solve_first(dl_op* op, const double2* b, double2* x, int m, int k, double tol, const dl_first_opts& o,
                dl_eig** eig_out, dl_stats* st, History* hist) {
  const double t0 = now_s();
  dl_ctx* ctx = op->ctx;
  hipStream_t s = ctx->stream;
  const long n = op->lat.nc;
  const bool lan = op->kind == DL_MDAGM;
  const int apv = lan ? 2 : 1;
  Scratch S;
  init_scratch(S, n, m + 1);
  zero(s, n, x);
  const double bn2 = host_norm2(op, b, S);
  if (!std::isfinite(bn2)) fail(DL_E_NONFINITE, "right-hand side contains NaN or Inf");
  dl_stats out{};
  if (bn2 == 0.0) {
    out.status = DL_OK;
    out.stop_rule = DL_STOP_LINEAR;
    if (eig_out) *eig_out = eig_build(op, 0, DBuf<double2>(), nullptr);
    if (st) *st = out;
    return DL_OK;
  }
  const double bnorm = std::sqrt(bn2);
  // basis: m + k + 2 physical slots
  const int nslots = m + k + 2;
  DBuf<double2> Vb((size_t)nslots * n);
  DBuf<double2> w(n), tmp(n), rr(n);
  zero(s, (long)nslots * n, Vb.get());
  DBuf<int> slot_d(nslots);
  std::vector<int> slot(nslots);
  for (int i = 0; i < nslots; ++i) slot[i] = i;
  DL_HIP(hipMemcpyAsync(slot_d.get(), slot.data(), nslots * sizeof(int), hipMemcpyHostToDevice, s));
  auto V = [&](int logical) { return Vb.get() + (long)slot[logical] * n; };
  // small problem buffers
  DBuf<double> Tb((size_t)(m + 1) * m), cvec(m + 1), dvec(m), Gk((size_t)(m + 1) * (k + 1) + 1);
  DBuf<double> theta(k + 1), rho(k + 1), hth(k + 1), Smat((size_t)k * k + 1), info(8);
  DBuf<double> c1(2 * (size_t)(m + 1)), c2(2 * (size_t)(m + 1)), c3(4 * (size_t)(m + 1));
  // the best cycle-end iterate: after the linear system has met tol the cycles go on for the
  // eigenvectors, and at the FP64 residual floor their corrections move the residual by small
  // factors either way
  DBuf<double2> xbest(n);
  double best = HUGE_VAL;
  DBuf<double> dgks(2);  // [0]: second Gram-Schmidt pass needed (1) or not (0); [1]: ||w||^2
  const bool kept_reorth = o.reorth == DL_REORTH_KEPT;
  const int period = std::max(1, o.reorth_period);
  DBuf<double> work(std::max(landr_work(m), minresdr_work(m)));
  {
    std::vector<double> z((size_t)(m + 1) * m, 0.0);
    DL_HIP(hipMemcpy(Tb.get(), z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  long mvp = 0;
  // r0 = bA - A x0 = bA (x0 = 0); bA = M^dag b or gamma5 b
  double2* v0 = V(0);
  if (lan) {
    apply_wilson(op, 1, b, w.get());
    mvp += 1;
  } else {
    gamma5_f64(s, op->lat, b, w.get());
  }
  {
    const int nb = norm2_partials(s, n, w.get(), S.part.get());
    hipLaunchKernelGGL(k_fin_norm, dim3(1), dim3(kBlock), 0, s, S.part.get(), nb, S.sc.get());
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kBlock), 0, s, n, S.sc.get(), (int)S_INV, w.get(), v0);
    double h[S_COUNT];
    read_scalars(ctx, S.sc.get(), S_COUNT, h);
    std::vector<double> c0(m + 1, 0.0);
    c0[0] = h[S_NRM];
    DL_HIP(hipMemcpy(cvec.get(), c0.data(), (m + 1) * sizeof(double), hipMemcpyHostToDevice));
    h[S_FLAG] = 0.0;
    write_scalars(ctx, S.sc.get(), S_COUNT, h);
  }
  int j0 = 0, cycles = 0;
  double t_line = t0;  // time of the last progress line
  long mvp_lin = -1;
  double anorm = 0.0, relres = 1.0;
  int rule = -1;
  bool breakdown = false;
  std::vector<double> h_rho(k), h_info(8);
  while (true) {
    // ---- extend the basis from column j0 to m ----
    int mm = m;
    for (int j = j0; j < m; ++j) {
      mvp += apply_A(op, V(j), w.get(), tmp.get());
      // Classical Gram-Schmidt against logical vectors [v0, v0 + nv), the second pass only when the
      // first removed more than half of ||w||^2 (the DGKS criterion, eta = 1/sqrt(2); decided on
      // the device, a skipped pass leaves zero coefficients); the coefficients land at cb[v0..]
      // (k_fin_lanczos takes alpha_j from entry j of c1 + c2).
      auto cgs2 = [&](int v0, int nv, double* ca, double* cb2) {
        for (int pass = 0; pass < 2; ++pass) {
          double* cb = (pass == 0 ? ca : cb2) + 2 * v0;
          const double* gate = pass == 0 ? nullptr : dgks.get();
          int nb;
          {
            TimeScope ts(ctx, T_TSK_DOTS);
            nb = tsk_dots(s, n, nv, Vb.get(), n, slot_d.get() + v0, w.get(), S.part.get(), gate, pass == 0);
          }
          sum_partials(s, S.part.get(), nb, 2 * nv, cb);
          if (pass == 0) sum_partials(s, S.part.get() + (size_t)2 * nv * nb, nb, 1, dgks.get() + 1);
          TimeScope ts(ctx, T_TSK_UPDATE);
          tsk_update(s, n, nv, Vb.get(), n, slot_d.get() + v0, reinterpret_cast<const double2*>(cb), -1.0, w.get(),
                     gate);
          if (pass == 0) tsk_dgks_gate(s, cb, nv, dgks.get() + 1, 0.5, dgks.get());
        }
      };
      if (!kept_reorth || j == j0 || j == 0) {
        cgs2(0, j + 1, c1.get(), c2.get());  // the whole basis (the arrow column after a restart)
      } else {
        // the paper's policy: the three-term recurrence's two vectors, and every `period` steps
        // the vectors kept at the last restart (coefficients discarded: zero in exact arithmetic)
        cgs2(j - 1, 2, c1.get(), c2.get());
        if (j0 > 0 && (j - j0) % period == 0) cgs2(0, j0, c3.get(), c3.get() + 2 * (m + 1));
      }
      const int nb = norm2_partials(s, n, w.get(), S.part.get());
      hipLaunchKernelGGL(k_fin_lanczos, dim3(1), dim3(kBlock), 0, s, S.part.get(), nb, Tb.get(), m, j, c1.get(),
                         c2.get(), S.sc.get(), 1e-14 * anorm);
      hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kBlock), 0, s, n, S.sc.get(), (int)S_INV, w.get(), V(j + 1));
      DL_HIP(hipGetLastError());
      if (anorm == 0.0 || (j - j0) % 16 == 15 || j == m - 1) {
        double h[S_COUNT];
        read_scalars(ctx, S.sc.get(), S_COUNT, h);
        // a long cycle (large m, large lattice) reports its own progress as well
        if (verbose() && now_s() - t_line >= 20.0) {
          std::fprintf(stderr, "[deflan] %s cycle %d: Lanczos step %d of %d, mvp %ld (%.1fs)\n", lan ? "Lan-DR" : "MinRes-DR",
                       cycles + 1, j + 1, m, mvp, now_s() - t0);
          std::fflush(stderr);
          t_line = now_s();
        }
        if (h[S_FLAG] == 1.0) fail(DL_E_NONFINITE, "non-finite value in the Lanczos process");
        if (h[S_FLAG] == 2.0) {
          // breakdown: V(0..brk) spans an invariant subspace; finish with an exact solve
          breakdown = true;
          mm = (int)h[S_BRKJ] + 1;
          break;
        }
      }
    }
    if (breakdown) {
      TimeScope ts(ctx, T_SMALL);
      landr_cycle(s, mm, m, 0, Tb.get(), cvec.get(), work.get(), dvec.get(), Gk.get(), theta.get(), rho.get(),
                  info.get());
    }
    // ---- cycle end ----
    cycles += 1;
    if (!breakdown) {
      TimeScope ts(ctx, T_SMALL);
      if (lan)
        landr_cycle(s, m, m, k, Tb.get(), cvec.get(), work.get(), dvec.get(), Gk.get(), theta.get(), rho.get(),
                    info.get());
      else
        minresdr_cycle(s, m, k, Tb.get(), cvec.get(), work.get(), dvec.get(), Gk.get(), theta.get(), Smat.get(),
                       rho.get(), hth.get(), info.get());
    }
    {  // x += V_mm d
      TimeScope ts(ctx, T_TSK_UPDATE);
      tsk_combine(s, n, mm, Vb.get(), n, slot_d.get(), dvec.get(), 1, 1, x, 0, nullptr, 1);
    }
    enqueue_true_residual(op, b, x, rr.get(), tmp.get(), S, (int)S_RN2);
    mvp += 1;
    double h[S_COUNT];
    read_scalars(ctx, S.sc.get(), S_COUNT, h);
    relres = std::sqrt(h[S_RN2]) / bnorm;
    if (!std::isfinite(relres)) fail(DL_E_NONFINITE, "non-finite residual");
    if (hist) hist->add(0, (double)mvp, relres);
    if (relres < best) {
      best = relres;
      copy(s, n, x, xbest.get());
    }
    if (k > 0) DL_HIP(hipMemcpy(h_rho.data(), rho.get(), k * sizeof(double), hipMemcpyDeviceToHost));
    DL_HIP(hipMemcpy(h_info.data(), info.get(), 8 * sizeof(double), hipMemcpyDeviceToHost));
    anorm = std::max(anorm, h_info[0]);
    if (verbose()) {
      double rmax = 0.0;
      for (int i = 0; i < k; ++i) rmax = std::max(rmax, h_rho[i]);
      std::fprintf(stderr, "[deflan] %s cycle %d: mvp %ld relres %.3e max eig-resid %.3e (%.1fs)\n",
                   lan ? "Lan-DR" : "MinRes-DR", cycles, mvp, relres, rmax, now_s() - t0);
      std::fflush(stderr);
      t_line = now_s();
    }
    if (breakdown) { rule = DL_STOP_BREAKDOWN; break; }
    // ---- stopping rule ----
    if (mvp_lin < 0 && relres <= tol) mvp_lin = mvp;
    bool stop = false;
    if (mvp_lin >= 0) {
      if (k == 0) { rule = DL_STOP_LINEAR; stop = true; }
      else {
        bool all = true;
        for (int i = 0; i < k; ++i) all = all && (h_rho[i] <= o.eig_tol * anorm);
        if (all) { rule = DL_STOP_EIGEN; stop = true; }
        else if ((double)mvp >= o.past_conv_factor * (double)mvp_lin) { rule = DL_STOP_MVP_FACTOR; stop = true; }
      }
    }
    if (!stop && mvp >= o.max_mvp) { rule = DL_STOP_MAX_MVP; stop = true; }
    if (stop && lan) break;  // Lan-DR: eigenvectors are V_m G_k of this cycle
    // ---- restart: rebuild the basis out of place ----
    const int nnew = lan ? k : k + 1;
    std::vector<int> used(nslots, 0), spare;
    for (int i = 0; i <= m; ++i) used[slot[i]] = 1;
    for (int i = 0; i < nslots; ++i) if (!used[i]) spare.push_back(i);
    std::vector<int> newslot(nslots);
    for (int l = 0; l < nnew; ++l) newslot[l] = spare[l];
    DBuf<int> oslot_d(std::max(nnew, 1));
    DL_HIP(hipMemcpyAsync(oslot_d.get(), newslot.data(), std::max(nnew, 1) * sizeof(int), hipMemcpyHostToDevice, s));
    {
      TimeScope ts(ctx, T_TSK_UPDATE);
      if (lan)
        tsk_combine(s, n, m, Vb.get(), n, slot_d.get(), Gk.get(), k, k, Vb.get(), n, oslot_d.get(), 0);
      else
        tsk_combine(s, n, m + 1, Vb.get(), n, slot_d.get(), Gk.get(), k + 1, k + 1, Vb.get(), n, oslot_d.get(), 0);
    }
    // logical map of the next cycle
    if (lan) newslot[k] = slot[m];
    {
      std::vector<int> u2(nslots, 0);
      for (int l = 0; l <= k; ++l) u2[newslot[l]] = 1;
      int pos = k + 1;
      for (int i = 0; i < nslots; ++i) if (!u2[i]) newslot[pos++] = i;
    }
    DL_HIP(hipStreamSynchronize(s));
    slot = newslot;
    DL_HIP(hipMemcpyAsync(slot_d.get(), slot.data(), nslots * sizeof(int), hipMemcpyHostToDevice, s));
    DL_HIP(hipStreamSynchronize(s));
    j0 = k;
    if (stop) break;  // MinRes-DR: eigenvectors are V_k S after the restart
  }
  // ---- eigenvector output ----
  if (eig_out && k > 0 && !breakdown) {
    DBuf<double2> Y((size_t)k * n);
    TimeScope ts(ctx, T_TSK_UPDATE);
    if (lan) tsk_combine(s, n, m, Vb.get(), n, slot_d.get(), Gk.get(), k, k, Y.get(), n, nullptr, 0);
    else tsk_combine(s, n, k, Vb.get(), n, slot_d.get(), Smat.get(), k, k, Y.get(), n, nullptr, 0);
    *eig_out = eig_build(op, k, std::move(Y), nullptr);
  } else if (eig_out) {
    *eig_out = eig_build(op, 0, DBuf<double2>(), nullptr);
  }
  if (best < relres) {  // a later cycle ended above an earlier one: return the best iterate
    copy(s, n, xbest.get(), x);
    relres = best;
  }
  DL_HIP(hipStreamSynchronize(s));
  out.status = (relres <= tol) ? DL_OK : DL_NOT_CONVERGED;
  out.stop_rule = rule;
  out.cycles = cycles;
  out.mvp = mvp;
  out.mvp_lin = mvp_lin;
  out.iters = mvp / apv;
  out.relres = relres;
  out.time_s = now_s() - t0;
  if (st) *st = out;
  return out.status;
}

}  // namespace dl
