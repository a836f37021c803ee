// Wilson-Dirac operator on the tiled site-major layout (FP64).
//
//   (M psi)(x) = psi(x) - kappa * sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
//                                         + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]
//
// (the Wilson matrix of the paper's lattice tests, Section 2; conventions in
// include/deflan.h).  M^dag swaps the projector signs (gamma5 M gamma5 = M^dag)
// and gamma5 M flips the sign of spin components 2 and 3 of the result.
//
// Each (1 -/+ g_mu) has rank 2, so the neighbour spinor is first projected to
// a two-spin half spinor h (6 complex), multiplied by U or U^dag (two SU(3)
// mat-vecs instead of four), and the lower two spin rows are rebuilt from h.
// In the chiral basis, for the projector (1 + S g_mu), S = +-1:
//   mu=x: h0 = p0 + S i p3, h1 = p1 + S i p2;  rows 2,3 = -S i h1, -S i h0
//   mu=y: h0 = p0 - S p3,   h1 = p1 + S p2;    rows 2,3 =  S h1,   -S h0
//   mu=z: h0 = p0 + S i p2, h1 = p1 - S i p3;  rows 2,3 = -S i h0,  S i h1
//   mu=t: h0 = p0 + S p2,   h1 = p1 + S p3;    rows 2,3 =  S h0,    S h1
// One thread per site; loads of a component for 64 consecutive sites are one
// coalesced wavefront access; neighbour spinors and the backward links are
// re-read through L2 (blocks are mapped so that each XCD walks a contiguous
// slab of the lattice, keeping the +-z/+-t neighbours in its L2).
//
// The kernel is templated on the storage/arithmetic type (double: FP64,
// float: FP32 with FP32 accumulation) and applies the operator to a batch of
// right-hand sides: logical block b covers site block b / nrhs of right-hand
// side b % nrhs, so the nrhs blocks that read the same links are consecutive
// on one XCD and the links come from HBM once and from L2 for the others.
#include "internal.hpp"
#include "cplx.hpp"

namespace dl {

// Element offsets are signed 32-bit ints (a field holds far fewer than 2^31
// elements), so component c of a site is base + off + c*64 and the c*64 part
// folds into the load's immediate offset.
__device__ __forceinline__ int sp_base(int site) { return (site >> 6) * (kSpin * kTile) + (site & 63); }
__device__ __forceinline__ int lk_base(int site, int mu) {
  return (site >> 6) * (kLinkC * kTile) + mu * 9 * kTile + (site & 63);
}

template <int MU, int S, class C>
__device__ __forceinline__ void project(const C p[12], C h[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const C p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    if (MU == 0) {
      h[c] = S > 0 ? c_add(p0, c_i(p3)) : c_sub(p0, c_i(p3));
      h[3 + c] = S > 0 ? c_add(p1, c_i(p2)) : c_sub(p1, c_i(p2));
    } else if (MU == 1) {
      h[c] = S > 0 ? c_sub(p0, p3) : c_add(p0, p3);
      h[3 + c] = S > 0 ? c_add(p1, p2) : c_sub(p1, p2);
    } else if (MU == 2) {
      h[c] = S > 0 ? c_add(p0, c_i(p2)) : c_sub(p0, c_i(p2));
      h[3 + c] = S > 0 ? c_sub(p1, c_i(p3)) : c_add(p1, c_i(p3));
    } else {
      h[c] = S > 0 ? c_add(p0, p2) : c_sub(p0, p2);
      h[3 + c] = S > 0 ? c_add(p1, p3) : c_sub(p1, p3);
    }
  }
}

template <int MU, int S, class C>
__device__ __forceinline__ void reconstruct(C acc[12], const C g[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const C g0 = g[c], g1 = g[3 + c];
    acc[c] = c_add(acc[c], g0);
    acc[3 + c] = c_add(acc[3 + c], g1);
    if (MU == 0) {
      acc[6 + c] = S > 0 ? c_sub(acc[6 + c], c_i(g1)) : c_add(acc[6 + c], c_i(g1));
      acc[9 + c] = S > 0 ? c_sub(acc[9 + c], c_i(g0)) : c_add(acc[9 + c], c_i(g0));
    } else if (MU == 1) {
      acc[6 + c] = S > 0 ? c_add(acc[6 + c], g1) : c_sub(acc[6 + c], g1);
      acc[9 + c] = S > 0 ? c_sub(acc[9 + c], g0) : c_add(acc[9 + c], g0);
    } else if (MU == 2) {
      acc[6 + c] = S > 0 ? c_sub(acc[6 + c], c_i(g0)) : c_add(acc[6 + c], c_i(g0));
      acc[9 + c] = S > 0 ? c_add(acc[9 + c], c_i(g1)) : c_sub(acc[9 + c], c_i(g1));
    } else {
      acc[6 + c] = S > 0 ? c_add(acc[6 + c], g0) : c_sub(acc[6 + c], g0);
      acc[9 + c] = S > 0 ? c_add(acc[9 + c], g1) : c_sub(acc[9 + c], g1);
    }
  }
}

template <int S, class C>
__device__ __forceinline__ void project_mu(int mu, const C p[12], C h[6]) {
  switch (mu) {
    case 0: project<0, S>(p, h); break;
    case 1: project<1, S>(p, h); break;
    case 2: project<2, S>(p, h); break;
    default: project<3, S>(p, h); break;
  }
}

template <int S, class C>
__device__ __forceinline__ void reconstruct_mu(int mu, C acc[12], const C g[6]) {
  switch (mu) {
    case 0: reconstruct<0, S>(acc, g); break;
    case 1: reconstruct<1, S>(acc, g); break;
    case 2: reconstruct<2, S>(acc, g); break;
    default: reconstruct<3, S>(acc, g); break;
  }
}

// One hop in direction mu (runtime): load the neighbour spinor and the link,
// project, multiply by U (forward) or U^dag (backward, link taken at the
// neighbour), rebuild and accumulate.  Every load address depends on mu, so
// the loads of different directions cannot be hoisted ahead of each other.
template <int S, bool DAG, class C>
__device__ __forceinline__ void hop(const C* U, const C* in, int mu, int nb, int lsite, C acc[12]) {
  C p[12], h[6], g[6], u[9];
  const C* pp = in + sp_base(nb);
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = pp[c * kTile];
  const C* up = U + lk_base(lsite, mu);
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = up[e * kTile];
  project_mu<S>(mu, p, h);
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      C r = c_scale(h[s * 3], 0);
      if (!DAG) {
        r = c_fma(u[a * 3 + 0], h[s * 3 + 0], r);
        r = c_fma(u[a * 3 + 1], h[s * 3 + 1], r);
        r = c_fma(u[a * 3 + 2], h[s * 3 + 2], r);
      } else {
        r = c_fmac(u[0 * 3 + a], h[s * 3 + 0], r);
        r = c_fmac(u[1 * 3 + a], h[s * 3 + 1], r);
        r = c_fmac(u[2 * 3 + a], h[s * 3 + 2], r);
      }
      g[s * 3 + a] = r;
    }
  reconstruct_mu<S>(mu, acc, g);
}

// WHICH: 0 M, 1 M^dag, 2 gamma5 M.  RED: 0 none, 1 ||out||^2, 2 Re<in, out> (partials in FP64,
// column-major [nrhs][nbs]).  scale (optional, per rhs): out = scale * op(in).
// active (optional, per rhs): blocks of inactive right-hand sides return at once.
// Launch shape: NT threads per block, OCC the occupancy hint (waves per SIMD the
// register budget must allow); ORDER 0: rhs fastest, XCD-contiguous blocks; 1: sites
// fastest, XCD-contiguous; 2: rhs fastest, hardware block order.
template <class R, int WHICH, int RED, int NT, int OCC>
__global__ void __launch_bounds__(NT, OCC)
k_wilson(const typename CT<R>::type* __restrict__ U, const typename CT<R>::type* __restrict__ in,
         typename CT<R>::type* __restrict__ out, long fstride, int nrhs, double kappa, int Lx, int Ly, int Lz,
         int Lt, long V, long Vpad, int nbs, int order, const double* __restrict__ scale,
         const int* __restrict__ active, double* __restrict__ part) {
  using C = typename CT<R>::type;
  const int lb = order == 2 ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int rhs = order == 1 ? lb / nbs : lb % nrhs;
  const int sb = order == 1 ? lb % nbs : lb / nrhs;
  if (active && !active[rhs]) return;
  in += rhs * fstride;
  out += rhs * fstride;
  const int site = sb * NT + (int)threadIdx.x;
  double red = 0.0;
  if (site >= V && site < Vpad) {
    // padding sites of the last tile are kept at zero
    C* op = out + sp_base(site);
#pragma unroll
    for (int c = 0; c < 12; ++c) op[c * kTile] = CT<R>::make(0, 0);
  }
  if (site < V) {
    const int x = site % Lx;
    const int y = (site / Lx) % Ly;
    const int z = (site / (Lx * Ly)) % Lz;
    const int t = site / (Lx * Ly * Lz);
    const int sy = Lx, sz = Lx * Ly, st = Lx * Ly * Lz;
    // neighbour offsets per direction
    const int fx = x == Lx - 1 ? 1 - Lx : 1, bx = x == 0 ? Lx - 1 : -1;
    const int fy = y == Ly - 1 ? (1 - Ly) * sy : sy, by = y == 0 ? (Ly - 1) * sy : -sy;
    const int fz = z == Lz - 1 ? (1 - Lz) * sz : sz, bz = z == 0 ? (Lz - 1) * sz : -sz;
    const int ft = t == Lt - 1 ? (1 - Lt) * st : st, bt = t == 0 ? (Lt - 1) * st : -st;
    C acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = CT<R>::make(0, 0);
    constexpr int SF = (WHICH == 1) ? 1 : -1;  // forward projector 1 + SF g_mu, backward 1 - SF g_mu
    // A runtime loop over the four directions (loads depend on mu) keeps the
    // compiler from hoisting all 168 neighbour/link loads ahead of the arithmetic.
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      const int df = mu == 0 ? fx : mu == 1 ? fy : mu == 2 ? fz : ft;
      const int db = mu == 0 ? bx : mu == 1 ? by : mu == 2 ? bz : bt;
      hop<SF, false>(U, in, mu, site + df, site, acc);
      hop<-SF, true>(U, in, mu, site + db, site + db, acc);
    }
    const R sc = scale ? (R)scale[rhs] : (R)1;
    const R mk = (R)(-kappa);
    const C* ip = in + sp_base(site);
    C* op = out + sp_base(site);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const C p = ip[c * kTile];
      C r = CT<R>::make(fma(mk, acc[c].x, p.x) * sc, fma(mk, acc[c].y, p.y) * sc);
      if (WHICH == 2 && c >= 6) r = CT<R>::make(-r.x, -r.y);
      op[c * kTile] = r;
      if (RED == 1) red += (double)r.x * r.x + (double)r.y * r.y;
      if (RED == 2) red += ((double)p.x * r.x + (double)p.y * r.y) * sc;
    }
  }
  if (RED != 0) {
    __shared__ double lds[NT / 64];
    const double s = block_sum<NT>(red, lds);
    if (threadIdx.x == 0) part[(long)rhs * nbs + sb] = s;
  }
}

// Launch-shape variants: (threads per block, occupancy hint).
static constexpr int kVariantNT[kWilsonVariants] = {256, 128, 512, 256};

template <class R, int WHICH, int RED, int NT, int OCC>
static void launch_one(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, const cplx_t<R>* in,
                       cplx_t<R>* out, long fstride, int nrhs, int order, const double* scale, const int* active,
                       double* part, int nbs) {
  const int* L = lat.L;
  hipLaunchKernelGGL((k_wilson<R, WHICH, RED, NT, OCC>), dim3(nbs * nrhs), dim3(NT), 0, s, U, in, out, fstride, nrhs,
                     kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, nbs, order, scale, active, part);
}

template <class R, int WHICH, int RED>
static void launch_variant(int variant, hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa,
                           const cplx_t<R>* in, cplx_t<R>* out, long fstride, int nrhs, int order,
                           const double* scale, const int* active, double* part, int nbs) {
  switch (variant) {
    case 1: launch_one<R, WHICH, RED, 128, 2>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs); break;
    case 2: launch_one<R, WHICH, RED, 512, 1>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs); break;
    case 3: launch_one<R, WHICH, RED, 256, 1>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs); break;
    default: launch_one<R, WHICH, RED, 256, 2>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs); break;
  }
}

int wilson_nbs(const Lattice& lat, const WilsonCfg& cfg) {
  const int nt = kVariantNT[cfg.variant % kWilsonVariants];
  return (int)((lat.V + nt - 1) / nt);
}

int wilson_max_nbs(const Lattice& lat) { return (int)((lat.V + 127) / 128); }

template <class R>
int wilson_batched(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, int which,
                   const cplx_t<R>* in, cplx_t<R>* out, long fstride, int nrhs, int red, const double* scale,
                   const int* active, double* part, WilsonCfg cfg) {
  const int v = cfg.variant % kWilsonVariants;
  const int nbs = wilson_nbs(lat, cfg);
  if (red && nbs > kMaxPartials) fail(DL_E_INVALID, "lattice too large for fused reduction");
  if ((long)nbs * nrhs > 2147483647L) fail(DL_E_INVALID, "grid too large");
  const int o = cfg.order;
#define DL_W(WH, RD) launch_variant<R, WH, RD>(v, s, lat, U, kappa, in, out, fstride, nrhs, o, scale, active, part, nbs)
  if (which == 0) { if (red == 0) DL_W(0, 0); else if (red == 1) DL_W(0, 1); else DL_W(0, 2); }
  else if (which == 1) { if (red == 0) DL_W(1, 0); else if (red == 1) DL_W(1, 1); else DL_W(1, 2); }
  else { if (red == 0) DL_W(2, 0); else if (red == 1) DL_W(2, 1); else DL_W(2, 2); }
#undef DL_W
  DL_HIP(hipGetLastError());
  return red ? nbs : 0;
}

template int wilson_batched<double>(hipStream_t, const Lattice&, const double2*, double, int, const double2*,
                                    double2*, long, int, int, const double*, const int*, double*, WilsonCfg);
template int wilson_batched<float>(hipStream_t, const Lattice&, const float2*, double, int, const float2*, float2*,
                                   long, int, int, const double*, const int*, double*, WilsonCfg);

int wilson_f64(hipStream_t s, const Lattice& lat, const double2* U, double kappa, int which,
               const double2* in, double2* out, int red, double* part, WilsonCfg cfg) {
  return wilson_batched<double>(s, lat, U, kappa, which, in, out, lat.nc, 1, red, nullptr, nullptr, part, cfg);
}

__global__ void k_gamma5_f64(const double2* __restrict__ in, double2* __restrict__ out, long nc) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc) return;
  const int c = (int)((i >> 6) % kSpin);
  const double2 v = in[i];
  out[i] = c >= 6 ? make_double2(-v.x, -v.y) : v;
}

void gamma5_f64(hipStream_t s, const Lattice& lat, const double2* in, double2* out) {
  const long n = lat.nc;
  hipLaunchKernelGGL(k_gamma5_f64, dim3((n + 255) / 256), dim3(256), 0, s, in, out, n);
  DL_HIP(hipGetLastError());
}

}  // namespace dl
