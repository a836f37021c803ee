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

#include <algorithm>
#include <map>
#include <mutex>

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

// g = U h (DAG false) or U^dag h (DAG true) on a half spinor (two colour vectors).
template <bool DAG, class C>
__device__ __forceinline__ void mul_half(const C u[9], const C h[6], C g[6]) {
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
}

// One hop in direction mu (runtime): load the neighbour spinor and the link (its 9
// components at up[e * ustride]), project, multiply by U (forward) or U^dag (backward,
// link taken at the neighbour), rebuild and accumulate.  Every load address depends on
// mu, so the loads of different directions cannot be hoisted ahead of each other.
template <int S, bool DAG, class C, class SV>
__device__ __forceinline__ void hop_at(const C* up, int ustride, const SV* in, int mu, int nb, C acc[12]) {
  C p[12], h[6], g[6], u[9];
  const SV* pp = in + sp_base(nb);
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = sld(pp + c * kTile);
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = up[e * ustride];
  project_mu<S>(mu, p, h);
  mul_half<DAG>(u, h, g);
  reconstruct_mu<S>(mu, acc, g);
}

template <int S, bool DAG, class C, class SV>
__device__ __forceinline__ void hop(const C* U, const SV* in, int mu, int nb, int lsite, C acc[12]) {
  hop_at<S, DAG>(U + lk_base(lsite, mu), kTile, in, mu, nb, acc);
}

// WHICH: 0 M, 1 M^dag, 2 gamma5 M.  RED: 0 none, 1 ||out||^2, 2 Re<in, out> (partials in FP64,
// column-major [nrhs][nbs]).  scale (optional, per rhs): out = scale * op(in).
// active (optional, per rhs): blocks of inactive right-hand sides return at once.
// Launch shape: NT threads per block, OCC the occupancy hint (waves per SIMD the
// register budget must allow); ORDER 0: rhs fastest, XCD-contiguous blocks; 1: sites
// fastest, XCD-contiguous; 2: rhs fastest, hardware block order.
// One site of the stencil for one field (zeroes padding sites); returns the fused
// reduction term (||out||^2 or Re<in, out>) of the site.
template <class R, class SV, int WHICH, int RED>
__device__ __forceinline__ double wilson_site(const typename CT<R>::type* __restrict__ U,
                                              const SV* __restrict__ in, SV* __restrict__ out, double kappa, int Lx, int Ly,
                                              int Lz, int Lt, long V, long Vpad, int site, R sc) {
  using C = typename CT<R>::type;
  double red = 0.0;
  if (site >= V && site < Vpad) {
    // padding sites of the last tile are kept at zero
    SV* op = out + sp_base(site);
#pragma unroll
    for (int c = 0; c < 12; ++c) sst(op + c * kTile, CT<R>::make(0, 0));
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
    const R mk = (R)(-kappa);
    const SV* ip = in + sp_base(site);
    SV* op = out + sp_base(site);
    R sred = 0;  // this site's share of the reduction, summed in R
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const C p = sld(ip + c * kTile);
      C r = CT<R>::make(fma(mk, acc[c].x, p.x) * sc, fma(mk, acc[c].y, p.y) * sc);
      if (WHICH == 2 && c >= 6) r = CT<R>::make(-r.x, -r.y);
      sst(op + c * kTile, r);
      if (RED == 1) sred = fma(r.x, r.x, fma(r.y, r.y, sred));
      if (RED == 2) sred = fma(p.x, r.x, fma(p.y, r.y, sred));
    }
    if (RED == 1) red += (double)sred;
    if (RED == 2) red += (double)sred * sc;
  }
  return red;
}

template <class R, class SV, int WHICH, int RED, int NT, int OCC>
__global__ void __launch_bounds__(NT, OCC)
k_wilson(const typename CT<R>::type* __restrict__ U, const SV* __restrict__ in,
         SV* __restrict__ out, long fstride, int nrhs, double kappa, int Lx, int Ly, int Lz,
         int Lt, long V, long Vpad, int nbs, int order, const double* __restrict__ scale,
         const int* __restrict__ active, double* __restrict__ part) {
  const int lb = order == 2 ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int rhs = order == 1 ? lb / nbs : lb % nrhs;
  const int sb = order == 1 ? lb % nbs : lb / nrhs;
  if (active && !active[rhs]) return;
  const int site = sb * NT + (int)threadIdx.x;
  const R sc = scale ? (R)scale[rhs] : (R)1;
  const double red = wilson_site<R, SV, WHICH, RED>(U, in + rhs * fstride, out + rhs * fstride, kappa, Lx, Ly, Lz, Lt,
                                                V, Vpad, site, sc);
  if (RED != 0) {
    __shared__ double lds[NT / 64];
    const double s = block_sum<NT>(red, lds);
    if (threadIdx.x == 0) part[(long)rhs * nbs + sb] = s;
  }
}

// Several lattices in one launch: a work list of items (lattice, links, kappa, range of
// right-hand sides).  Logical block b (XCD-contiguous) belongs to the item whose block
// range [block0, block0 + nbs * nrhs) holds it, and within the item to (site block, rhs)
// with the rhs fastest, so the blocks that read the same links are consecutive.  Field j
// starts at offs[j] (complex elements).  Partials: part[rhs * pstride + site block]; the
// first site block of each rhs zeroes the tail up to pstride, so every rhs reduces over
// pstride partials.
template <class R, class SV, int WHICH, int RED>
__global__ void __launch_bounds__(256, 2)
k_wilson_ml(const WilsonItem* __restrict__ items, int nitems, const SV* __restrict__ in,
            SV* __restrict__ out, const long* __restrict__ offs, int pstride,
            const double* __restrict__ scale, const int* __restrict__ active, double* __restrict__ part) {
  using C = typename CT<R>::type;
  const int b = xcd_block(blockIdx.x, gridDim.x);
  int it = 0;
  while (it + 1 < nitems && b >= items[it + 1].block0) ++it;
  const WilsonItem w = items[it];
  const int rl = (b - w.block0) % w.nrhs;
  const int sb = (b - w.block0) / w.nrhs;
  const int rhs = w.rhs0 + rl;
  if (active && !active[rhs]) return;
  const int site = sb * 256 + (int)threadIdx.x;
  const R sc = scale ? (R)scale[rhs] : (R)1;
  const long off = offs[rhs];
  const double red = wilson_site<R, SV, WHICH, RED>(static_cast<const C*>(w.U), in + off, out + off, w.kappa, w.L[0],
                                                w.L[1], w.L[2], w.L[3], w.V, w.Vpad, site, sc);
  if (RED != 0) {
    __shared__ double lds[256 / 64];
    const double s = block_sum<256>(red, lds);
    if (threadIdx.x == 0) part[(long)rhs * pstride + sb] = s;
    if (sb == 0)
      for (int q = w.nbs + (int)threadIdx.x; q < pstride; q += 256) part[(long)rhs * pstride + q] = 0.0;
  }
}

template <class R, class SV>
void wilson_multi(hipStream_t s, const WilsonItem* d_items, int nitems, int nblocks, int pstride, int which,
                  const SV* in, SV* out, const long* offs, int red, const double* scale, const int* active,
                  double* part) {
#define DL_ML(WH, RD)                                                                                          \
  hipLaunchKernelGGL((k_wilson_ml<R, SV, WH, RD>), dim3(nblocks), dim3(256), 0, s, d_items, nitems, in, out, offs, \
                     pstride, scale, active, part)
  if (which == 0) { if (red == 0) DL_ML(0, 0); else if (red == 1) DL_ML(0, 1); else DL_ML(0, 2); }
  else if (which == 1) { if (red == 0) DL_ML(1, 0); else if (red == 1) DL_ML(1, 1); else DL_ML(1, 2); }
  else { if (red == 0) DL_ML(2, 0); else if (red == 1) DL_ML(2, 1); else DL_ML(2, 2); }
#undef DL_ML
  DL_HIP(hipGetLastError());
}

template void wilson_multi<double, double2>(hipStream_t, const WilsonItem*, int, int, int, int, const double2*,
                                            double2*, const long*, int, const double*, const int*, double*);
template void wilson_multi<float, float2>(hipStream_t, const WilsonItem*, int, int, int, int, const float2*, float2*,
                                          const long*, int, const double*, const int*, double*);
template void wilson_multi<float, bf2>(hipStream_t, const WilsonItem*, int, int, int, int, const bf2*, bf2*,
                                       const long*, int, const double*, const int*, double*);

// t-marching form of the same operator.  A thread owns one (x, y, z) site and walks
// T consecutive time slices t0 .. t0+T-1 of it.  The forward-t neighbour psi(t+1)
// loaded at step t is the centre spinor of step t+1, and the backward-t hop of step
// t+1, U_t(t)^dag (1 + S g_t) psi(t), is formed at step t from the centre spinor and
// the forward link U_t(t) already in registers.  Every spinor and link is therefore
// read once along t; the x, y, z neighbours lie in the same time slice, which the
// blocks of one XCD walk together, so they come from L2.  A block is NT consecutive
// (x, y, z) sites of one time chunk of one right-hand side; logical block = (site block,
// rhs) with the same order options as k_wilson.  RES: out = add - op(in) (the residual
// b - M x, with its ||.||^2 under RED = 1), so M x is never written out.  LO = 1 / 2 (with RES):
// the residual is stored only rounded to FP32 / BF16 (through FP32) in lo, at the same element
// offsets, and RED = 1 sums the squares of the stored values.
template <class R, class SV, int WHICH, int RED, int NT, bool RES = false, int LO = 0>
__global__ void __launch_bounds__(NT)
k_wilson_tm(const typename CT<R>::type* __restrict__ U, const SV* __restrict__ in,
            SV* __restrict__ out, long fstride, int nrhs, double kappa, int Lx, int Ly, int Lz,
            int Lt, long V, long Vpad, int T, int nb3, int nbs, int order, const double* __restrict__ scale,
            const int* __restrict__ active, double* __restrict__ part, const SV* __restrict__ add,
            void* __restrict__ lo = nullptr) {
  using C = typename CT<R>::type;
  const int lb = order == 2 ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int rhs = order == 1 ? lb / nbs : lb % nrhs;
  const int sb = order == 1 ? lb % nbs : lb / nrhs;
  if (active && !active[rhs]) {
    if (RES && RED != 0 && threadIdx.x == 0) part[(long)rhs * nbs + sb] = 0.0;  // an inactive rhs sums to 0
    return;
  }
  in += rhs * fstride;
  if (LO == 0) out += rhs * fstride;
  if (RES) add += rhs * fstride;
  float2* lo32 = LO == 1 ? static_cast<float2*>(lo) + rhs * fstride : nullptr;
  bf2* lo16 = LO == 2 ? static_cast<bf2*>(lo) + rhs * fstride : nullptr;
  const int b3 = sb % nb3, tc = sb / nb3;
  const int V3 = Lx * Ly * Lz;
  const int s3 = b3 * NT + (int)threadIdx.x;
  double red = 0.0;
  // (the low-precision residual's padding sites are zero already and stay so)
  if (LO == 0 && b3 == 0 && (tc + 1) * T >= Lt) {
    // padding sites of the last tile are kept at zero (written by the last chunk's first block)
    for (long sp = V + threadIdx.x; sp < Vpad; sp += NT) {
      SV* op = out + sp_base((int)sp);
#pragma unroll
      for (int c = 0; c < 12; ++c) sst(op + c * kTile, CT<R>::make(0, 0));
    }
  }
  if (s3 < V3) {
    const int x = s3 % Lx;
    const int y = (s3 / Lx) % Ly;
    const int z = s3 / (Lx * Ly);
    const int sy = Lx, sz = Lx * Ly;
    const int fx = x == Lx - 1 ? 1 - Lx : 1, bx = x == 0 ? Lx - 1 : -1;
    const int fy = y == Ly - 1 ? (1 - Ly) * sy : sy, by = y == 0 ? (Ly - 1) * sy : -sy;
    const int fz = z == Lz - 1 ? (1 - Lz) * sz : sz, bz = z == 0 ? (Lz - 1) * sz : -sz;
    constexpr int SF = (WHICH == 1) ? 1 : -1;  // forward projector 1 + SF g_mu, backward 1 - SF g_mu
    const int t0 = tc * T;
    const int t1 = t0 + T < Lt ? t0 + T : Lt;
    const R sc = scale ? (R)scale[rhs] : (R)1;
    const R mk = (R)(-kappa);
    // carried state: centre spinor of the current slice and the backward-t hop into it
    C cen[12], gb[6];
    {
      const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
      const int sprev = tp * V3 + s3;
      C p[12], h[6], u[9];
      const SV* pp = in + sp_base(sprev);
#pragma unroll
      for (int c = 0; c < 12; ++c) p[c] = sld(pp + c * kTile);
      const C* up = U + lk_base(sprev, 3);
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = up[e * kTile];
      project<3, -SF>(p, h);
      mul_half<true>(u, h, gb);
      const SV* cp = in + sp_base(t0 * V3 + s3);
#pragma unroll
      for (int c = 0; c < 12; ++c) cen[c] = sld(cp + c * kTile);
    }
#pragma unroll 1
    for (int t = t0; t < t1; ++t) {
      const int site = t * V3 + s3;
      C acc[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = CT<R>::make(0, 0);
#pragma unroll 1
      for (int mu = 0; mu < 3; ++mu) {
        const int df = mu == 0 ? fx : mu == 1 ? fy : fz;
        const int db = mu == 0 ? bx : mu == 1 ? by : bz;
        hop<SF, false>(U, in, mu, site + df, site, acc);
        hop<-SF, true>(U, in, mu, site + db, site + db, acc);
      }
      // forward t: psi(t+1) is the next centre; U_t(t) also forms the next backward hop.
      // The hops are accumulated in k_wilson's order (x+, x-, y+, y-, z+, z-, t+, t-) with
      // the same arithmetic, so both kernels give the same result.
      const int snext = (t == Lt - 1 ? 0 : t + 1) * V3 + s3;
      C nx[12], u[9];
      {
        const SV* pp = in + sp_base(snext);
#pragma unroll
        for (int c = 0; c < 12; ++c) nx[c] = sld(pp + c * kTile);
        const C* up = U + lk_base(site, 3);
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = up[e * kTile];
        C h[6], g[6];
        project<3, SF>(nx, h);
        mul_half<false>(u, h, g);
        reconstruct<3, SF>(acc, g);
        // backward t: the hop carried from the previous slice
        reconstruct<3, -SF>(acc, gb);
        project<3, -SF>(cen, h);
        mul_half<true>(u, h, gb);
      }
      SV* op = LO == 0 ? out + sp_base(site) : nullptr;  // (LO: out is not used)
      R sred = 0;  // this site's share of the reduction, summed in R
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const C p = cen[c];
        C r = CT<R>::make(fma(mk, acc[c].x, p.x) * sc, fma(mk, acc[c].y, p.y) * sc);
        if (WHICH == 2 && c >= 6) r = CT<R>::make(-r.x, -r.y);
        if (RES) {
          const C bv = sld(add + sp_base(site) + c * kTile);
          r = CT<R>::make(bv.x - r.x, bv.y - r.y);
        }
        if (LO != 0) {
          const float2 vf = make_float2((float)r.x, (float)r.y);
          float2 vs = vf;  // the stored value, as read back
          if (LO == 1) {
            lo32[sp_base(site) + c * kTile] = vf;
          } else {
            sst(lo16 + sp_base(site) + c * kTile, vf);
            vs = make_float2(__uint_as_float((unsigned)f2bf(vf.x) << 16), __uint_as_float((unsigned)f2bf(vf.y) << 16));
          }
          r = CT<R>::make((R)vs.x, (R)vs.y);
        } else {
          sst(op + c * kTile, r);
        }
        if (RED == 1) sred = fma(r.x, r.x, fma(r.y, r.y, sred));
        if (RED == 2) sred = fma(p.x, r.x, fma(p.y, r.y, sred));
      }
      if (RED == 1) red += (double)sred;
      if (RED == 2) red += (double)sred * sc;
#pragma unroll
      for (int c = 0; c < 12; ++c) cen[c] = nx[c];
    }
  }
  if (RED != 0) {
    __shared__ double lds[NT / 64];
    const double s = block_sum<NT>(red, lds);
    if (threadIdx.x == 0) part[(long)rhs * nbs + sb] = s;
  }
}

// Helpers of the slice-staged form: where hop h's neighbour comes from, and the loads of its
// spinor (raw storage values) and link, returned by value so they stay in registers.
struct HopSrc {
  bool near;    // the neighbour lies in the block's LDS slice
  unsigned li;  // its LDS index
  int d;        // site offset of the neighbour
};
template <class SV>
struct SpRaw {
  SV e[12];
};
template <class C>
struct Lk {
  C e[9];
};
template <int NT>
__device__ __forceinline__ HopSrc hop_src(int hh, int d, int s3, int base3, int V3) {
  const int mu = hh >> 1;
  const int nb3 = s3 + d;
  HopSrc r;
  r.d = d;
  r.li = (unsigned)(nb3 - base3);
  r.near = mu < 2 && r.li < (unsigned)NT && nb3 < V3;
  return r;
}
// Neighbour source for a block that is a box of whole x rows: Lx x by x bz sites of the
// slice, thread tid = lx + Lx (ly + by lz).  The x neighbour is always in the box (the box
// holds the whole periodic row); the y (z) neighbour is in it unless the site sits on the
// box's y (z) face, or the box spans the lattice in y (z), where the periodic neighbour is
// in the box again.  d is the neighbour's site offset, as for hop_src.
__device__ __forceinline__ HopSrc hop_src_box(int hh, int d, int tid, int Lx, int ly, int lz, int by, int bz,
                                              int Ly, int Lz) {
  const int mu = hh >> 1;
  const bool fwd = (hh & 1) == 0;
  HopSrc r;
  r.d = d;
  int dl;
  if (mu == 0) {
    r.near = true;
    dl = d;  // the row's own sites: lx + 1 or the periodic wrap, as in site numbering
  } else if (mu == 1) {
    const bool face = fwd ? ly == by - 1 : ly == 0;
    r.near = !face || by == Ly;
    dl = (face ? (fwd ? 1 - by : by - 1) : (fwd ? 1 : -1)) * Lx;
  } else {
    const bool face = fwd ? lz == bz - 1 : lz == 0;
    r.near = !face || bz == Lz;
    dl = (face ? (fwd ? 1 - bz : bz - 1) : (fwd ? 1 : -1)) * (Lx * by);
  }
  r.li = (unsigned)(tid + dl);
  return r;
}
template <class SV>
__device__ __forceinline__ SpRaw<SV> fetch_sp(const SV* __restrict__ in, int site) {
  SpRaw<SV> r;
  const SV* pp = in + sp_base(site);
#pragma unroll
  for (int c = 0; c < 12; ++c) r.e[c] = pp[c * kTile];
  return r;
}
// link of hop hh: forward hops use U_mu(x), backward hops U_mu(x - mu); with LK the x and y
// links of the block's sites come from LDS (pu: [2][9][NT])
template <bool LK, int NT, class C>
__device__ __forceinline__ Lk<C> fetch_link(const C* __restrict__ U, const C* pu, int hh, const HopSrc& src, int site,
                                            int tid) {
  const int mu = hh >> 1;
  const bool fwd = (hh & 1) == 0;
  Lk<C> r;
  if (LK && fwd && mu < 2) {
#pragma unroll
    for (int e = 0; e < 9; ++e) r.e[e] = pu[(mu * 9 + e) * NT + tid];
  } else if (LK && !fwd && src.near) {
#pragma unroll
    for (int e = 0; e < 9; ++e) r.e[e] = pu[(mu * 9 + e) * NT + src.li];
  } else {
    const C* up = U + lk_base(fwd ? site : site + src.d, mu);
#pragma unroll
    for (int e = 0; e < 9; ++e) r.e[e] = up[e * kTile];
  }
  return r;
}

// Time-marching form with the slice staged in LDS: a block is NT consecutive (x, y, z)
// sites of one time chunk of one rhs.  At each slice every thread writes its centre spinor
// and its forward x and y links to LDS; the x and y neighbours (and the backward x, y links)
// that fall inside the block's site range are then read from LDS instead of L2 (for a
// 16 x 16 plane per block that is all of them), the z neighbours and the z, t links come
// from memory, and the t hops are carried along t as in k_wilson_tm.  Same arithmetic and
// order as k_wilson.
// BOX: the block is instead a box of by x bz whole x rows (Lx by bz = NT, by | Ly, bz | Lz),
// so the z neighbours inside the box come from LDS as well; for a 16^3 or 32^3 slice a box
// of 4 x 4 or 4 x 2 rows leaves 1-1.5 neighbour spinors per site to memory instead of 2-2.25.
template <class R, class SV, int WHICH, int RED, int NT, bool LK, bool PF, bool BOX = false>
__global__ void __launch_bounds__(NT)
k_wilson_tmp(const typename CT<R>::type* __restrict__ U, const SV* __restrict__ in,
             SV* __restrict__ out, long fstride, int nrhs, double kappa, int Lx, int Ly, int Lz,
             int Lt, long V, long Vpad, int T, int nb3, int nbs, int order, const double* __restrict__ scale,
             const int* __restrict__ active, double* __restrict__ part, int boy, int boz) {
  static_assert(!(LK && BOX), "the staged links cover the x and y hops only");
  using C = typename CT<R>::type;
  __shared__ C ps[12 * NT];               // centre spinors of the block's sites, component-major
  __shared__ C pu[LK ? 2 * 9 * NT : 1];   // forward x and y links of the block's sites (LK)
  const int lb = order == 2 ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int rhs = order == 1 ? lb / nbs : lb % nrhs;
  const int sb = order == 1 ? lb % nbs : lb / nrhs;
  if (active && !active[rhs]) return;
  in += rhs * fstride;
  out += rhs * fstride;
  const int b3 = sb % nb3, tc = sb / nb3;
  const int V3 = Lx * Ly * Lz;
  const int base3 = b3 * NT;
  const int tid = (int)threadIdx.x;
  int s3 = base3 + tid, ly = 0, lz = 0;
  if (BOX) {
    const int nby = Ly / boy;
    ly = (tid / Lx) % boy;
    lz = tid / (Lx * boy);
    s3 = tid % Lx + Lx * ((b3 % nby) * boy + ly + Ly * ((b3 / nby) * boz + lz));
  }
  const bool valid = BOX || s3 < V3;
  double red = 0.0;
  if (b3 == 0 && (tc + 1) * T >= Lt) {
    for (long sp = V + tid; sp < Vpad; sp += NT) {
      SV* op = out + sp_base((int)sp);
#pragma unroll
      for (int c = 0; c < 12; ++c) sst(op + c * kTile, CT<R>::make(0, 0));
    }
  }
  int x = 0, y = 0, z = 0;
  if (valid) {
    x = s3 % Lx;
    y = (s3 / Lx) % Ly;
    z = s3 / (Lx * Ly);
  }
  const int sy = Lx, sz = Lx * Ly;
  const int fx = x == Lx - 1 ? 1 - Lx : 1, bx = x == 0 ? Lx - 1 : -1;
  const int fy = y == Ly - 1 ? (1 - Ly) * sy : sy, by = y == 0 ? (Ly - 1) * sy : -sy;
  const int fz = z == Lz - 1 ? (1 - Lz) * sz : sz, bz = z == 0 ? (Lz - 1) * sz : -sz;
  constexpr int SF = (WHICH == 1) ? 1 : -1;
  const int t0 = tc * T;
  const int t1 = t0 + T < Lt ? t0 + T : Lt;
  const R sc = scale ? (R)scale[rhs] : (R)1;
  const R mk = (R)(-kappa);
  C cen[12], gb[6];
  if (valid) {
    const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
    const int sprev = tp * V3 + s3;
    C p[12], h[6], u[9];
    const SV* pp = in + sp_base(sprev);
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = sld(pp + c * kTile);
    const C* up = U + lk_base(sprev, 3);
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = up[e * kTile];
    project<3, -SF>(p, h);
    mul_half<true>(u, h, gb);
    const SV* cp = in + sp_base(t0 * V3 + s3);
#pragma unroll
    for (int c = 0; c < 12; ++c) cen[c] = sld(cp + c * kTile);
  }
#pragma unroll 1
  for (int t = t0; t < t1; ++t) {
    const int site = t * V3 + s3;
    __syncthreads();  // the previous slice is no longer read from LDS
    if (valid) {
#pragma unroll
      for (int c = 0; c < 12; ++c) ps[c * NT + tid] = cen[c];
      if (LK) {
#pragma unroll
        for (int e = 0; e < 9; ++e) {
          pu[e * NT + tid] = U[lk_base(site, 0) + e * kTile];
          pu[(9 + e) * NT + tid] = U[lk_base(site, 1) + e * kTile];
        }
      }
    }
    __syncthreads();
    if (valid) {
      C acc[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = CT<R>::make(0, 0);
      const int snext = (t == Lt - 1 ? 0 : t + 1) * V3 + s3;
      C nx[12];
      // Hop h (0..5: x+, x-, y+, y-, z+, z-) reads the neighbour's spinor from LDS (near) or
      // memory, and its link.  PF: the memory loads of hop h + 1 are issued before hop h is
      // computed, so two hops' loads are in flight at once.
      auto hop_d = [=](int hh) {
        return hh == 0 ? fx : hh == 1 ? bx : hh == 2 ? fy : hh == 3 ? by : hh == 4 ? fz : bz;
      };
      auto src_of = [=](int hh) {
        return BOX ? hop_src_box(hh, hop_d(hh), tid, Lx, ly, lz, boy, boz, Ly, Lz)
                   : hop_src<NT>(hh, hop_d(hh), s3, base3, V3);
      };
      HopSrc nsrc{};
      SpRaw<SV> nraw{};
      Lk<C> nu{};
      if (PF) {
        nsrc = src_of(0);
        if (!nsrc.near) nraw = fetch_sp(in, site + nsrc.d);
        nu = fetch_link<LK, NT>(U, pu, 0, nsrc, site, tid);
      }
#pragma unroll 1
      for (int hop2 = 0; hop2 < 6; ++hop2) {
        const int mu = hop2 >> 1;
        const bool fwd = (hop2 & 1) == 0;
        C p[12], h[6], g[6], u[9];
        HopSrc src;
        SpRaw<SV> raw;
        Lk<C> lk;
        if (PF) {
          src = nsrc;
          raw = nraw;
          lk = nu;
          if (hop2 < 5) {
            nsrc = src_of(hop2 + 1);
            if (!nsrc.near) nraw = fetch_sp(in, site + nsrc.d);
            nu = fetch_link<LK, NT>(U, pu, hop2 + 1, nsrc, site, tid);
          }
        } else {
          src = src_of(hop2);
          if (!src.near) raw = fetch_sp(in, site + src.d);
          lk = fetch_link<LK, NT>(U, pu, hop2, src, site, tid);
        }
        if (src.near) {
#pragma unroll
          for (int c = 0; c < 12; ++c) p[c] = ps[c * NT + src.li];
        } else {
#pragma unroll
          for (int c = 0; c < 12; ++c) p[c] = sldv(raw.e[c]);
        }
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lk.e[e];
        if (fwd) {
          project_mu<SF>(mu, p, h);
          mul_half<false>(u, h, g);
          reconstruct_mu<SF>(mu, acc, g);
        } else {
          project_mu<-SF>(mu, p, h);
          mul_half<true>(u, h, g);
          reconstruct_mu<-SF>(mu, acc, g);
        }
      }
      C u[9];
      {
        {
          const SV* pp = in + sp_base(snext);
#pragma unroll
          for (int c = 0; c < 12; ++c) nx[c] = sld(pp + c * kTile);
        }
        const C* up = U + lk_base(site, 3);
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = up[e * kTile];
        C h[6], g[6];
        project<3, SF>(nx, h);
        mul_half<false>(u, h, g);
        reconstruct<3, SF>(acc, g);
        reconstruct<3, -SF>(acc, gb);
        project<3, -SF>(cen, h);
        mul_half<true>(u, h, gb);
      }
      SV* op = out + sp_base(site);
      R sred = 0;  // this site's share of the reduction, summed in R
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const C p = cen[c];
        C r = CT<R>::make(fma(mk, acc[c].x, p.x) * sc, fma(mk, acc[c].y, p.y) * sc);
        if (WHICH == 2 && c >= 6) r = CT<R>::make(-r.x, -r.y);
        sst(op + c * kTile, r);
        if (RED == 1) sred = fma(r.x, r.x, fma(r.y, r.y, sred));
        if (RED == 2) sred = fma(p.x, r.x, fma(p.y, r.y, sred));
      }
      if (RED == 1) red += (double)sred;
      if (RED == 2) red += (double)sred * sc;
#pragma unroll
      for (int c = 0; c < 12; ++c) cen[c] = nx[c];
    }
  }
  if (RED != 0) {
    __shared__ double lds[NT / 64];
    const double s2 = block_sum<NT>(red, lds);
    if (threadIdx.x == 0) part[(long)rhs * nbs + sb] = s2;
  }
}

// Multi-rhs time-marching form: a block is 64 consecutive (x, y, z) sites (one wave per
// rhs) of one time chunk for RB right-hand sides.  At each time slice the block stages
// the seven links its sites use from that slice (U_x, U_y, U_z at x, at x - mu for the
// backward hops, and U_t at x) in LDS once, and all RB waves read them from there, so a
// link leaves L2 once per RB right-hand sides instead of once per right-hand side.  The
// t hops are carried along t as in k_wilson_tm; the arithmetic and its order are the
// same as in k_wilson.  Logical block = (site block, rhs group).
template <class R, class SV, int WHICH, int RED, int RB>
__global__ void __launch_bounds__(64 * RB)
k_wilson_tml(const typename CT<R>::type* __restrict__ U, const SV* __restrict__ in,
             SV* __restrict__ out, long fstride, int nrhs, double kappa, int Lx, int Ly, int Lz,
             int Lt, long V, long Vpad, int T, int nb3, int nbs, int ngroups, int order,
             const double* __restrict__ scale, const int* __restrict__ active, double* __restrict__ part) {
  using C = typename CT<R>::type;
  constexpr int kSlots = 7, kL = kSlots * 9 * 64;
  __shared__ C lu[kL];
  const int lb = order == 2 ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int grp = order == 1 ? lb / nbs : lb % ngroups;
  const int sb = order == 1 ? lb % nbs : lb / ngroups;
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  const int rhs = grp * RB + w;
  bool any = false;
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const int r = grp * RB + q;
    any |= r < nrhs && (!active || active[r]);
  }
  if (!any) return;  // uniform over the block
  const bool on = rhs < nrhs && (!active || active[rhs]);
  const int b3 = sb % nb3, tc = sb / nb3;
  const int V3 = Lx * Ly * Lz;
  const int s3 = b3 * 64 + lane;
  const bool valid = s3 < V3;
  if (on) {
    in += rhs * fstride;
    out += rhs * fstride;
  }
  if (on && b3 == 0 && (tc + 1) * T >= Lt) {
    for (long sp = V + lane; sp < Vpad; sp += 64) {
      SV* op = out + sp_base((int)sp);
#pragma unroll
      for (int c = 0; c < 12; ++c) sst(op + c * kTile, CT<R>::make(0, 0));
    }
  }
  int x = 0, y = 0, z = 0;
  if (valid) {
    x = s3 % Lx;
    y = (s3 / Lx) % Ly;
    z = s3 / (Lx * Ly);
  }
  const int sy = Lx, sz = Lx * Ly;
  const int fx = x == Lx - 1 ? 1 - Lx : 1, bx = x == 0 ? Lx - 1 : -1;
  const int fy = y == Ly - 1 ? (1 - Ly) * sy : sy, by = y == 0 ? (Ly - 1) * sy : -sy;
  const int fz = z == Lz - 1 ? (1 - Lz) * sz : sz, bz = z == 0 ? (Lz - 1) * sz : -sz;
  constexpr int SF = (WHICH == 1) ? 1 : -1;
  const int t0 = tc * T;
  const int t1 = t0 + T < Lt ? t0 + T : Lt;
  const R sc = (on && scale) ? (R)scale[rhs] : (R)1;
  const R mk = (R)(-kappa);
  const bool work = on && valid;
  double red = 0.0;
  C cen[12], gb[6];
  if (work) {
    const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
    const int sprev = tp * V3 + s3;
    C p[12], h[6], u[9];
    const SV* pp = in + sp_base(sprev);
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c] = sld(pp + c * kTile);
    const C* up = U + lk_base(sprev, 3);
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = up[e * kTile];
    project<3, -SF>(p, h);
    mul_half<true>(u, h, gb);
    const SV* cp = in + sp_base(t0 * V3 + s3);
#pragma unroll
    for (int c = 0; c < 12; ++c) cen[c] = sld(cp + c * kTile);
  }
#pragma unroll 1
  for (int t = t0; t < t1; ++t) {
    const int site = t * V3 + s3;
    __syncthreads();  // the previous slice's links are no longer read
    if (valid) {
      // slot k: 0-2 U_mu(x), 3-5 U_mu(x - mu) for mu = x, y, z, 6 U_t(x); this thread loads
      // components of its own lane's site
      for (int q = w; q < kSlots * 9; q += RB) {
        const int slot = q / 9, e = q % 9;
        const int mu = slot < 3 ? slot : slot < 6 ? slot - 3 : 3;
        const int ls = slot < 3 || slot == 6 ? site : site + (mu == 0 ? bx : mu == 1 ? by : bz);
        lu[(slot * 9 + e) * 64 + lane] = U[lk_base(ls, mu) + e * kTile];
      }
    }
    __syncthreads();
    if (work) {
      C acc[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = CT<R>::make(0, 0);
#pragma unroll 1
      for (int mu = 0; mu < 3; ++mu) {
        const int df = mu == 0 ? fx : mu == 1 ? fy : fz;
        const int db = mu == 0 ? bx : mu == 1 ? by : bz;
        hop_at<SF, false>(lu + (mu * 9) * 64 + lane, 64, in, mu, site + df, acc);
        hop_at<-SF, true>(lu + ((3 + mu) * 9) * 64 + lane, 64, in, mu, site + db, acc);
      }
      const int snext = (t == Lt - 1 ? 0 : t + 1) * V3 + s3;
      C nx[12], u[9];
      {
        const SV* pp = in + sp_base(snext);
#pragma unroll
        for (int c = 0; c < 12; ++c) nx[c] = sld(pp + c * kTile);
#pragma unroll
        for (int e = 0; e < 9; ++e) u[e] = lu[(6 * 9 + e) * 64 + lane];
        C h[6], g[6];
        project<3, SF>(nx, h);
        mul_half<false>(u, h, g);
        reconstruct<3, SF>(acc, g);
        reconstruct<3, -SF>(acc, gb);
        project<3, -SF>(cen, h);
        mul_half<true>(u, h, gb);
      }
      SV* op = out + sp_base(site);
      R sred = 0;  // this site's share of the reduction, summed in R
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const C p = cen[c];
        C r = CT<R>::make(fma(mk, acc[c].x, p.x) * sc, fma(mk, acc[c].y, p.y) * sc);
        if (WHICH == 2 && c >= 6) r = CT<R>::make(-r.x, -r.y);
        sst(op + c * kTile, r);
        if (RED == 1) sred = fma(r.x, r.x, fma(r.y, r.y, sred));
        if (RED == 2) sred = fma(p.x, r.x, fma(p.y, r.y, sred));
      }
      if (RED == 1) red += (double)sred;
      if (RED == 2) red += (double)sred * sc;
#pragma unroll
      for (int c = 0; c < 12; ++c) cen[c] = nx[c];
    }
  }
  if (RED != 0) {
    red = wave_sum(red);
    if (lane == 0 && on) part[(long)rhs * nbs + sb] = red;
  }
}

// Several right-hand sides per thread: a thread owns one site and RT consecutive rhs of a
// group; each hop's link is loaded once into registers and applied to the RT neighbour
// spinors, so links and neighbour offsets are read and computed once per site for the group
// (the one-rhs-per-block forms read each site's links once per rhs, from L2 at best) and the
// RT spinor loads of a hop are independent and in flight together.  Logical block = (site
// block, rhs group), order as k_wilson.  Same arithmetic and hop order as k_wilson per rhs.
template <class R, class SV, int WHICH, int RED, int NT, int RT>
__global__ void __launch_bounds__(NT)
k_wilson_mr(const typename CT<R>::type* __restrict__ U, const SV* __restrict__ in,
            SV* __restrict__ out, long fstride, int nrhs, double kappa, int Lx, int Ly, int Lz,
            int Lt, long V, long Vpad, int nbs, int ngroups, int order, const double* __restrict__ scale,
            const int* __restrict__ active, double* __restrict__ part) {
  using C = typename CT<R>::type;
  const int lb = order == 2 ? (int)blockIdx.x : xcd_block(blockIdx.x, gridDim.x);
  const int rg = order == 1 ? lb / nbs : lb % ngroups;
  const int sb = order == 1 ? lb % nbs : lb / ngroups;
  const int r0 = rg * RT;
  bool on[RT];
  bool any = false;
#pragma unroll
  for (int j = 0; j < RT; ++j) {
    on[j] = r0 + j < nrhs && (!active || active[r0 + j]);
    any |= on[j];
  }
  if (!any) return;
  const int site = sb * NT + (int)threadIdx.x;
  double red[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) red[j] = 0.0;
  if (site >= V && site < Vpad) {
#pragma unroll
    for (int j = 0; j < RT; ++j)
      if (on[j]) {
        SV* op = out + (r0 + j) * fstride + sp_base(site);
#pragma unroll
        for (int c = 0; c < 12; ++c) sst(op + c * kTile, CT<R>::make(0, 0));
      }
  }
  if (site < V) {
    const int x = site % Lx;
    const int y = (site / Lx) % Ly;
    const int z = (site / (Lx * Ly)) % Lz;
    const int t = site / (Lx * Ly * Lz);
    const int sy = Lx, sz = Lx * Ly, st = Lx * Ly * Lz;
    const int fx = x == Lx - 1 ? 1 - Lx : 1, bx = x == 0 ? Lx - 1 : -1;
    const int fy = y == Ly - 1 ? (1 - Ly) * sy : sy, by = y == 0 ? (Ly - 1) * sy : -sy;
    const int fz = z == Lz - 1 ? (1 - Lz) * sz : sz, bz = z == 0 ? (Lz - 1) * sz : -sz;
    const int ft = t == Lt - 1 ? (1 - Lt) * st : st, bt = t == 0 ? (Lt - 1) * st : -st;
    C acc[RT][12];
#pragma unroll
    for (int j = 0; j < RT; ++j)
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[j][c] = CT<R>::make(0, 0);
    constexpr int SF = (WHICH == 1) ? 1 : -1;
#pragma unroll 1
    for (int hh = 0; hh < 8; ++hh) {
      const int mu = hh >> 1;
      const bool fwd = (hh & 1) == 0;
      const int d = fwd ? (mu == 0 ? fx : mu == 1 ? fy : mu == 2 ? fz : ft)
                        : (mu == 0 ? bx : mu == 1 ? by : mu == 2 ? bz : bt);
      const int nb = site + d;
      C u[9];
      const C* up = U + lk_base(fwd ? site : nb, mu);
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = up[e * kTile];
      const SV* pb = in + sp_base(nb);
#pragma unroll
      for (int j = 0; j < RT; ++j) {
        if (!on[j]) continue;
        C p[12], h[6], g[6];
        const SV* pp = pb + (r0 + j) * fstride;
#pragma unroll
        for (int c = 0; c < 12; ++c) p[c] = sld(pp + c * kTile);
        if (fwd) {
          project_mu<SF>(mu, p, h);
          mul_half<false>(u, h, g);
          reconstruct_mu<SF>(mu, acc[j], g);
        } else {
          project_mu<-SF>(mu, p, h);
          mul_half<true>(u, h, g);
          reconstruct_mu<-SF>(mu, acc[j], g);
        }
      }
    }
    const R mk = (R)(-kappa);
#pragma unroll
    for (int j = 0; j < RT; ++j) {
      if (!on[j]) continue;
      const R sc = scale ? (R)scale[r0 + j] : (R)1;
      const SV* ip = in + (r0 + j) * fstride + sp_base(site);
      SV* op = out + (r0 + j) * fstride + sp_base(site);
      R sred = 0;
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        const C p = sld(ip + c * kTile);
        C r = CT<R>::make(fma(mk, acc[j][c].x, p.x) * sc, fma(mk, acc[j][c].y, p.y) * sc);
        if (WHICH == 2 && c >= 6) r = CT<R>::make(-r.x, -r.y);
        sst(op + c * kTile, r);
        if (RED == 1) sred = fma(r.x, r.x, fma(r.y, r.y, sred));
        if (RED == 2) sred = fma(p.x, r.x, fma(p.y, r.y, sred));
      }
      if (RED == 1) red[j] = (double)sred;
      if (RED == 2) red[j] = (double)sred * sc;
    }
  }
  if (RED != 0) {
    __shared__ double lds[NT / 64];
#pragma unroll
    for (int j = 0; j < RT; ++j) {
      if (!on[j]) continue;  // uniform over the block
      const double s = block_sum<NT>(red[j], lds);
      if (threadIdx.x == 0) part[(long)(r0 + j) * nbs + sb] = s;
      __syncthreads();  // lds is reused by the next rhs's sum
    }
  }
}

// Launch-shape variants.  0-3: k_wilson with (threads per block, occupancy hint)
// {(256,2), (128,2), (512,1), (256,1)}; 4-6: k_wilson_tm, 256 threads per block, time
// chunks of T = 4, 8, 16 slices; 7-10: k_wilson_tml with 64 sites per block and
// (rhs per block, T) = (4, 8), (4, 16), (8, 8), (2, 8).
// 15-17: k_wilson_mr with (threads per block, rhs per thread) = (256, 2), (256, 4), (128, 2).
// 18-19: k_wilson_tmp with box blocks of whole x rows (T = 8, 16); where no box tiles the
// slice they launch variants 12 and 13.
static constexpr int kVariantNT[kWilsonVariants] = {256, 128, 512, 256, 256, 256, 256, 64, 64, 64, 64, 256, 256, 256, 256,
                                                    256, 256, 128, 256, 256};
static constexpr int kVariantT[kWilsonVariants] = {0, 0, 0, 0, 4, 8, 16, 8, 16, 8, 8, 8, 8, 16, 8, 0, 0, 0, 8, 16};
static constexpr int kVariantRT[kWilsonVariants] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 4, 2, 1, 1};

static int tm_nb3(const Lattice& lat, int v) {
  return (lat.L[0] * lat.L[1] * lat.L[2] + kVariantNT[v] - 1) / kVariantNT[v];
}
static int tm_chunks(const Lattice& lat, int v) { return (lat.L[3] + kVariantT[v] - 1) / kVariantT[v]; }

template <class R, class SV, int WHICH, int RED, int NT>
static void launch_tm(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, const SV* in,
                      SV* out, long fstride, int nrhs, int order, const double* scale, const int* active,
                      double* part, int nbs, int v) {
  const int* L = lat.L;
  hipLaunchKernelGGL((k_wilson_tm<R, SV, WHICH, RED, NT>), dim3(nbs * nrhs), dim3(NT), 0, s, U, in, out, fstride, nrhs,
                     kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, kVariantT[v], tm_nb3(lat, v), nbs,
                     order, scale, active, part, static_cast<const SV*>(nullptr), static_cast<void*>(nullptr));
}

template <class R, class SV, int WHICH, int RED, int NT, int OCC>
static void launch_one(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, const SV* in,
                       SV* out, long fstride, int nrhs, int order, const double* scale, const int* active,
                       double* part, int nbs) {
  const int* L = lat.L;
  hipLaunchKernelGGL((k_wilson<R, SV, WHICH, RED, NT, OCC>), dim3(nbs * nrhs), dim3(NT), 0, s, U, in, out, fstride, nrhs,
                     kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, nbs, order, scale, active, part);
}

// Box of whole x rows for k_wilson_tmp<..., BOX>: y and z extents (by, bz) with
// Lx by bz = nt, by | Ly and bz | Lz, chosen for the fewest neighbour spinors outside the box
// per site (2 / by for the y faces unless by = Ly, 2 / bz for the z faces unless bz = Lz; a
// tie goes to the larger by, the longer contiguous run of sites).  False if no box fits.
static bool tmp_box(const Lattice& lat, int nt, int* by, int* bz) {
  const int* L = lat.L;
  if (L[0] > nt || nt % L[0] != 0) return false;
  const int rows = nt / L[0];
  double best = 1e300;
  bool found = false;
  for (int y = 1; y <= rows; ++y) {
    if (rows % y != 0 || L[1] % y != 0) continue;
    const int z = rows / y;
    if (L[2] % z != 0) continue;
    const double cost = (y < L[1] ? 2.0 / y : 0.0) + (z < L[2] ? 2.0 / z : 0.0);
    if (cost <= best) {
      best = cost;
      *by = y;
      *bz = z;
      found = true;
    }
  }
  return found;
}

template <class R, class SV, int WHICH, int RED, int NT, bool LK, bool PF, bool BOX = false>
static void launch_tmp(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, const SV* in,
                       SV* out, long fstride, int nrhs, int order, const double* scale, const int* active,
                       double* part, int nbs, int v) {
  const int* L = lat.L;
  int by = 0, bz = 0;
  if (BOX && !tmp_box(lat, NT, &by, &bz)) {
    // no box tiles this slice: the same chunks with blocks of consecutive sites
    launch_tmp<R, SV, WHICH, RED, NT, LK, PF, false>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active,
                                                     part, nbs, v);
    return;
  }
  hipLaunchKernelGGL((k_wilson_tmp<R, SV, WHICH, RED, NT, LK, PF, BOX>), dim3(nbs * nrhs), dim3(NT), 0, s, U, in,
                     out, fstride, nrhs, kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, kVariantT[v],
                     tm_nb3(lat, v), nbs, order, scale, active, part, by, bz);
}

template <class R, class SV, int WHICH, int RED, int RB>
static void launch_tml(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, const SV* in,
                       SV* out, long fstride, int nrhs, int order, const double* scale, const int* active,
                       double* part, int nbs, int v) {
  const int* L = lat.L;
  const int ngroups = (nrhs + RB - 1) / RB;
  hipLaunchKernelGGL((k_wilson_tml<R, SV, WHICH, RED, RB>), dim3(nbs * ngroups), dim3(64 * RB), 0, s, U, in, out,
                     fstride, nrhs, kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, kVariantT[v],
                     tm_nb3(lat, v), nbs, ngroups, order, scale, active, part);
}

template <class R, class SV, int WHICH, int RED, int NT, int RT>
static void launch_mr(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, const SV* in, SV* out,
                      long fstride, int nrhs, int order, const double* scale, const int* active, double* part,
                      int nbs) {
  const int* L = lat.L;
  const int ngroups = (nrhs + RT - 1) / RT;
  hipLaunchKernelGGL((k_wilson_mr<R, SV, WHICH, RED, NT, RT>), dim3(nbs * ngroups), dim3(NT), 0, s, U, in, out,
                     fstride, nrhs, kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, nbs, ngroups, order,
                     scale, active, part);
}

template <class R, class SV, int WHICH, int RED>
static void launch_variant(int variant, hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa,
                           const SV* in, SV* out, long fstride, int nrhs, int order,
                           const double* scale, const int* active, double* part, int nbs) {
  switch (variant) {
    case 1: launch_one<R, SV, WHICH, RED, 128, 2>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs); break;
    case 2: launch_one<R, SV, WHICH, RED, 512, 1>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs); break;
    case 3: launch_one<R, SV, WHICH, RED, 256, 1>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs); break;
    case 4: case 5: case 6:
      launch_tm<R, SV, WHICH, RED, 256>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs, variant);
      break;
    case 7: case 8:
      launch_tml<R, SV, WHICH, RED, 4>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs, variant);
      break;
    case 9:
      launch_tml<R, SV, WHICH, RED, 8>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs, variant);
      break;
    case 10:
      launch_tml<R, SV, WHICH, RED, 2>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs, variant);
      break;
    case 11:
      // FP64 spinors and links of a slice together exceed the LDS budget: the FP64 form stages spinors only
      if constexpr (sizeof(R) == 4)
        launch_tmp<R, SV, WHICH, RED, 256, true, false>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale,
                                                        active, part, nbs, variant);
      else
        launch_tmp<R, SV, WHICH, RED, 256, false, false>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale,
                                                         active, part, nbs, variant);
      break;
    case 12: case 13:
      launch_tmp<R, SV, WHICH, RED, 256, false, false>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active,
                                                       part, nbs, variant);
      break;
    case 18: case 19:
      launch_tmp<R, SV, WHICH, RED, 256, false, false, true>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale,
                                                             active, part, nbs, variant);
      break;
    case 14:
      launch_tmp<R, SV, WHICH, RED, 256, false, true>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active,
                                                      part, nbs, variant);
      break;
    case 15:
      launch_mr<R, SV, WHICH, RED, 256, 2>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs);
      break;
    case 16:
      launch_mr<R, SV, WHICH, RED, 256, 4>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs);
      break;
    case 17:
      launch_mr<R, SV, WHICH, RED, 128, 2>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs);
      break;
    default: launch_one<R, SV, WHICH, RED, 256, 2>(s, lat, U, kappa, in, out, fstride, nrhs, order, scale, active, part, nbs); break;
  }
}

// ---- even-odd (Schur complement) operator ---------------------------------------------
// Half fields hold the sites of one parity p(x) = (x + y + z + t) mod 2 in increasing full-site
// order; with every extent even the half index of a site is site / 2.  One thread per output
// half site; logical block = (site block, rhs), rhs fastest.

template <class C>
__device__ __forceinline__ C czero() {
  C z;
  z.x = 0;
  z.y = 0;
  return z;
}

// full coordinates of half site h of parity par
__device__ __forceinline__ void eo_coords(int h, int par, int Lx, int Ly, int Lz, int& x, int& y, int& z, int& t) {
  const int lxh = Lx >> 1;
  const int xh = h % lxh, r = h / lxh;
  y = r % Ly;
  z = (r / Ly) % Lz;
  t = r / (Ly * Lz);
  x = 2 * xh + ((par + y + z + t) & 1);
}

// acc = D_{par, 1-par} applied at half site h (input: half field of the other parity, in storage SV)
template <int SF, class C, class SV>
__device__ __forceinline__ void eo_hops(const C* __restrict__ U, const SV* __restrict__ in, int h, int par, int Lx,
                                        int Ly, int Lz, int Lt, C acc[12]) {
  int x, y, z, t;
  eo_coords(h, par, Lx, Ly, Lz, x, y, z, t);
  const int sy = Lx, sz = Lx * Ly, st = Lx * Ly * Lz;
  const int site = x + sy * y + sz * z + st * t;
  const int fx = x == Lx - 1 ? 1 - Lx : 1, bx = x == 0 ? Lx - 1 : -1;
  const int fy = y == Ly - 1 ? (1 - Ly) * sy : sy, by = y == 0 ? (Ly - 1) * sy : -sy;
  const int fz = z == Lz - 1 ? (1 - Lz) * sz : sz, bz = z == 0 ? (Lz - 1) * sz : -sz;
  const int ft = t == Lt - 1 ? (1 - Lt) * st : st, bt = t == 0 ? (Lt - 1) * st : -st;
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = czero<C>();
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    const int df = mu == 0 ? fx : mu == 1 ? fy : mu == 2 ? fz : ft;
    const int db = mu == 0 ? bx : mu == 1 ? by : mu == 2 ? bz : bt;
    hop<SF, false>(U, in, mu, (site + df) >> 1, site, acc);
    hop<-SF, true>(U, in, mu, (site + db) >> 1, site + db, acc);
  }
}

// Stage 1: tmp (arithmetic precision) = D_{1-par0, par0} in for the rhs of the launch.
template <class R, class SV, int WHICH>
__global__ void __launch_bounds__(256)
k_eo_hop1(const typename CT<R>::type* __restrict__ U, const SV* __restrict__ in, typename CT<R>::type* __restrict__ tmp,
          long fstride, int nrhs, int Lx, int Ly, int Lz, int Lt, long V, long Vpad, int par,
          const int* __restrict__ active) {
  using C = typename CT<R>::type;
  const int rhs = (int)blockIdx.x % nrhs, sb = (int)blockIdx.x / nrhs;
  if (active && !active[rhs]) return;
  const int h = sb * 256 + (int)threadIdx.x;
  C* op = tmp + rhs * fstride;
  if (h >= V && h < Vpad) {
#pragma unroll
    for (int c = 0; c < 12; ++c) op[sp_base(h) + c * kTile] = czero<C>();
  }
  if (h >= V) return;
  constexpr int SF = (WHICH == 1) ? 1 : -1;
  C acc[12];
  eo_hops<SF>(U, in + rhs * fstride, h, par, Lx, Ly, Lz, Lt, acc);
#pragma unroll
  for (int c = 0; c < 12; ++c) op[sp_base(h) + c * kTile] = acc[c];
}

// Stage 2: out = scale * (in - kappa^2 D_{par, 1-par} tmp) (gamma5 on the result for WHICH 2), with
// the fused reduction of the result (RED 1: ||out||^2, RED 2: Re<in, out>) per block.
template <class R, class SV, int WHICH, int RED>
__global__ void __launch_bounds__(256)
k_eo_schur(const typename CT<R>::type* __restrict__ U, const typename CT<R>::type* __restrict__ tmp,
           const SV* __restrict__ in, SV* __restrict__ out, long fstride, int nrhs, double kappa2, int Lx, int Ly,
           int Lz, int Lt, long V, long Vpad, int par, int nbs, const double* __restrict__ scale,
           const int* __restrict__ active, double* __restrict__ part) {
  using C = typename CT<R>::type;
  const int rhs = (int)blockIdx.x % nrhs, sb = (int)blockIdx.x / nrhs;
  if (active && !active[rhs]) return;
  const int h = sb * 256 + (int)threadIdx.x;
  SV* op = out + rhs * fstride;
  double red = 0.0;
  if (h >= V && h < Vpad) {
#pragma unroll
    for (int c = 0; c < 12; ++c) sst(op + sp_base(h) + c * kTile, CT<R>::make(0, 0));
  }
  if (h < V) {
    constexpr int SF = (WHICH == 1) ? 1 : -1;
    C acc[12];
    eo_hops<SF>(U, tmp + rhs * fstride, h, par, Lx, Ly, Lz, Lt, acc);
    const R sc = scale ? (R)scale[rhs] : (R)1;
    const R mk = (R)(-kappa2);
    const SV* ip = in + rhs * fstride + sp_base(h);
    R sred = 0;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const C p = sld(ip + c * kTile);
      C r = CT<R>::make(fma(mk, acc[c].x, p.x) * sc, fma(mk, acc[c].y, p.y) * sc);
      if (WHICH == 2 && c >= 6) r = CT<R>::make(-r.x, -r.y);
      sst(op + sp_base(h) + c * kTile, r);
      if (RED == 1) sred = fma(r.x, r.x, fma(r.y, r.y, sred));
      if (RED == 2) sred = fma(p.x, r.x, fma(p.y, r.y, sred));
    }
    if (RED == 1) red = (double)sred;
    if (RED == 2) red = (double)sred * sc;
  }
  if (RED != 0) {
    __shared__ double lds[256 / 64];
    const double s = block_sum<256>(red, lds);
    if (threadIdx.x == 0) part[(long)rhs * nbs + sb] = s;
  }
}

namespace {
std::mutex g_eo_mu;
std::map<hipStream_t, DBuf<char>> g_eo_scratch;
}  // namespace

void eo_reserve(hipStream_t s, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_eo_mu);
  DBuf<char>& b = g_eo_scratch[s];
  if (b.n < bytes) b.alloc(bytes);
}

void eo_release(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_eo_mu);
  g_eo_scratch.erase(s);
}

static void* eo_buffer(hipStream_t s, size_t bytes) {
  eo_reserve(s, bytes);
  std::lock_guard<std::mutex> lk(g_eo_mu);
  return g_eo_scratch[s].get();
}

template <class R, class SV>
static int wilson_eo(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, int which, const SV* in,
                     SV* out, long fstride, int nrhs, int red, const double* scale, const int* active, double* part) {
  using C = cplx_t<R>;
  const int nbs = (int)((lat.V + 255) / 256);
  if (red && nbs > kMaxPartials) fail(DL_E_INVALID, "lattice too large for fused reduction");
  C* tmp = static_cast<C*>(eo_buffer(s, (size_t)nrhs * fstride * sizeof(C)));
  const int* L = lat.L;
  const long Vpad = lat.ntiles * kTile;
  const dim3 grid((unsigned)((long)nbs * nrhs)), block(256);
  // stage 1: odd intermediate D_oe in (par 1 output); stage 2: even result
#define DL_EO1(WH) hipLaunchKernelGGL((k_eo_hop1<R, SV, WH>), grid, block, 0, s, U, in, tmp, fstride, nrhs, L[0], L[1], \
                                      L[2], L[3], lat.V, Vpad, 1, active)
#define DL_EO2(WH, RD) hipLaunchKernelGGL((k_eo_schur<R, SV, WH, RD>), grid, block, 0, s, U, tmp, in, out, fstride, \
                                          nrhs, kappa * kappa, L[0], L[1], L[2], L[3], lat.V, Vpad, 0, nbs, scale, \
                                          active, part)
  if (which == 1) DL_EO1(1); else DL_EO1(0);
  if (which == 0) { if (red == 0) DL_EO2(0, 0); else if (red == 1) DL_EO2(0, 1); else DL_EO2(0, 2); }
  else if (which == 1) { if (red == 0) DL_EO2(1, 0); else if (red == 1) DL_EO2(1, 1); else DL_EO2(1, 2); }
  else { if (red == 0) DL_EO2(2, 0); else if (red == 1) DL_EO2(2, 1); else DL_EO2(2, 2); }
#undef DL_EO1
#undef DL_EO2
  DL_HIP(hipGetLastError());
  return red ? nbs : 0;
}

__global__ void k_eo_split(const double2* __restrict__ in, double2* __restrict__ half, long nc_full, long nc_half,
                           long Vh, int par, int Lx, int Ly, int Lz) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long f = blockIdx.y;
  if (i >= Vh * kSpin) return;
  const int h = (int)(i / kSpin), c = (int)(i % kSpin);
  int x, y, z, t;
  eo_coords(h, par, Lx, Ly, Lz, x, y, z, t);
  const int site = x + Lx * (y + Ly * (z + Lz * t));
  half[f * nc_half + sp_base(h) + c * kTile] = in[f * nc_full + sp_base(site) + c * kTile];
}

__global__ void k_eo_merge(const double2* __restrict__ half, double2* __restrict__ out, long nc_full, long nc_half,
                           long Vh, int par, int Lx, int Ly, int Lz) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long f = blockIdx.y;
  if (i >= Vh * kSpin) return;
  const int h = (int)(i / kSpin), c = (int)(i % kSpin);
  int x, y, z, t;
  eo_coords(h, par, Lx, Ly, Lz, x, y, z, t);
  const int site = x + Lx * (y + Ly * (z + Lz * t));
  out[f * nc_full + sp_base(site) + c * kTile] = half[f * nc_half + sp_base(h) + c * kTile];
}

// out = fac * D_{par, 1-par} in + add (FP64, one field)
__global__ void __launch_bounds__(256)
k_eo_hop_f64(const double2* __restrict__ U, const double2* __restrict__ in, const double2* __restrict__ add,
             double2* __restrict__ out, double fac, int Lx, int Ly, int Lz, int Lt, long V, long Vpad, int par) {
  const int h = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (h >= V && h < Vpad) {
#pragma unroll
    for (int c = 0; c < 12; ++c) out[sp_base(h) + c * kTile] = make_double2(0.0, 0.0);
  }
  if (h >= V) return;
  double2 acc[12];
  eo_hops<-1>(U, in, h, par, Lx, Ly, Lz, Lt, acc);
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    const double2 a = add ? add[sp_base(h) + c * kTile] : make_double2(0.0, 0.0);
    out[sp_base(h) + c * kTile] = make_double2(fma(fac, acc[c].x, a.x), fma(fac, acc[c].y, a.y));
  }
}

void eo_split(hipStream_t s, const Lattice& full, const double2* in, double2* half, int par, int nfield) {
  if (nfield <= 0) return;
  const Lattice hl = make_lattice_eo(full.L);
  const long n = hl.V * kSpin;
  hipLaunchKernelGGL(k_eo_split, dim3((unsigned)((n + 255) / 256), nfield), dim3(256), 0, s, in, half, full.nc,
                     hl.nc, hl.V, par, full.L[0], full.L[1], full.L[2]);
  DL_HIP(hipGetLastError());
}

void eo_merge(hipStream_t s, const Lattice& full, const double2* half, double2* out, int par, int nfield) {
  if (nfield <= 0) return;
  const Lattice hl = make_lattice_eo(full.L);
  const long n = hl.V * kSpin;
  hipLaunchKernelGGL(k_eo_merge, dim3((unsigned)((n + 255) / 256), nfield), dim3(256), 0, s, half, out, full.nc,
                     hl.nc, hl.V, par, full.L[0], full.L[1], full.L[2]);
  DL_HIP(hipGetLastError());
}

void eo_hop_f64(hipStream_t s, const Lattice& lat, const double2* U, double fac, int par, const double2* in,
                const double2* add, double2* out) {
  const int* L = lat.L;
  hipLaunchKernelGGL(k_eo_hop_f64, dim3((unsigned)((lat.V + 255) / 256)), dim3(256), 0, s, U, in, add, out, fac, L[0],
                     L[1], L[2], L[3], lat.V, lat.ntiles * kTile, par);
  DL_HIP(hipGetLastError());
}

int wilson_residual_f64(hipStream_t s, const Lattice& lat, const double2* U, double kappa, const double2* x,
                        const double2* b, double2* r, long fstride, int nrhs, const int* active, double* part,
                        void* lo, int lo_prec) {
  if (lat.eo) fail(DL_E_INVALID, "the fused residual serves whole-lattice operators");
  if ((lo == nullptr) == (r == nullptr)) fail(DL_E_INVALID, "the fused residual goes to r or to lo");
  constexpr int v = 6;  // time-marching, 256 threads, chunks of 16 slices
  const int nbs = tm_nb3(lat, v) * tm_chunks(lat, v);
  if (nbs > kMaxPartials) fail(DL_E_INVALID, "lattice too large for fused reduction");
  if ((long)nbs * nrhs > 2147483647L) fail(DL_E_INVALID, "grid too large");
  const int* L = lat.L;
#define DL_RES(LOP)                                                                                                 \
  hipLaunchKernelGGL((k_wilson_tm<double, double2, 0, 1, 256, true, LOP>), dim3(nbs * nrhs), dim3(256), 0, s, U, x,  \
                     r, fstride, nrhs, kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, kVariantT[v],       \
                     tm_nb3(lat, v), nbs, 2, static_cast<const double*>(nullptr), active, part, b, lo)
  if (!lo) DL_RES(0);
  else if (lo_prec == DL_FP32) DL_RES(1);
  else if (lo_prec == DL_BF16) DL_RES(2);
  else fail(DL_E_INVALID, "lo_prec must be DL_FP32 or DL_BF16");
#undef DL_RES
  DL_HIP(hipGetLastError());
  return nbs;
}

int wilson_nbs(const Lattice& lat, const WilsonCfg& cfg) {
  if (lat.eo) return (int)((lat.V + 255) / 256);
  const int v = cfg.variant % kWilsonVariants;
  if (kVariantT[v] > 0) return tm_nb3(lat, v) * tm_chunks(lat, v);
  const int nt = kVariantNT[v];
  return (int)((lat.V + nt - 1) / nt);
}

int wilson_max_nbs(const Lattice& lat) {
  int m = 0;
  for (int v = 0; v < kWilsonVariants; ++v) m = std::max(m, wilson_nbs(lat, WilsonCfg{v, 0}));
  return m;
}

template <class R, class SV>
int wilson_batched(hipStream_t s, const Lattice& lat, const cplx_t<R>* U, double kappa, int which,
                   const SV* in, SV* out, long fstride, int nrhs, int red, const double* scale,
                   const int* active, double* part, WilsonCfg cfg) {
  if (lat.eo) return wilson_eo<R, SV>(s, lat, U, kappa, which, in, out, fstride, nrhs, red, scale, active, part);
  const int v = cfg.variant % kWilsonVariants;
  const int nbs = wilson_nbs(lat, cfg);
  if (red && nbs > kMaxPartials) fail(DL_E_INVALID, "lattice too large for fused reduction");
  if ((long)nbs * ((nrhs + kVariantRT[v] - 1) / kVariantRT[v]) > 2147483647L) fail(DL_E_INVALID, "grid too large");
  const int o = cfg.order;
#define DL_W(WH, RD) launch_variant<R, SV, WH, RD>(v, s, lat, U, kappa, in, out, fstride, nrhs, o, scale, active, part, nbs)
  if (which == 0) { if (red == 0) DL_W(0, 0); else if (red == 1) DL_W(0, 1); else DL_W(0, 2); }
  else if (which == 1) { if (red == 0) DL_W(1, 0); else if (red == 1) DL_W(1, 1); else DL_W(1, 2); }
  else { if (red == 0) DL_W(2, 0); else if (red == 1) DL_W(2, 1); else DL_W(2, 2); }
#undef DL_W
  DL_HIP(hipGetLastError());
  return red ? nbs : 0;
}

template int wilson_batched<double, double2>(hipStream_t, const Lattice&, const double2*, double, int, const double2*,
                                             double2*, long, int, int, const double*, const int*, double*, WilsonCfg);
template int wilson_batched<float, float2>(hipStream_t, const Lattice&, const float2*, double, int, const float2*,
                                           float2*, long, int, int, const double*, const int*, double*, WilsonCfg);
template int wilson_batched<float, bf2>(hipStream_t, const Lattice&, const float2*, double, int, const bf2*, bf2*,
                                        long, int, int, const double*, const int*, double*, WilsonCfg);

int wilson_f64(hipStream_t s, const Lattice& lat, const double2* U, double kappa, int which,
               const double2* in, double2* out, int red, double* part, WilsonCfg cfg) {
  return wilson_batched<double, double2>(s, lat, U, kappa, which, in, out, lat.nc, 1, red, nullptr, nullptr, part, cfg);
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
