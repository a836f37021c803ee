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
// coalesced 1 KiB wavefront access; neighbour spinors and the backward links
// are re-read through L2 (blocks are mapped so that each XCD walks a
// contiguous slab of the lattice, keeping the +-z/+-t neighbours in its L2).
#include "internal.hpp"
#include "cplx.hpp"

namespace dl {

__device__ __forceinline__ long sp_idx(long site, int c) {
  return ((site >> 6) * kSpin + c) * kTile + (site & 63);
}
__device__ __forceinline__ long lk_idx(long site, int mu, int e) {
  return ((site >> 6) * kLinkC + mu * 9 + e) * kTile + (site & 63);
}

template <int MU, int S>
__device__ __forceinline__ void project(const double2 p[12], double2 h[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double2 p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
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

template <int MU, int S>
__device__ __forceinline__ void reconstruct(double2 acc[12], const double2 g[6]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double2 g0 = g[c], g1 = g[3 + c];
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

// g = U h (per spin row) for the forward hop, U loaded from `site`.
__device__ __forceinline__ void mul_u(const double2* __restrict__ U, long site, int mu,
                                      const double2 h[6], double2 g[6]) {
  double2 u[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[lk_idx(site, mu, e)];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double2 r = c_mul(u[a * 3 + 0], h[s * 3 + 0]);
      r = c_fma(u[a * 3 + 1], h[s * 3 + 1], r);
      r = c_fma(u[a * 3 + 2], h[s * 3 + 2], r);
      g[s * 3 + a] = r;
    }
}

// g = U^dag h for the backward hop, U loaded from `site` (= x - mu).
__device__ __forceinline__ void mul_udag(const double2* __restrict__ U, long site, int mu,
                                         const double2 h[6], double2 g[6]) {
  double2 u[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) u[e] = U[lk_idx(site, mu, e)];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double2 r = make_double2(0.0, 0.0);
      r = c_fmac(u[0 * 3 + a], h[s * 3 + 0], r);
      r = c_fmac(u[1 * 3 + a], h[s * 3 + 1], r);
      r = c_fmac(u[2 * 3 + a], h[s * 3 + 2], r);
      g[s * 3 + a] = r;
    }
}

__device__ __forceinline__ void load_spinor(const double2* __restrict__ in, long site, double2 p[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) p[c] = in[sp_idx(site, c)];
}

template <int MU, int SF>
__device__ __forceinline__ void hop_dir(const double2* __restrict__ U, const double2* __restrict__ in,
                                        long site, long fwd, long bwd, double2 acc[12]) {
  double2 p[12], h[6], g[6];
  // forward: (1 + SF g_mu) U_mu(x) psi(x + mu)
  load_spinor(in, fwd, p);
  project<MU, SF>(p, h);
  mul_u(U, site, MU, h, g);
  reconstruct<MU, SF>(acc, g);
  // backward: (1 - SF g_mu) U_mu(x - mu)^dag psi(x - mu)
  load_spinor(in, bwd, p);
  project<MU, -SF>(p, h);
  mul_udag(U, bwd, MU, h, g);
  reconstruct<MU, -SF>(acc, g);
}

// WHICH: 0 M, 1 M^dag, 2 gamma5 M.  RED: 0 none, 1 ||out||^2, 2 Re<in, out>.
template <int WHICH, int RED>
__global__ void __launch_bounds__(kBlock)
k_wilson_f64(const double2* __restrict__ U, const double2* __restrict__ in, double2* __restrict__ out,
             double kappa, int Lx, int Ly, int Lz, int Lt, long V, long Vpad, double* __restrict__ part) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const long site = (long)lb * kBlock + threadIdx.x;
  double red = 0.0;
  if (site >= V && site < Vpad) {
    // padding sites of the last tile are kept at zero
#pragma unroll
    for (int c = 0; c < 12; ++c) out[sp_idx(site, c)] = make_double2(0.0, 0.0);
  }
  if (site < V) {
    const int x = site % Lx;
    const int y = (site / Lx) % Ly;
    const int z = (site / ((long)Lx * Ly)) % Lz;
    const int t = site / ((long)Lx * Ly * Lz);
    const long sy = Lx, sz = (long)Lx * Ly, st = (long)Lx * Ly * Lz;
    const long xf = site + (x == Lx - 1 ? 1 - Lx : 1), xb = site + (x == 0 ? Lx - 1 : -1);
    const long yf = site + (y == Ly - 1 ? (1 - Ly) * sy : sy), yb = site + (y == 0 ? (Ly - 1) * sy : -sy);
    const long zf = site + (z == Lz - 1 ? (1 - Lz) * sz : sz), zb = site + (z == 0 ? (Lz - 1) * sz : -sz);
    const long tf = site + (t == Lt - 1 ? (1 - Lt) * st : st), tb = site + (t == 0 ? (Lt - 1) * st : -st);
    double2 acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = make_double2(0.0, 0.0);
    constexpr int SF = (WHICH == 1) ? 1 : -1;  // forward projector sign
    hop_dir<0, SF>(U, in, site, xf, xb, acc);
    hop_dir<1, SF>(U, in, site, yf, yb, acc);
    hop_dir<2, SF>(U, in, site, zf, zb, acc);
    hop_dir<3, SF>(U, in, site, tf, tb, acc);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      const double2 p = in[sp_idx(site, c)];
      double2 r = make_double2(fma(-kappa, acc[c].x, p.x), fma(-kappa, acc[c].y, p.y));
      if (WHICH == 2 && c >= 6) r = make_double2(-r.x, -r.y);
      out[sp_idx(site, c)] = r;
      if (RED == 1) red += r.x * r.x + r.y * r.y;
      if (RED == 2) red += p.x * r.x + p.y * r.y;
    }
  }
  if (RED != 0) {
    __shared__ double lds[kBlock / 64];
    const double s = block_sum<kBlock>(red, lds);
    if (threadIdx.x == 0) part[lb] = s;
  }
}

template <int WHICH>
static void launch_which(hipStream_t s, const Lattice& lat, const double2* U, double kappa,
                         const double2* in, double2* out, int red, double* part, int nb) {
  const dim3 grid(nb), block(kBlock);
  const int* L = lat.L;
  if (red == 0)
    hipLaunchKernelGGL((k_wilson_f64<WHICH, 0>), grid, block, 0, s, U, in, out, kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, part);
  else if (red == 1)
    hipLaunchKernelGGL((k_wilson_f64<WHICH, 1>), grid, block, 0, s, U, in, out, kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, part);
  else
    hipLaunchKernelGGL((k_wilson_f64<WHICH, 2>), grid, block, 0, s, U, in, out, kappa, L[0], L[1], L[2], L[3], lat.V, lat.ntiles * kTile, part);
}

int wilson_f64(hipStream_t s, const Lattice& lat, const double2* U, double kappa, int which,
               const double2* in, double2* out, int red, double* part) {
  const int nb = (int)((lat.V + kBlock - 1) / kBlock);
  if (red && nb > kMaxPartials) fail(DL_E_INVALID, "lattice too large for fused reduction");
  if (which == 0) launch_which<0>(s, lat, U, kappa, in, out, red, part, nb);
  else if (which == 1) launch_which<1>(s, lat, U, kappa, in, out, red, part, nb);
  else launch_which<2>(s, lat, U, kappa, in, out, red, part, nb);
  DL_HIP(hipGetLastError());
  return red ? nb : 0;
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
