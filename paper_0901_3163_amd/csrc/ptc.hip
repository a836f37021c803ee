// Gauge-covariant parallel-transport convolution network (learned initial guess), FP32.
//
// Activations are colour triplets per site and channel in the tiled layout
//     elem(site, ch, col) = ((site / 64) * (C * 3) + ch * 3 + col) * 64 + site % 64
// (for C = 4 this is the spinor layout with spin as channel).  A layer computes
//     out[o](x) = sum_h sum_i W_h[o][i] (T_h in[i])(x)
// over the nine hops h = 0, +x, -x, +y, -y, +z, -z, +t, -t, with T_0 = 1,
// (T_{+mu} a)(x) = U_mu(x) a(x + mu) and (T_{-mu} a)(x) = U_mu(x - mu)^dag a(x - mu),
// optionally followed by f(z) = z / sqrt(1 + |z|^2) per site and channel (|z| the
// gauge-invariant colour norm).  Widths 4 -> 16 -> 16 -> 4; the input is scaled by
// 1/s with s the root-mean-square site norm of b over its nonzero sites and the output
// by s, so net(c b) = c net(b) and point and extended sources both enter at unit scale.
//
// Backward pass: the adjoint of T_h is T_{-h} and channel mixing commutes with the
// transport, so the data gradient is the forward kernel with W'_{-h} = W_h^H.  The
// weight gradient G_W[h][o][i] = sum_x sum_c G_out[o](x)_c conj((T_h in[i])(x)_c)
// is accumulated per 64-site chunk from LDS in FP64 and reduced in a fixed order.
#include "ptc.hpp"
#include "small.hpp"
#include "tsk.hpp"
#include "cplx.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace dl {

namespace {

__device__ __forceinline__ long act_idx(int site, int C, int ch, int col) {
  return ((long)(site >> 6) * (C * 3) + ch * 3 + col) * kTile + (site & 63);
}
__device__ __forceinline__ long lnk_idx(int site, int mu, int e) {
  return ((long)(site >> 6) * kLinkC + mu * 9 + e) * kTile + (site & 63);
}

// Neighbour of `site` along hop h (1..8: +x, -x, +y, -y, +z, -z, +t, -t), the hop's direction
// and whether it is forward.  The link of a forward hop sits at `site`, of a backward hop at nb.
__device__ __forceinline__ void hop_geom(int h, int site, int Lx, int Ly, int Lz, int Lt, int& nb, int& mu,
                                         bool& fwd) {
  mu = (h - 1) >> 1;
  fwd = ((h - 1) & 1) == 0;
  const int st = mu == 0 ? 1 : mu == 1 ? Lx : mu == 2 ? Lx * Ly : Lx * Ly * Lz;
  const int L = mu == 0 ? Lx : mu == 1 ? Ly : mu == 2 ? Lz : Lt;
  const int c = (site / st) % L;
  if (fwd) nb = c == L - 1 ? site - (L - 1) * st : site + st;
  else nb = c == 0 ? site + (L - 1) * st : site - st;
}

// tr = U a (forward hop) or U^dag a (backward hop)
__device__ __forceinline__ void transport3(const float2 u[9], bool fwd, const float2 a[3], float2 tr[3]) {
  if (fwd) {
#pragma unroll
    for (int r = 0; r < 3; ++r) tr[r] = c_fma(u[r * 3 + 2], a[2], c_fma(u[r * 3 + 1], a[1], c_mul(u[r * 3], a[0])));
  } else {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      float2 v = c_fmac(u[0 * 3 + r], a[0], make_float2(0.f, 0.f));
      v = c_fmac(u[1 * 3 + r], a[1], v);
      tr[r] = c_fmac(u[2 * 3 + r], a[2], v);
    }
  }
}

// One network layer over `gridDim.y` fields: thread = site.  W ([9][COUT][CIN]) is staged in LDS.
// NONLIN: out = f(z), z saved to zsave if given; else out = out_scale[item] * z (out_scale may be NULL).
template <int CIN, int COUT, bool NONLIN>
__global__ void __launch_bounds__(256)
k_ptc_layer(const float2* __restrict__ U, const float2* __restrict__ in, float2* __restrict__ out,
            float2* __restrict__ zsave, const float2* __restrict__ W, int Lx, int Ly, int Lz, int Lt, int V,
            int Vpad, long in_stride, long out_stride, const double* __restrict__ out_scale) {
  __shared__ float2 ws[9 * COUT * CIN];
  for (int e = threadIdx.x; e < 9 * COUT * CIN; e += blockDim.x) ws[e] = W[e];
  __syncthreads();
  const int item = blockIdx.y;
  in += item * in_stride;
  out += item * out_stride;
  if (zsave) zsave += item * out_stride;
  const int site = blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= Vpad) return;
  if (site >= V) {  // padding sites stay zero
    for (int o = 0; o < COUT; ++o)
      for (int c = 0; c < 3; ++c) {
        out[act_idx(site, COUT, o, c)] = make_float2(0.f, 0.f);
        if (zsave) zsave[act_idx(site, COUT, o, c)] = make_float2(0.f, 0.f);
      }
    return;
  }
  float2 acc[COUT][3];
#pragma unroll
  for (int o = 0; o < COUT; ++o)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[o][c] = make_float2(0.f, 0.f);
#pragma unroll 1
  for (int h = 0; h < 9; ++h) {
    int nb = site, mu = 0;
    bool fwd = true;
    float2 u[9];
    if (h > 0) {
      hop_geom(h, site, Lx, Ly, Lz, Lt, nb, mu, fwd);
      const int ls = fwd ? site : nb;
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = U[lnk_idx(ls, mu, e)];
    }
    const float2* wh = ws + h * COUT * CIN;
#pragma unroll 2
    for (int i = 0; i < CIN; ++i) {
      float2 a[3], tr[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) a[c] = in[act_idx(nb, CIN, i, c)];
      if (h == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) tr[c] = a[c];
      } else {
        transport3(u, fwd, a, tr);
      }
#pragma unroll
      for (int o = 0; o < COUT; ++o) {
        const float2 w = wh[o * CIN + i];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[o][c] = c_fma(w, tr[c], acc[o][c]);
      }
    }
  }
  const float sc = out_scale ? (float)out_scale[item] : 1.f;
#pragma unroll
  for (int o = 0; o < COUT; ++o) {
    if (NONLIN) {
      float n2 = 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) n2 += acc[o][c].x * acc[o][c].x + acc[o][c].y * acc[o][c].y;
      const float g = 1.f / sqrtf(1.f + n2);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (zsave) zsave[act_idx(site, COUT, o, c)] = acc[o][c];
        out[act_idx(site, COUT, o, c)] = c_scale(acc[o][c], g);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) out[act_idx(site, COUT, o, c)] = c_scale(acc[o][c], sc);
    }
  }
}

// ---- 16 -> 16 layer with BF16 channel mixing on the matrix cores (inference) ------------------
//
// Per wave: one tile of 64 sites.  For each hop the wave transports its 16 input channels (FP32,
// one thread per site), rounds them to BF16 and stages them in LDS; the channel mixing is then
// the real form of a complex product: with K = (channel i, re/im) interleaved (32 per hop) and
// rows m < 16 the real parts, m >= 16 the imaginary parts of the 16 output channels,
//     A[o][2i] = Re W, A[o][2i+1] = -Im W, A[16+o][2i] = Im W, A[16+o][2i+1] = Re W,
// and out[m][(site, colour)] += sum_k A[m][k] T[k][(site, colour)] on v_mfma_f32_32x32x16_bf16:
// six 32-column tiles (3 colours x 2 halves of the tile's sites) and two K-steps per hop, FP32
// accumulation over all nine hops.  Lane l supplies row / column l % 32 and K-slice 8 * (l / 32)
// of both operands; the result register j of lane l is row 8 (j / 4) + 4 (l / 32) + j % 4, so a
// lane holds the real and imaginary parts of 8 output channels for the 3 colours of two sites,
// which is all the per-channel non-linearity needs.
typedef __bf16 bf16x8_n __attribute__((ext_vector_type(8)));
typedef float f32x16_n __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4_n __attribute__((ext_vector_type(4)));
typedef float f32x2_n __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_n __attribute__((ext_vector_type(2)));

constexpr int kMixRow = 40;  // BF16 entries per (colour, site) row of the LDS stage (32 used; 80 B keeps 16 B alignment)

__device__ __forceinline__ unsigned pack_bf16x2(float a, float b) {
  const f32x2_n f = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2_n));
}

// A fragments of a 16 -> 16 layer: frag[(h * 2 + ks) * 64 + lane] = 8 BF16 entries
// A[m = lane % 32][k = 16 ks + 8 (lane / 32) + j], j = 0..7.
__global__ void k_ptc_wfrag16(const float2* __restrict__ W, u32x4_n* __restrict__ frag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 9 * 2 * 64) return;
  const int lane = t % 64, hk = t / 64, h = hk / 2, ks = hk % 2;
  const int m = lane % 32, kb = 16 * ks + 8 * (lane / 32);
  float v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kk = kb + j, i = kk / 2, p = kk % 2;
    const int o = m % 16;
    const float2 w = W[(h * 16 + o) * 16 + i];
    v[j] = m < 16 ? (p == 0 ? w.x : -w.y) : (p == 0 ? w.y : w.x);
  }
  u32x4_n r;
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = pack_bf16x2(v[2 * q], v[2 * q + 1]);
  frag[t] = r;
}

template <bool NONLIN>
__global__ void __launch_bounds__(256)
k_ptc_layer16_mfma(const float2* __restrict__ U, const float2* __restrict__ in, float2* __restrict__ out,
                   const u32x4_n* __restrict__ frag, int Lx, int Ly, int Lz, int Lt, int V, int ntiles,
                   long in_stride, long out_stride, const double* __restrict__ out_scale) {
  __shared__ unsigned short stage[4][3][64 * kMixRow];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int tile = blockIdx.x * 4 + wid;
  const int item = blockIdx.y;
  if (tile >= ntiles) return;  // whole waves only: no barrier below spans waves
  in += item * in_stride;
  out += item * out_stride;
  const int site = tile * 64 + lane;
  const bool valid = site < V;
  unsigned short* st = &stage[wid][0][0];
  f32x16_n acc[6];
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[q][j] = 0.f;
  const int g = lane >> 5, col = lane & 31;
#pragma unroll 1
  for (int h = 0; h < 9; ++h) {
    int nb = site, mu = 0;
    bool fwd = true;
    float2 u[9];
    if (valid && h > 0) {
      hop_geom(h, site, Lx, Ly, Lz, Lt, nb, mu, fwd);
      const int ls = fwd ? site : nb;
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = U[lnk_idx(ls, mu, e)];
    }
    // transport the 16 channels of this site's neighbour, BF16 into the stage [colour][site][k]
#pragma unroll 2
    for (int i = 0; i < 16; ++i) {
      float2 a[3], tr[3];
      if (valid) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c] = in[act_idx(nb, 16, i, c)];
        if (h == 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) tr[c] = a[c];
        } else {
          transport3(u, fwd, a, tr);
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) tr[c] = make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c)
        *reinterpret_cast<unsigned*>(st + (c * 64 + lane) * kMixRow + 2 * i) = pack_bf16x2(tr[c].x, tr[c].y);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const u32x4_n af = frag[(h * 2 + ks) * 64 + lane];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int half = 0; half < 2; ++half) {
          const u32x4_n bf = *reinterpret_cast<const u32x4_n*>(st + (c * 64 + half * 32 + col) * kMixRow + 16 * ks +
                                                               8 * g);
          acc[c * 2 + half] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8_n, af), __builtin_bit_cast(bf16x8_n, bf), acc[c * 2 + half], 0, 0, 0);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  // epilogue: lane holds rows 8q + 4g + r (q, r < 4) of the six tiles: channel o = 8 (q % 2) + 4g + r,
  // real part for q < 2, imaginary part (row 16 + o) for q >= 2
  const float sc = out_scale ? (float)out_scale[item] : 1.f;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int s2 = tile * 64 + half * 32 + col;
    const bool ok = s2 < V;
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = 8 * q + 4 * g + r;
        float2 z[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) z[c] = make_float2(acc[c * 2 + half][4 * q + r], acc[c * 2 + half][4 * (q + 2) + r]);
        float gsc = sc;
        if (NONLIN) {
          float n2 = 0.f;
#pragma unroll
          for (int c = 0; c < 3; ++c) n2 += z[c].x * z[c].x + z[c].y * z[c].y;
          gsc = 1.f / sqrtf(1.f + n2);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) out[act_idx(s2, 16, o, c)] = ok ? c_scale(z[c], gsc) : make_float2(0.f, 0.f);
      }
  }
}

// Backward of f: G_z = g G_f + 2 g' Re<G_f, z> z with g(s) = (1 + s)^-1/2, s = |z|^2 (in place on G).
__global__ void k_ptc_nonlin_bwd(const float2* __restrict__ zs, float2* __restrict__ G, int C, int V, long stride) {
  const int item = blockIdx.y;
  zs += item * stride;
  G += item * stride;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;  // (site, channel)
  if (idx >= (long)V * C) return;
  const int site = (int)(idx / C), ch = (int)(idx % C);
  float2 z[3], g[3];
  float n2 = 0.f, re = 0.f;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    z[c] = zs[act_idx(site, C, ch, c)];
    g[c] = G[act_idx(site, C, ch, c)];
    n2 += z[c].x * z[c].x + z[c].y * z[c].y;
    re += g[c].x * z[c].x + g[c].y * z[c].y;
  }
  const float gf = 1.f / sqrtf(1.f + n2);
  const float dgf = -0.5f * gf * gf * gf;
#pragma unroll
  for (int c = 0; c < 3; ++c) G[act_idx(site, C, ch, c)] = c_axpy(2.f * dgf * re, z[c], c_scale(g[c], gf));
}

// Adjoint weights of a [9][cout][cin] layer: Wt[rev(h)][i][o] = conj(W[h][o][i]).
__global__ void k_ptc_adjoint_weights(const float2* __restrict__ W, float2* __restrict__ Wt, int cin, int cout) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 9 * cout * cin) return;
  const int h = e / (cout * cin), o = (e / cin) % cout, i = e % cin;
  const int rh = h == 0 ? 0 : (((h - 1) & 1) == 0 ? h + 1 : h - 1);
  const float2 w = W[e];
  Wt[((long)rh * cin + i) * cout + o] = make_float2(w.x, -w.y);
}

// Weight-gradient partials: block (chunk group, hop h, item); thread p = (o, i) for p < COUT*CIN.
// The block walks chunks blockIdx.x, blockIdx.x + gridDim.x, ... staging the transported inputs
// and output gradients of each 64-site chunk in LDS.  part layout:
//   part[((item * 9 + h) * COUT * CIN + p) * 2 * gridDim.x + {block (re), gridDim.x + block (im)}]
template <int CIN, int COUT>
__global__ void __launch_bounds__(256)
k_ptc_wgrad(const float2* __restrict__ U, const float2* __restrict__ in, const float2* __restrict__ G, int Lx,
            int Ly, int Lz, int Lt, int V, int nchunks, long in_stride, long g_stride, double* __restrict__ part) {
  __shared__ float2 tl[64][CIN][3];
  __shared__ float2 gl[64][COUT][3];
  const int h = blockIdx.y, item = blockIdx.z;
  in += item * in_stride;
  G += item * g_stride;
  const int p = threadIdx.x;
  const int o = p / CIN, i = p % CIN;
  double re = 0.0, im = 0.0;
  for (int chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    for (int e = threadIdx.x; e < 64 * CIN; e += blockDim.x) {
      const int ls = e / CIN, ci = e % CIN;
      const int site = chunk * 64 + ls;
      float2 tr[3] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
      if (site < V) {
        int nb = site, mu = 0;
        bool fwd = true;
        if (h > 0) hop_geom(h, site, Lx, Ly, Lz, Lt, nb, mu, fwd);
        float2 a[3];
        for (int c = 0; c < 3; ++c) a[c] = in[act_idx(nb, CIN, ci, c)];
        if (h == 0) {
          for (int c = 0; c < 3; ++c) tr[c] = a[c];
        } else {
          float2 u[9];
          const int lsite = fwd ? site : nb;
          for (int q = 0; q < 9; ++q) u[q] = U[lnk_idx(lsite, mu, q)];
          transport3(u, fwd, a, tr);
        }
      }
      for (int c = 0; c < 3; ++c) tl[ls][ci][c] = tr[c];
    }
    for (int e = threadIdx.x; e < 64 * COUT; e += blockDim.x) {
      const int ls = e / COUT, co = e % COUT;
      const int site = chunk * 64 + ls;
      for (int c = 0; c < 3; ++c) gl[ls][co][c] = site < V ? G[act_idx(site, COUT, co, c)] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    if (p < COUT * CIN) {
      for (int ls = 0; ls < 64; ++ls)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float2 g = gl[ls][o][c], a = tl[ls][i][c];
          re += (double)g.x * a.x + (double)g.y * a.y;  // g * conj(a)
          im += (double)g.y * a.x - (double)g.x * a.y;
        }
    }
    __syncthreads();
  }
  if (p < COUT * CIN) {
    const long base = (((long)item * 9 + h) * COUT * CIN + p) * 2 * gridDim.x;
    part[base + blockIdx.x] = re;
    part[base + gridDim.x + blockIdx.x] = im;
  }
}

// grad[e] = sum over items and blocks of the partials of entry e = (h, o, i), fixed order.
__global__ void k_ptc_wgrad_reduce(const double* __restrict__ part, int nitems, int nentries, int nblk,
                                   float2* __restrict__ grad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nentries) return;
  double re = 0.0, im = 0.0;
  for (int it = 0; it < nitems; ++it) {
    const long base = ((long)it * nentries + e) * 2 * nblk;
    for (int c = 0; c < nblk; ++c) {
      re += part[base + c];
      im += part[base + nblk + c];
    }
  }
  grad[e] = make_float2((float)re, (float)im);
}

// Adam with bias correction on each real component.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per item: ||b||^2 partials (part[item * gridDim.x + block]) and partial counts of the sites
// where b is nonzero (part[(nitems + item) * gridDim.x + block]); thread = site of the tiled field.
__global__ void __launch_bounds__(kBlock) k_site_stats(const double2* __restrict__ a, long nc, long Vpad,
                                                         int nitems, double* __restrict__ part) {
  const int item = blockIdx.y;
  a += item * nc;
  double acc = 0.0, cnt = 0.0;
  for (long site = (long)blockIdx.x * kBlock + threadIdx.x; site < Vpad; site += (long)gridDim.x * kBlock) {
    const long base = (site >> 6) * (kSpin * kTile) + (site & 63);
    double n2 = 0.0;
#pragma unroll
    for (int c = 0; c < kSpin; ++c) {
      const double2 v = a[base + c * kTile];
      n2 += v.x * v.x + v.y * v.y;
    }
    acc += n2;
    cnt += n2 > 0.0 ? 1.0 : 0.0;
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  __syncthreads();
  const double c = block_sum<kBlock>(cnt, lds);
  if (threadIdx.x == 0) {
    part[(long)item * gridDim.x + blockIdx.x] = s;
    part[(long)(nitems + item) * gridDim.x + blockIdx.x] = c;
  }
}
// per-item ||a||^2 partials of FP32 fields
__global__ void __launch_bounds__(kBlock) k_norm2_items_f32(const float2* __restrict__ a, long n,
                                                              double* __restrict__ part) {
  const int item = blockIdx.y;
  double acc = 0.0;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
    const float2 v = a[item * n + i];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  __shared__ double lds[kBlock / 64];
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) part[(long)item * gridDim.x + blockIdx.x] = s;
}
// Input scale per item: the root-mean-square site norm over the sites where b is nonzero,
// s = sqrt(||b||^2 / n_nonzero), inv_s = 1/s (0 for b = 0), bn2 = ||b||^2; one thread per item.
__global__ void k_net_scales(const double* __restrict__ part, int nparts, int nitems, double* s, double* inv_s,
                             double* bn2) {
  const int it = blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= nitems) return;
  double t = 0.0, c = 0.0;
  for (int g = 0; g < nparts; ++g) {
    t += part[(long)it * nparts + g];
    c += part[(long)(nitems + it) * nparts + g];
  }
  const double sv = c > 0.0 ? sqrt(t / c) : 0.0;
  s[it] = sv;
  inv_s[it] = sv > 0.0 ? 1.0 / sv : 0.0;
  bn2[it] = t;
}
// b32 = (float)(b64 * sc[item])
__global__ void k_to_f32_scaled(const double2* __restrict__ a, float2* __restrict__ b, long n,
                                const double* __restrict__ sc) {
  const int item = blockIdx.y;
  const double s = sc[item];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double2 v = a[item * n + i];
    b[item * n + i] = make_float2((float)(v.x * s), (float)(v.y * s));
  }
}
__global__ void k_to_f64(const float2* __restrict__ a, double2* __restrict__ b, long n) {
  const int item = blockIdx.y;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    b[item * n + i] = make_double2(a[item * n + i].x, a[item * n + i].y);
}
// d = y - x (FP32 minus FP64, rounded to FP32)
__global__ void k_sub_f32_f64(const float2* __restrict__ y, const double2* __restrict__ x, float2* __restrict__ d,
                              long n) {
  const int item = blockIdx.y;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long k = item * n + i;
    d[k] = make_float2((float)((double)y[k].x - x[k].x), (float)((double)y[k].y - x[k].y));
  }
}
__global__ void k_scale_items_f32(float2* a, long n, const float* __restrict__ sc) {
  const int item = blockIdx.y;
  const float s = sc[item];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[item * n + i] = c_scale(a[item * n + i], s);
}

constexpr int kStreamBlocks = 512;  // blocks per item of the streaming kernels here
constexpr int kStatBlocks = 128;    // blocks per item of the site statistics
constexpr int kWgradBlocks = 64;    // chunk groups of the weight-gradient kernel

long act_len(const Lattice& lat, int C) { return lat.ntiles * kTile * C * 3; }

void launch_layer(hipStream_t s, const Lattice& lat, const float2* U, const float2* in, float2* out, float2* zsave,
                  const float2* W, int cin, int cout, bool nonlin, int nitems, const double* out_scale) {
  const int Vpad = (int)(lat.ntiles * kTile);
  const dim3 grid((unsigned)((Vpad + 255) / 256), nitems), block(256);
  const int* L = lat.L;
  const long is = act_len(lat, cin), os = act_len(lat, cout);
  const int V = (int)lat.V;
#define DL_LAYER(CI, CO, NL)                                                                                  \
  hipLaunchKernelGGL((k_ptc_layer<CI, CO, NL>), grid, block, 0, s, U, in, out, zsave, W, L[0], L[1], L[2], L[3], \
                     V, Vpad, is, os, out_scale)
  if (cin == 4 && cout == 16) {
    if (nonlin) DL_LAYER(4, 16, true); else DL_LAYER(4, 16, false);
  } else if (cin == 16 && cout == 16) {
    if (nonlin) DL_LAYER(16, 16, true); else DL_LAYER(16, 16, false);
  } else if (cin == 16 && cout == 4) {
    if (nonlin) DL_LAYER(16, 4, true); else DL_LAYER(16, 4, false);
  } else {
    fail(DL_E_INVALID, "unsupported layer width");
  }
#undef DL_LAYER
  DL_HIP(hipGetLastError());
}

// G (entries 9*cout*cin) = weight gradient of a layer with input `in` and output gradient `g`.
void layer_wgrad(hipStream_t s, const Lattice& lat, const float2* U, const float2* in, const float2* g, int cin,
                 int cout, int nitems, double* part, float2* G) {
  const int nblk = (int)std::min<long>(lat.ntiles, kWgradBlocks);
  const dim3 grid(nblk, 9, nitems), block(256);
  const int* L = lat.L;
  const long is = act_len(lat, cin), gs = act_len(lat, cout);
  const int V = (int)lat.V, nch = (int)lat.ntiles;
  if (cin == 4 && cout == 16)
    hipLaunchKernelGGL((k_ptc_wgrad<4, 16>), grid, block, 0, s, U, in, g, L[0], L[1], L[2], L[3], V, nch, is, gs,
                       part);
  else if (cin == 16 && cout == 16)
    hipLaunchKernelGGL((k_ptc_wgrad<16, 16>), grid, block, 0, s, U, in, g, L[0], L[1], L[2], L[3], V, nch, is, gs,
                       part);
  else
    hipLaunchKernelGGL((k_ptc_wgrad<16, 4>), grid, block, 0, s, U, in, g, L[0], L[1], L[2], L[3], V, nch, is, gs,
                       part);
  const int ne = 9 * cout * cin;
  hipLaunchKernelGGL(k_ptc_wgrad_reduce, dim3((ne + 255) / 256), dim3(256), 0, s, part, nitems, ne, nblk, G);
  DL_HIP(hipGetLastError());
}

// Forward pass; activations of layers 1, 2 (and pre-activations if keep) stay in net->acts.
void forward(dl_net* net, dl_op* op, int nitems, const double2* B, float2* Y, bool keep, bool bf16 = false) {
  hipStream_t s = net->ctx->stream;
  const Lattice& lat = op->lat;
  NetActs& a = net->acts;
  a.ensure(lat, nitems);
  const float2* U = op_links32_public(op);
  const long n = lat.nc;
  hipLaunchKernelGGL(k_site_stats, dim3(kStatBlocks, nitems), dim3(kBlock), 0, s, B, n, lat.ntiles * kTile, nitems,
                     a.part.get());
  hipLaunchKernelGGL(k_net_scales, dim3((nitems + 63) / 64), dim3(64), 0, s, a.part.get(), kStatBlocks, nitems,
                     a.s.get(), a.inv_s.get(), a.bn2.get());
  hipLaunchKernelGGL(k_to_f32_scaled, dim3(kStreamBlocks, nitems), dim3(256), 0, s, B, a.a0.get(), n,
                     (const double*)a.inv_s.get());
  DL_HIP(hipGetLastError());
  const float2* W = net->W.get();
  launch_layer(s, lat, U, a.a0.get(), a.a1.get(), keep ? a.z1.get() : nullptr, W + net_weight_offset(0), 4, 16, true,
               nitems, nullptr);
  if (bf16 && !keep) {
    // inference: the 16 -> 16 layer's channel mixing in BF16 on the matrix cores
    if (net->frag16.n < (size_t)9 * 2 * 64 * 4) net->frag16.alloc((size_t)9 * 2 * 64 * 4);
    u32x4_n* fr = reinterpret_cast<u32x4_n*>(net->frag16.get());
    hipLaunchKernelGGL(k_ptc_wfrag16, dim3((9 * 2 * 64 + 255) / 256), dim3(256), 0, s, W + net_weight_offset(1), fr);
    const int* L = lat.L;
    const int ntiles = (int)lat.ntiles;
    hipLaunchKernelGGL((k_ptc_layer16_mfma<true>), dim3((ntiles + 3) / 4, nitems), dim3(256), 0, s, U, a.a1.get(),
                       a.a2.get(), fr, L[0], L[1], L[2], L[3], (int)lat.V, ntiles, act_len(lat, 16),
                       act_len(lat, 16), nullptr);
    DL_HIP(hipGetLastError());
  } else {
    launch_layer(s, lat, U, a.a1.get(), a.a2.get(), keep ? a.z2.get() : nullptr, W + net_weight_offset(1), 16, 16,
                 true, nitems, nullptr);
  }
  launch_layer(s, lat, U, a.a2.get(), Y, nullptr, W + net_weight_offset(2), 16, 4, false, nitems, a.s.get());
}

}  // namespace

int net_num_weights() {
  int n = 0;
  for (int l = 0; l < kNetLayers; ++l) n += 9 * kNetWidth[l + 1] * kNetWidth[l];
  return n;
}

long net_weight_offset(int layer) {
  long o = 0;
  for (int q = 0; q < layer; ++q) o += 9 * kNetWidth[q + 1] * kNetWidth[q];
  return o;
}

void NetActs::ensure(const Lattice& lat, int nitems) {
  if (items >= nitems && nc == lat.nc) return;
  items = nitems;
  nc = lat.nc;
  const size_t l4 = (size_t)act_len(lat, 4), l16 = (size_t)act_len(lat, 16);
  a0.alloc(nitems * l4);
  z1.alloc(nitems * l16);
  a1.alloc(nitems * l16);
  z2.alloc(nitems * l16);
  a2.alloc(nitems * l16);
  g16a.alloc(nitems * l16);
  g16b.alloc(nitems * l16);
  g4.alloc(nitems * l4);
  y.alloc(nitems * l4);
  r.alloc(nitems * l4);
  const size_t wg = (size_t)9 * 256 * 2 * kWgradBlocks;
  part.alloc((size_t)nitems * std::max<size_t>(wg, kStreamBlocks));
  s.alloc(nitems);
  inv_s.alloc(nitems);
  bn2.alloc(nitems);
  gsc.alloc(nitems);
}

void net_apply(dl_net* net, dl_op* op, int nitems, const double2* B, double2* Y64, bool bf16) {
  net->acts.ensure(op->lat, nitems);
  forward(net, op, nitems, B, net->acts.y.get(), false, bf16);
  hipLaunchKernelGGL(k_to_f64, dim3(kStreamBlocks, nitems), dim3(256), 0, net->ctx->stream, net->acts.y.get(), Y64,
                     op->lat.nc);
  DL_HIP(hipGetLastError());
}

// d' = d - Y H^-1 Y^H (M^dag M d) for the error fields d (FP32, in acts.g4): the part of the
// guess's error that the D-CG start (net(b), then the Galerkin projection over Y) leaves.  The
// loss ||M d'||^2 then has gradient M^dag M d' with respect to d (the projection is orthogonal
// in the M^dag M inner product), so the backward pass below is unchanged.
__global__ void k_negate(long n, double2* a) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a[i] = make_double2(-a[i].x, -a[i].y);
}

static void project_error(dl_net* net, dl_op* op, int nitems) {
  const dl_eig* e = net->proj;
  if (e->fingerprint != op->fingerprint || e->kind != op->kind)
    fail(DL_E_MISMATCH, "the training projection's eigenvectors belong to another operator");
  if (op->kind != DL_MDAGM) fail(DL_E_INVALID, "the projected training loss is the D-CG one (M^dag M operators)");
  hipStream_t s = net->ctx->stream;
  const Lattice& lat = op->lat;
  const long n = lat.nc, tot = (long)nitems * n;
  NetActs& a = net->acts;
  const float2* U = op_links32_public(op);
  const WilsonCfg cfg = wilson_cfg(op, DL_FP32, nitems);
  // A d (FP32 stencils) in a.g16a, widened; d widened
  wilson_batched<float>(s, lat, U, op->kappa, 0, a.g4.get(), a.r.get(), n, nitems, 0, nullptr, nullptr, nullptr, cfg);
  wilson_batched<float>(s, lat, U, op->kappa, 1, a.r.get(), a.g16a.get(), n, nitems, 0, nullptr, nullptr, nullptr,
                        cfg);
  DBuf<double2> ad((size_t)tot), d64((size_t)tot);
  widen_f64(s, tot, a.g16a.get(), ad.get());
  widen_f64(s, tot, a.g4.get(), d64.get());
  const int k = e->k;
  constexpr int kCols = 16, kRows = 64;
  DBuf<double> part((size_t)2 * kRows * kCols * tsk_multi_nblocks(n) + 64);
  DBuf<double2> cbuf(2 * (size_t)nitems * k);
  for (int c0 = 0; c0 < nitems; c0 += kCols) {
    const int nw = std::min(kCols, nitems - c0);
    for (int j0 = 0; j0 < k; j0 += kRows) {
      const int nv = std::min(kRows, k - j0);
      const int np = tsk_dots_multi(s, n, nv, e->Y.get() + (long)j0 * n, n, ad.get() + (long)c0 * n, n, nw, nullptr,
                                    part.get());
      for (int r = 0; r < nw; ++r)
        sum_partials(s, part.get() + (size_t)2 * r * nv * np, np, 2 * nv,
                     reinterpret_cast<double*>(cbuf.get() + (long)(c0 + r) * k + j0));
    }
  }
  double2* D = cbuf.get() + (long)nitems * k;
  proj_solve(s, k, nitems, e->Zr.get(), e->lamr.get(), cbuf.get(), D);
  hipLaunchKernelGGL(k_negate, dim3(64), dim3(256), 0, s, (long)nitems * k, D);
  for (int c0 = 0; c0 < nitems; c0 += kCols) {
    const int nw = std::min(kCols, nitems - c0);
    tsk_update_multi(s, n, k, e->Y.get(), n, D + (long)c0 * k, nw, nullptr, d64.get() + (long)c0 * n, n);
  }
  round_f32(s, tot, d64.get(), a.g4.get());
  DL_HIP(hipGetLastError());
}

double net_loss_grad(dl_net* net, dl_op* op, int nitems, const double2* B, const double2* X, bool grad) {
  hipStream_t s = net->ctx->stream;
  const Lattice& lat = op->lat;
  const long n = lat.nc;
  NetActs& a = net->acts;
  a.ensure(lat, nitems);
  const float2* U = op_links32_public(op);
  forward(net, op, nitems, B, a.y.get(), grad);
  // d = net(b) - x; r = M d; loss = mean ||r||^2 / ||b||^2
  hipLaunchKernelGGL(k_sub_f32_f64, dim3(kStreamBlocks, nitems), dim3(256), 0, s, a.y.get(), X, a.g4.get(), n);
  if (net->proj && net->proj->k > 0) project_error(net, op, nitems);
  wilson_batched<float>(s, lat, U, op->kappa, 0, a.g4.get(), a.r.get(), n, nitems, 0, nullptr, nullptr, nullptr,
                        wilson_cfg(op, DL_FP32, nitems));
  hipLaunchKernelGGL(k_norm2_items_f32, dim3(kStreamBlocks, nitems), dim3(kBlock), 0, s, a.r.get(), n, a.part.get());
  std::vector<double> hr((size_t)kStreamBlocks * nitems), hs(nitems), hb(nitems);
  DL_HIP(hipMemcpyAsync(hr.data(), a.part.get(), hr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  DL_HIP(hipMemcpyAsync(hs.data(), a.s.get(), nitems * sizeof(double), hipMemcpyDeviceToHost, s));
  DL_HIP(hipMemcpyAsync(hb.data(), a.bn2.get(), nitems * sizeof(double), hipMemcpyDeviceToHost, s));
  DL_HIP(hipStreamSynchronize(s));
  double L = 0.0;
  std::vector<float> gsc(nitems);
  for (int it = 0; it < nitems; ++it) {
    double rr = 0.0;
    for (int g = 0; g < kStreamBlocks; ++g) rr += hr[(size_t)it * kStreamBlocks + g];
    const double bn2 = hb[it];
    if (bn2 == 0.0) fail(DL_E_INVALID, "training pair with b = 0");
    L += rr / bn2 / nitems;
    // dL/dy = 2 M^dag r / (||b||^2 nitems) and y = s a3, so dL/da3 = s dL/dy
    gsc[it] = (float)(2.0 * hs[it] / bn2 / nitems);
  }
  if (!std::isfinite(L)) fail(DL_E_NONFINITE, "non-finite network loss");
  if (!grad) return L;
  DL_HIP(hipMemcpyAsync(a.gsc.get(), gsc.data(), nitems * sizeof(float), hipMemcpyHostToDevice, s));
  wilson_batched<float>(s, lat, U, op->kappa, 1, a.r.get(), a.g4.get(), n, nitems, 0, nullptr, nullptr, nullptr,
                        wilson_cfg(op, DL_FP32, nitems));
  hipLaunchKernelGGL(k_scale_items_f32, dim3(kStreamBlocks, nitems), dim3(256), 0, s, a.g4.get(), n,
                     (const float*)a.gsc.get());
  float2* W = net->W.get();
  float2* G = net->G.get();
  float2* Wt = net->Wt.get();
  const unsigned nl16 = (unsigned)((lat.V * 16 + 255) / 256);
  // layer 3 (16 -> 4)
  layer_wgrad(s, lat, U, a.a2.get(), a.g4.get(), 16, 4, nitems, a.part.get(), G + net_weight_offset(2));
  hipLaunchKernelGGL(k_ptc_adjoint_weights, dim3((9 * 64 + 255) / 256), dim3(256), 0, s, W + net_weight_offset(2),
                     Wt + net_weight_offset(2), 16, 4);
  launch_layer(s, lat, U, a.g4.get(), a.g16a.get(), nullptr, Wt + net_weight_offset(2), 4, 16, false, nitems,
               nullptr);
  hipLaunchKernelGGL(k_ptc_nonlin_bwd, dim3(nl16, nitems), dim3(256), 0, s, a.z2.get(), a.g16a.get(), 16,
                     (int)lat.V, act_len(lat, 16));
  // layer 2 (16 -> 16)
  layer_wgrad(s, lat, U, a.a1.get(), a.g16a.get(), 16, 16, nitems, a.part.get(), G + net_weight_offset(1));
  hipLaunchKernelGGL(k_ptc_adjoint_weights, dim3((9 * 256 + 255) / 256), dim3(256), 0, s, W + net_weight_offset(1),
                     Wt + net_weight_offset(1), 16, 16);
  launch_layer(s, lat, U, a.g16a.get(), a.g16b.get(), nullptr, Wt + net_weight_offset(1), 16, 16, false, nitems,
               nullptr);
  hipLaunchKernelGGL(k_ptc_nonlin_bwd, dim3(nl16, nitems), dim3(256), 0, s, a.z1.get(), a.g16b.get(), 16,
                     (int)lat.V, act_len(lat, 16));
  // layer 1 (4 -> 16): weight gradient only
  layer_wgrad(s, lat, U, a.a0.get(), a.g16b.get(), 4, 16, nitems, a.part.get(), G + net_weight_offset(0));
  DL_HIP(hipGetLastError());
  return L;
}

void net_reset_adam(dl_net* net) {
  // m and v hold 2 * nw floats each = nw / 2 double2 (nw is even)
  const long nw = net_num_weights();
  zero(net->ctx->stream, nw / 2, reinterpret_cast<double2*>(net->m.get()));
  zero(net->ctx->stream, nw / 2, reinterpret_cast<double2*>(net->v.get()));
  net->step = 0;
}

void net_adam_step(dl_net* net, float lr) {
  net->step += 1;
  const int n = 2 * net_num_weights();
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - std::pow(b1, (float)net->step), c2 = 1.f - std::pow(b2, (float)net->step);
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, net->ctx->stream,
                     reinterpret_cast<float*>(net->W.get()), reinterpret_cast<const float*>(net->G.get()),
                     net->m.get(), net->v.get(), n, lr, b1, b2, eps, c1, c2);
  DL_HIP(hipGetLastError());
}

}  // namespace dl
