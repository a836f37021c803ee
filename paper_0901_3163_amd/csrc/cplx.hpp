// Complex arithmetic on double2 / float2 and wavefront reductions for gfx950.
#pragma once

#include <hip/hip_runtime.h>

namespace dl {

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_scale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i * a
__device__ __forceinline__ double2 c_i(double2 a) { return make_double2(-a.y, a.x); }
// a * b
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// acc + a * b
__device__ __forceinline__ double2 c_fma(double2 a, double2 b, double2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a) * b
__device__ __forceinline__ double2 c_fmac(double2 a, double2 b, double2 acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}
// acc + s * a (real s)
__device__ __forceinline__ double2 c_axpy(double s, double2 a, double2 acc) {
  return make_double2(fma(s, a.x, acc.x), fma(s, a.y, acc.y));
}

// float2 versions (FP32 storage and arithmetic)
__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 c_i(float2 a) { return make_float2(-a.y, a.x); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 c_fma(float2 a, float2 b, float2 acc) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ float2 c_fmac(float2 a, float2 b, float2 acc) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(-a.y, b.x, acc.y);
  return acc;
}
__device__ __forceinline__ float2 c_axpy(float s, float2 a, float2 acc) {
  return make_float2(fmaf(s, a.x, acc.x), fmaf(s, a.y, acc.y));
}

// Storage loads and stores: FP32/FP64 as is, BF16 widened to / rounded from FP32.
__device__ __forceinline__ float2 sld(const float2* p) { return *p; }
__device__ __forceinline__ double2 sld(const double2* p) { return *p; }
__device__ __forceinline__ float2 sld(const bf2* p) {
  const bf2 b = *p;
  return make_float2(__uint_as_float((unsigned)b.x << 16), __uint_as_float((unsigned)b.y << 16));
}
__device__ __forceinline__ float2 sldv(float2 v) { return v; }
__device__ __forceinline__ double2 sldv(double2 v) { return v; }
__device__ __forceinline__ float2 sldv(bf2 b) {
  return make_float2(__uint_as_float((unsigned)b.x << 16), __uint_as_float((unsigned)b.y << 16));
}
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ void sst(float2* p, float2 v) { *p = v; }
__device__ __forceinline__ void sst(double2* p, double2 v) { *p = v; }
// one v_cvt_pk_bf16_f32 (round to nearest even, as f2bf for every finite value)
typedef float f32x2_st __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_st __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void sst(bf2* p, float2 v) {
  const f32x2_st f = {v.x, v.y};
  *reinterpret_cast<unsigned*>(p) = __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2_st));
}

// Four consecutive storage elements (16 B of BF16, 32 B of FP32; the address a multiple of
// four elements) widened to / rounded from FP32.
__device__ __forceinline__ void sld4(const float2* p, float2* o) {
  const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
  o[0] = make_float2(a.x, a.y);
  o[1] = make_float2(a.z, a.w);
  o[2] = make_float2(b.x, b.y);
  o[3] = make_float2(b.z, b.w);
}
__device__ __forceinline__ float2 bf_word(unsigned w) {
  return make_float2(__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u));
}
__device__ __forceinline__ void sld4(const bf2* p, float2* o) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  o[0] = bf_word(u.x);
  o[1] = bf_word(u.y);
  o[2] = bf_word(u.z);
  o[3] = bf_word(u.w);
}
__device__ __forceinline__ void sst4(float2* p, const float2* v) {
  reinterpret_cast<float4*>(p)[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
  reinterpret_cast<float4*>(p)[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
}
__device__ __forceinline__ unsigned bf_pack(float2 v) {
  const f32x2_st f = {v.x, v.y};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f, bf16x2_st));
}
__device__ __forceinline__ void sst4(bf2* p, const float2* v) {
  *reinterpret_cast<uint4*>(p) = make_uint4(bf_pack(v[0]), bf_pack(v[1]), bf_pack(v[2]), bf_pack(v[3]));
}

template <class R> struct CT;
template <> struct CT<double> {
  using type = double2;
  __device__ static __forceinline__ double2 make(double x, double y) { return make_double2(x, y); }
};
template <> struct CT<float> {
  using type = float2;
  __device__ static __forceinline__ float2 make(float x, float y) { return make_float2(x, y); }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a block of kBlock threads; result valid in thread 0.  Fixed order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* lds /* NT/64 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += lds[w];
  }
  __syncthreads();
  return r;
}

// Map the hardware block index to a logical block so that each of the 8 XCDs
// (blocks are dealt round-robin to XCDs) works on one contiguous range of the
// lattice: neighbouring tiles then share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

}  // namespace dl
