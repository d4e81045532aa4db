// Internal helpers shared by the libmlpf kernels (gfx950 / CDNA4 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlpf {

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// Matrix-product operand types. Storage of a bf16 value is its 16 raw bits.
struct F32 {
  using storage = float;
  static constexpr int kBytes = 4;
};
struct BF16 {
  using storage = __bf16;
  static constexpr int kBytes = 2;
};
// FP8 E4M3 (OCP: bias 7, max 448), one raw byte per value.
struct FP8 {
  using storage = uint8_t;
  static constexpr int kBytes = 1;
};
constexpr float kFp8Max = 448.0f;

// Rounds to FP8 E4M3 (nearest even) after clamping to +-448, so out-of-range values saturate.
__device__ __forceinline__ uint8_t to_fp8(float x) {
  x = fminf(fmaxf(x, -kFp8Max), kFp8Max);
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, x, 0, false) & 0xff);
}
// Four floats (already scaled) to four FP8 bytes in one dword.
__device__ __forceinline__ uint32_t pack_fp8x4(float a, float b, float c, float d) {
  a = fminf(fmaxf(a, -kFp8Max), kFp8Max);
  b = fminf(fmaxf(b, -kFp8Max), kFp8Max);
  c = fminf(fmaxf(c, -kFp8Max), kFp8Max);
  d = fminf(fmaxf(d, -kFp8Max), kFp8Max);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (uint32_t)w;
}

constexpr float kLog2e = 1.4426950408889634f;

// Fourth dword of a raw buffer resource on GFX9-family GPUs (gfx950): untyped 32-bit access,
// bounds-checked against num_records (loads past it return zero).
constexpr int kBufferWord3 = 0x00020000;

// The value of lane (this lane ^ o) for a constant o in 1..32: offsets below 16 move through DPP
// lane permutations on the VALU (quad_perm xor 1 and xor 2; xor 4 = half-row mirror then xor 3;
// xor 8 = row mirror then half-row mirror), the others through ds_bpermute. Same values as
// __shfl_xor, without its LDS round trip for the short offsets.
__device__ __forceinline__ float xor_lane(float v, int o) {
  const int x = __float_as_int(v);
  switch (o) {
    case 1: return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, true));
    case 2: return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, true));
    case 4: {
      const int m = __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, true);
      return __int_as_float(__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, true));
    }
    case 8: {
      const int m = __builtin_amdgcn_mov_dpp(x, 0x140, 0xF, 0xF, true);
      return __int_as_float(__builtin_amdgcn_mov_dpp(m, 0x141, 0xF, 0xF, true));
    }
    default: return __shfl_xor(v, o, 64);
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += xor_lane(v, o);
  return v;
}

// GELU(z) = z/2 (1 + erf(z / sqrt 2)), the exact (erf) form. erf is Abramowitz & Stegun's
// formula 7.1.26 (Handbook of Mathematical Functions, 1964): for x >= 0,
//   erf(x) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-x^2),  t = 1 / (1 + p x),
// with |error| <= 1.5e-7, odd-extended to x < 0. Branch-free: one reciprocal, one exp2, five FMAs,
// about half the issue slots of the library erff.
__device__ __forceinline__ float gelu_erf(float z) {
  const float x = z * 0.70710678118654752f;
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  float poly = fmaf(1.061405429f, t, -1.453152027f);
  poly = fmaf(poly, t, 1.421413741f);
  poly = fmaf(poly, t, -0.284496736f);
  poly = fmaf(poly, t, 0.254829592f);
  poly *= t;
  const float e = __builtin_amdgcn_exp2f(-(ax * ax) * 1.4426950408889634f);
  const float erf_abs = fmaf(-poly, e, 1.0f);
  return 0.5f * z * (1.0f + copysignf(erf_abs, x));
}

// GELU of the BF16 and FP8 paths, whose hidden activations are rounded to bf16 or E4M3 next:
// z * sigma(g(z)), sigma the logistic function and g(z) = z (c1 + c3 z^2 + c5 z^4) a
// least-maximum-error fit of the normal CDF made for this library (c1 = 1.59543567,
// c3 = 0.073596512, c5 = -6.31614093e-4; z is clamped to [-10, 10] inside g, where the fit still
// rises). In FP32 evaluation max |sigma(g(z)) - Phi(z)| = 1.9e-5 and the GELU error is at most
// 5.5e-5 (absolute) for |z| <= 1e6 (below -10 the result is z * 3.6e-12 rather than 0); in an
// FP64 forward pass it moves the model's outputs
// by at most 1.4e-4 of their norm. Below, the constants carry -log2(e) so that one exp2 gives
// exp(-g). Two transcendentals (exp2, reciprocal) and five other operations, against eleven for
// gelu_erf, which the FP32 path keeps.
__device__ __forceinline__ float gelu_fast(float z) {
  const float zc = fminf(fmaxf(z, -10.f), 10.f);
  const float z2 = zc * zc;
  float p = fmaf(z2, 0.00091122650f, -0.10617732f);
  p = fmaf(p, z2, -2.3017271f);
  const float e = __builtin_amdgcn_exp2f(zc * p);
  return z * __builtin_amdgcn_rcpf(1.0f + e);
}

// Rounds 4 floats to bf16 (round to nearest even) and packs them into 2 dwords.
__device__ __forceinline__ u32x2 pack_bf16x4(float a, float b, float c, float d) {
  bf16x4 v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)d};
  return __builtin_bit_cast(u32x2, v);
}

// acc + bf16(a) + bf16(b) + bf16(c) + bf16(d) (two v_dot2 with (1, 1); the products are exact),
// i.e. the sum of exactly the values pack_bf16x4(a, b, c, d) carries into a bf16 MFMA operand.
// The pairs are built from the floats: taking them out of an already packed u32x2 has been
// miscompiled (the second dot read the first pair's register).
__device__ __forceinline__ float add_bf16x4(float a, float b, float c, float d, float acc) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 one = {(__bf16)1.0f, (__bf16)1.0f};
  const bf16x2 ab = {(__bf16)a, (__bf16)b}, cd = {(__bf16)c, (__bf16)d};
  acc = __builtin_amdgcn_fdot2_f32_bf16(ab, one, acc, false);
  return __builtin_amdgcn_fdot2_f32_bf16(cd, one, acc, false);
}

// One 32x32 MFMA "k-group": each lane holds 16 bytes of A (row l%32) and 16 bytes of B
// (column l%32); lane half h = l/32 holds the h-th half of the group's k-values. The k order
// inside a group is the same for A and B, so any fixed permutation gives the same sum.
//   F32 : 4 x v_mfma_f32_32x32x2_f32  (group = 8 k-values: half h holds k = 4h .. 4h+3)
//   BF16: 1 x v_mfma_f32_32x32x16_bf16 (group = 16 k-values: half h holds k = 8h .. 8h+7)
// (FP8 operands take 64-value groups, mma_fp8_k64 below.)
template <class T>
__device__ __forceinline__ void mma_kg(const u32x4& a, const u32x4& b, f32x16& c);

template <>
__device__ __forceinline__ void mma_kg<F32>(const u32x4& a, const u32x4& b, f32x16& c) {
#pragma unroll
  for (int t = 0; t < 4; ++t)
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[t]), __uint_as_float(b[t]), c, 0, 0, 0);
}

template <>
__device__ __forceinline__ void mma_kg<BF16>(const u32x4& a, const u32x4& b, f32x16& c) {
  c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                              __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// FP8 E4M3 k-group of 64 values on gfx950's 32x32x64 F8F6F4 MFMA (twice the FP8 rate of the
// 32x32x16 FP8 instruction): each lane holds 32 bytes of A (row l%32) and of B (column l%32), lane
// half h the h-th 32 k-values of the group (a0 and b0 its first 16 bytes, a1 and b1 the next 16).
// The unscaled form: format fields 0 (E4M3 for both operands), block scales 0.
__device__ __forceinline__ void mma_fp8_k64(const u32x4& a0, const u32x4& a1, const u32x4& b0,
                                            const u32x4& b1, f32x16& c) {
  typedef int i32x8 __attribute__((ext_vector_type(8)));
  const i32x8 a = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
  const i32x8 b = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
  c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

// Converts E = 16 / sizeof(T) floats to one 16-byte chunk of T.
template <class T>
__device__ __forceinline__ u32x4 to_chunk(const float* v);

template <>
__device__ __forceinline__ u32x4 to_chunk<F32>(const float* v) {
  return u32x4{__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
               __float_as_uint(v[3])};
}

template <>
__device__ __forceinline__ u32x4 to_chunk<BF16>(const float* v) {
  u32x2 lo = pack_bf16x4(v[0], v[1], v[2], v[3]);
  u32x2 hi = pack_bf16x4(v[4], v[5], v[6], v[7]);
  return u32x4{lo[0], lo[1], hi[0], hi[1]};
}

// Raises *dst to v (v >= 0) with an integer atomic max on the float bits (order-independent).
__device__ __forceinline__ void atomic_max_nonneg(float* dst, float v) {
  atomicMax((int*)dst, __float_as_int(v));
}

// LayerNorm arithmetic (biased variance, Sec. 5.3), with floating-point contraction switched off so
// that the LayerNorm kernel and the epilogues that fuse a LayerNorm produce the same bits.
__device__ __forceinline__ float ln_sum4(float a, float b, float c, float d) {
#pragma clang fp contract(off)
  return (a + b) + (c + d);
}
__device__ __forceinline__ float ln_sq4(float a, float b, float c, float d, float mu) {
#pragma clang fp contract(off)
  const float x = a - mu, y = b - mu, z = c - mu, w = d - mu;
  return (x * x + y * y) + (z * z + w * w);
}
__device__ __forceinline__ float ln_mean(float sum, int d) { return sum / (float)d; }
__device__ __forceinline__ float ln_rstd(float sumsq, int d, float eps) {
#pragma clang fp contract(off)
  return 1.0f / sqrtf(sumsq / (float)d + eps);
}
__device__ __forceinline__ float ln_out(float v, float mu, float rs, float g, float b) {
#pragma clang fp contract(off)
  return __builtin_fmaf((v - mu) * rs, g, b);
}
__device__ __forceinline__ float add_nc(float a, float b) {
#pragma clang fp contract(off)
  return a + b;
}

// LayerNorm of a row of D = 8 CPR bf16 values held by CPR consecutive lanes (lane-aligned groups),
// each with 8 consecutive values x[0..7] (gamma g0, g1 and beta b0, b1 of those 8 columns); returns
// the 8 outputs as bf16.
// The sums follow the LayerNorm kernel's tree (its lane l holds values 4l .. 4l+3, so this lane's
// halves are its lanes 2j and 2j+1; zero lanes beyond D add exactly nothing), so the result is that
// kernel's bit for bit. Every lane of the group must call it (shuffles).
template <int CPR>
__device__ __forceinline__ u32x4 ln_row_chunk8(const float* x, const f32x4& g0, const f32x4& g1,
                                               const f32x4& b0, const f32x4& b1, float eps) {
  constexpr int D = 8 * CPR;
  float se = add_nc(0.f, ln_sum4(x[0], x[1], x[2], x[3])), so = add_nc(0.f, ln_sum4(x[4], x[5], x[6], x[7]));
#pragma unroll
  for (int off = CPR / 2; off >= 1; off >>= 1) {
    se = add_nc(se, xor_lane(se, off));
    so = add_nc(so, xor_lane(so, off));
  }
  const float mu = ln_mean(add_nc(se, so), D);
  float qe = add_nc(0.f, ln_sq4(x[0], x[1], x[2], x[3], mu)), qo = add_nc(0.f, ln_sq4(x[4], x[5], x[6], x[7], mu));
#pragma unroll
  for (int off = CPR / 2; off >= 1; off >>= 1) {
    qe = add_nc(qe, xor_lane(qe, off));
    qo = add_nc(qo, xor_lane(qo, off));
  }
  const float rs = ln_rstd(add_nc(qe, qo), D, eps);
  const u32x2 lo = pack_bf16x4(ln_out(x[0], mu, rs, g0[0], b0[0]), ln_out(x[1], mu, rs, g0[1], b0[1]),
                               ln_out(x[2], mu, rs, g0[2], b0[2]), ln_out(x[3], mu, rs, g0[3], b0[3]));
  const u32x2 hi = pack_bf16x4(ln_out(x[4], mu, rs, g1[0], b1[0]), ln_out(x[5], mu, rs, g1[1], b1[1]),
                               ln_out(x[6], mu, rs, g1[2], b1[2]), ln_out(x[7], mu, rs, g1[3], b1[3]));
  return u32x4{lo[0], lo[1], hi[0], hi[1]};
}

// The 8 values of a 16-byte chunk of bf16.
__device__ __forceinline__ void unpack_bf16x8(const u32x4& w, float* x) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    x[2 * e] = __uint_as_float(w[e] << 16);
    x[2 * e + 1] = __uint_as_float(w[e] & 0xffff0000u);
  }
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, xor_lane(v, o));
  return v;
}

// Workgroups of a launch are dealt round-robin to the 8 XCDs (each with its own L2). This maps
// the hardware order to a logical order in which consecutive logical ids share an XCD, so tiles
// that reuse the same operand rows sit behind the same L2. It is a bijection for any grid size.
__device__ __forceinline__ int xcd_remap(int b, int g) {
  const int q = g / 8, r = g % 8;
  const int xcd = b % 8, local = b / 8;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

}  // namespace mlpf
