// Per-contact warm-start network on gfx950 matrix cores (device side).
//
// Network: 24 features, z-scored, -> Linear(24,128) -> GELU -> Linear(128,128) -> GELU
// -> Linear(128,3).  Operands are bfloat16, accumulation FP32 (v_mfma_f32_16x16x32_bf16).
//
// Inference works on the transposed problem: for a tile of 16 contacts, H1^T = W1^T X^T,
// H2^T = W2^T H1^T, Y^T = W3^T H2^T, so the contacts are the MFMA's N dimension and the
// weights are its A operand.  A 16x16 result tile leaves lane l holding rows 4*(l/16)+i
// (i = 0..3) of column l%16; that is already the B-operand shape of the next product if
// the next weight matrix's K index is permuted to match (see kappa below), so activations
// never leave registers between layers.
//
// Packed weights (written by the pack kernel, read with one 16-byte load per lane):
//   w1[m][lane]      m = 0..7   rows 16m + lane%16 of W1^T; K slots: features 0..23,
//                               slot 24 holds b1 (the staged input carries a 1 there)
//   w2[mo][kb][lane]            rows 16mo + lane%16 of W2^T, K block kb in kappa order
//   w3[kb][lane]                rows 0..2 of W3^T (rows 3..15 zero), K block kb in kappa order
//   b2[mo][g]  float4           b2[16mo + 4g + i], the accumulator rows lane group g holds
//   b3[4]                       b3[0..2], 0
//   mean[24], sd[24]            feature normalisation
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jg {
namespace mlp {

constexpr int kFeat = 24;
constexpr int kHidden = 128;
constexpr int kOut = 3;
constexpr int kChunk = 64;            // contacts per inference chunk (4 MFMA column tiles)
constexpr int kRowWords = 16;         // staged input row: 32 bf16 = 16 words
// parameter vector (FP32 master copy): W1[24][128], b1, W2[128][128], b2, W3[128][3], b3, mean, sd
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kFeat * kHidden;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden * kOut;
constexpr int kOffMean = kOffB3 + kOut;
constexpr int kOffSd = kOffMean + kFeat;
constexpr int kParams = kOffSd + kFeat;       // 20147
constexpr int kTrainable = kOffMean;          // 20099
// packed inference blob, in 16-byte units
constexpr int kPkW1 = 0;
constexpr int kPkW2 = kPkW1 + 8 * 64;
constexpr int kPkW3 = kPkW2 + 8 * 4 * 64;
constexpr int kPkB2 = kPkW3 + 4 * 64;
constexpr int kPkB3 = kPkB2 + 8 * 4;
constexpr int kPkMean = kPkB3 + 1;
constexpr int kPkSd = kPkMean + 6;
constexpr int kPkUnits = kPkSd + 6;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// hidden index held by K slot (g, j) of K block kb, for an input that is the previous
// layer's result tiles 2kb (j < 4) and 2kb + 1 (j >= 4)
__host__ __device__ constexpr int kappa(int kb, int g, int j) { return 32 * kb + 16 * (j >> 2) + 4 * g + (j & 3); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// round to nearest even bfloat16, returned as the raw 16 bits: the conversion instruction of
// gfx950 (v_cvt_pk_bf16_f32), one for two values in pack2
__device__ inline uint32_t bf16_bits(float f) { return (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline uint32_t pack2(float lo, float hi) {
  const bf16x2 v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}

// Phi(-s) = erfc(s / sqrt 2) / 2 for s >= 0, with erfc from Abramowitz and Stegun 7.1.26
// (|error| <= 1.5e-7 on erf): erfc(a) = t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^{-a^2},
// t = 1 / (1 + p a).  The halving is folded into the coefficients and 1 / sqrt 2 into p and the
// exponent; e returns e^{-s^2 / 2}.  GELU and its derivative share it.
__device__ inline float phi_tail(float s, float& e) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, s, 1.f));
  float poly = fmaf(t, 0.5f * 1.061405429f, 0.5f * -1.453152027f);
  poly = fmaf(t, poly, 0.5f * 1.421413741f);
  poly = fmaf(t, poly, 0.5f * -0.284496736f);
  poly = fmaf(t, poly, 0.5f * 0.254829592f);
  e = __builtin_amdgcn_exp2f((-0.72134752044448170f * s) * s);   // 2^{-s^2 log2(e) / 2}
  return (poly * t) * e;
}

// GELU x Phi(x), written as max(x, 0) - |x| Phi(-|x|) (the two agree for either sign of x)
__device__ inline float gelu(float x) {
  const float s = fabsf(x);
  float e;
  const float q = phi_tail(s, e);
  return fmaf(-s, q, fmaxf(x, 0.f));
}

// dGELU/dx = Phi(x) + x phi(x), phi(x) = e^{-x^2 / 2} / sqrt(2 pi)
__device__ inline float gelu_grad(float x) {
  float e;
  const float q = phi_tail(fabsf(x), e);
  const float phi = x >= 0.f ? 1.f - q : q;
  return fmaf(x * 0.3989422804014327f, e, phi);
}

__device__ inline bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Normalised, rounded input row of one contact: 32 bf16 (features, 1 for the bias, zeros).
__device__ inline void stage_row(const uint4* pk, const float f[kFeat], uint32_t* row) {
  const float* mean = reinterpret_cast<const float*>(pk + kPkMean);
  const float* sd = reinterpret_cast<const float*>(pk + kPkSd);
#pragma unroll
  for (int k = 0; k < kFeat; k += 2) row[k >> 1] = pack2((f[k] - mean[k]) / sd[k], (f[k + 1] - mean[k + 1]) / sd[k + 1]);
  row[12] = pack2(1.f, 0.f);
#pragma unroll
  for (int k = 13; k < kRowWords; ++k) row[k] = 0u;
}

// Network outputs for 64 staged rows (xs: 64 rows x 16 words in LDS).  On return, lanes 0..15
// hold in y[t][0..2] the outputs of row 16t + lane; other lanes hold padding.
__device__ inline void infer_chunk(const uint4* __restrict__ pk, const uint32_t* xs, int lane, f32x4 y[4]) {
  const int g = lane >> 4, r = lane & 15;
  bf16x8 xb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const uint4 u = *reinterpret_cast<const uint4*>(xs + (16 * t + r) * kRowWords + 4 * g);
    xb[t] = as_bf16x8(u);
  }
  uint32_t h1[4][4][4];   // [kb][t][word]: K block kb of layer 2's B operand, column tile t
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const bf16x8 a = as_bf16x8(pk[kPkW1 + m * 64 + lane]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma(a, xb[t], acc);
      h1[m >> 1][t][2 * (m & 1)] = pack2(gelu(acc[0]), gelu(acc[1]));
      h1[m >> 1][t][2 * (m & 1) + 1] = pack2(gelu(acc[2]), gelu(acc[3]));
    }
  }
  const float* b3 = reinterpret_cast<const float*>(pk + kPkB3);
  const f32x4 y0 = g == 0 ? f32x4{b3[0], b3[1], b3[2], 0.f} : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 4; ++t) y[t] = y0;
  uint32_t h2[4][4];      // [t][word]: current K block of layer 3's B operand
#pragma unroll
  for (int mo = 0; mo < 8; ++mo) {
    const float4 bb = reinterpret_cast<const float4*>(pk + kPkB2)[mo * 4 + g];
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f32x4{bb.x, bb.y, bb.z, bb.w};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const bf16x8 a = as_bf16x8(pk[kPkW2 + (mo * 4 + kb) * 64 + lane]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint4 u = {h1[kb][t][0], h1[kb][t][1], h1[kb][t][2], h1[kb][t][3]};
        acc[t] = mfma(a, as_bf16x8(u), acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      h2[t][2 * (mo & 1)] = pack2(gelu(acc[t][0]), gelu(acc[t][1]));
      h2[t][2 * (mo & 1) + 1] = pack2(gelu(acc[t][2]), gelu(acc[t][3]));
    }
    if (mo & 1) {
      const bf16x8 a = as_bf16x8(pk[kPkW3 + (mo >> 1) * 64 + lane]);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint4 u = {h2[t][0], h2[t][1], h2[t][2], h2[t][3]};
        y[t] = mfma(a, as_bf16x8(u), y[t]);
      }
    }
  }
}

}  // namespace mlp
}  // namespace jg
