// Per-contact warm-start network: packing, batch inference and training on gfx950.
//
//  - mlp_pack_kernel: FP32 parameters -> bfloat16 operand layouts (inference blob and the
//    training copies), every weight and bias rounded to bfloat16 once.
//  - mlp_infer_kernel: one wave per 64 feature rows, the same matrix-core chain the step
//    kernel runs for its contacts.
//  - mlp_grad_kernel: forward and backward of the mean squared error on 64-row chunks, four
//    waves per workgroup, operands staged in LDS, weight gradients held in matrix-core
//    accumulators across the workgroup's chunks; one partial gradient per workgroup.
//  - mlp_reduce_kernel: partials summed in a fixed order (deterministic), then
//  - mlp_adamw_kernel: decoupled weight decay Adam on the FP32 master parameters.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "../../include/jenga.h"
#include "jenga_device.h"
#include "mlp_device.h"

namespace jg {
namespace mlp {
namespace {

// training copies of the weights (bfloat16 bits), after the inference blob
constexpr int kTrW1t = 0;                       // [128][32]: W1^T with b1 in column 24
constexpr int kTrW2t = kTrW1t + 128 * 32;       // [128][128]: W2^T  (row = output)
constexpr int kTrW2n = kTrW2t + 128 * 128;      // [128][128]: W2    (row = input)
constexpr int kTrW3t = kTrW2n + 128 * 128;      // [16][128]: W3^T, rows 3..15 zero
constexpr int kTrHalfs = kTrW3t + 16 * 128;
constexpr int kTrBias = 132;                    // FP32: b2[128], b3[3], pad (bf16-rounded)
constexpr size_t kPackedBytes = (size_t)kPkUnits * 16 + (size_t)kTrHalfs * 2 + (size_t)kTrBias * 4;

__device__ inline float rbf(float f) { return __uint_as_float(bf16_bits(f) << 16); }

__device__ inline uint16_t w1aug(const float* P, int k, int o) {   // W1 with the bias as input 24
  const float v = k < kFeat ? P[kOffW1 + k * kHidden + o] : (k == kFeat ? P[kOffB1 + o] : 0.f);
  return (uint16_t)bf16_bits(v);
}

__global__ void mlp_pack_kernel(const float* __restrict__ P, uint4* __restrict__ blob) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint16_t* pk16 = reinterpret_cast<uint16_t*>(blob);
  float* pkf = reinterpret_cast<float*>(blob);
  // inference blob: one thread per 16-bit slot of the A-operand tiles
  if (tid < (kPkB2 - kPkW1) * 8) {
    const int unit = tid >> 3, j = tid & 7;
    uint16_t v;
    if (unit < kPkW2) {                              // W1 tiles
      const int m = unit >> 6, lane = unit & 63, g = lane >> 4, r = lane & 15;
      v = w1aug(P, 8 * g + j, 16 * m + r);
    } else if (unit < kPkW3) {                       // W2 tiles
      const int u = unit - kPkW2, lane = u & 63, kb = (u >> 6) & 3, mo = u >> 8, g = lane >> 4, r = lane & 15;
      v = (uint16_t)bf16_bits(P[kOffW2 + kappa(kb, g, j) * kHidden + 16 * mo + r]);
    } else {                                         // W3 tiles
      const int u = unit - kPkW3, lane = u & 63, kb = u >> 6, g = lane >> 4, r = lane & 15;
      v = r < kOut ? (uint16_t)bf16_bits(P[kOffW3 + kappa(kb, g, j) * kOut + r]) : (uint16_t)0;
    }
    pk16[tid] = v;
  }
  if (tid < kHidden) pkf[kPkB2 * 4 + tid] = rbf(P[kOffB2 + tid]);        // b2[16mo + 4g + i] in order
  if (tid < 4) pkf[kPkB3 * 4 + tid] = tid < kOut ? rbf(P[kOffB3 + tid]) : 0.f;
  if (tid < kFeat) {
    pkf[kPkMean * 4 + tid] = P[kOffMean + tid];
    pkf[kPkSd * 4 + tid] = P[kOffSd + tid];
  }
  // training copies
  uint16_t* tr = pk16 + kPkUnits * 8;
  if (tid < 128 * 32) { const int o = tid >> 5, k = tid & 31; tr[kTrW1t + tid] = w1aug(P, k, o); }
  if (tid < 128 * 128) {
    const int a = tid >> 7, b = tid & 127;
    tr[kTrW2t + tid] = (uint16_t)bf16_bits(P[kOffW2 + b * kHidden + a]);   // [out a][in b]
    tr[kTrW2n + tid] = (uint16_t)bf16_bits(P[kOffW2 + a * kHidden + b]);   // [in a][out b]
  }
  if (tid < 16 * 128) {
    const int o = tid >> 7, k = tid & 127;
    tr[kTrW3t + tid] = o < kOut ? (uint16_t)bf16_bits(P[kOffW3 + k * kOut + o]) : (uint16_t)0;
  }
  float* trb = reinterpret_cast<float*>(tr + kTrHalfs);
  if (tid < kTrBias) trb[tid] = tid < kHidden ? rbf(P[kOffB2 + tid]) : (tid < kHidden + kOut ? rbf(P[kOffB3 + tid - kHidden]) : 0.f);
}

__global__ void __launch_bounds__(64) mlp_infer_kernel(const uint4* __restrict__ pk, const float* __restrict__ feats,
                                                       int n, float* __restrict__ y) {
  __shared__ __align__(16) uint32_t xs[kChunk * kRowWords];
  const int lane = threadIdx.x;
  const int nchunks = (n + kChunk - 1) / kChunk;
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const int row = c * kChunk + lane;
    float f[kFeat];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) f[k] = row < n ? feats[(size_t)row * kFeat + k] : 0.f;
    stage_row(pk, f, xs + lane * kRowWords);
    __syncthreads();
    f32x4 out[4];
    infer_chunk(pk, xs, lane, out);
    if (lane < 16) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = c * kChunk + 16 * t + lane;
        if (r < n)
          for (int o = 0; o < kOut; ++o) y[(size_t)r * kOut + o] = out[t][o];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------------------------------
// training: forward + backward on 64-row chunks
// ------------------------------------------------------------------------------------------------
constexpr int kTrainThreads = 256;
// LDS row strides in 16-bit units (rows padded by 16 bytes against bank conflicts)
constexpr int kS128 = 136, kS64 = 72, kS32 = 40;
struct TrainLds {
  uint16_t X[64 * kS32];      // [p][k]  inputs (bias column 24)
  uint16_t Xt[32 * kS64];     // [k][p]
  uint16_t H1[64 * kS128];    // [p][h]
  uint16_t H1t[128 * kS64];   // [h][p]
  uint16_t H2[64 * kS128];
  uint16_t H2t[128 * kS64];
  uint16_t dZ2[64 * kS128];   // [p][h]
  uint16_t dZ2t[128 * kS64];  // [h][p]
  uint16_t dZ1t[128 * kS64];  // [h][p]
  uint16_t dYt[16 * kS64];    // [o][p], rows 3..15 zero
  float dY[64 * 4];           // [p][o]
  float T[64 * 4];            // targets
  float loss[4];
};

__device__ inline bf16x8 lds8(const uint16_t* base) { return as_bf16x8(*reinterpret_cast<const uint4*>(base)); }
__device__ inline bf16x8 glb8(const uint16_t* base) { return as_bf16x8(*reinterpret_cast<const uint4*>(base)); }

__global__ void __launch_bounds__(kTrainThreads, 1)
mlp_grad_kernel(const float* __restrict__ P, const uint4* __restrict__ pk, const float* __restrict__ feats,
                const float* __restrict__ targets, int n, float* __restrict__ partial) {
  extern __shared__ __align__(16) unsigned char smem[];
  TrainLds& S = *reinterpret_cast<TrainLds*>(smem);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, r = lane & 15;
  const uint16_t* tr = reinterpret_cast<const uint16_t*>(pk) + kPkUnits * 8;
  const float* trb = reinterpret_cast<const float*>(tr + kTrHalfs);
  const float inv_rows = 1.f / (3.f * (float)n);

  // persistent accumulators: dW1aug tiles (k-tile kt, h-tile 2w+hs), dW2 tiles (i-tile 2w+is,
  // h-tile ht), dW3 tiles (h-tile 2w+hs), db2 / db3 per lane
  f32x4 aW1[2][2], aW2[2][8], aW3[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    aW3[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 2; ++b) aW1[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 8; ++b) aW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  float db2[2] = {0.f, 0.f}, db3 = 0.f, lsum = 0.f;

  const int nchunks = (n + kChunk - 1) / kChunk;
  for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
    // ---- stage inputs and targets ----
    if (tid < kChunk) {
      const int row = c * kChunk + tid;
      uint32_t w[kRowWords];
      if (row < n) {
        float f[kFeat];
#pragma unroll
        for (int k = 0; k < kFeat; ++k) f[k] = feats[(size_t)row * kFeat + k];
        stage_row(pk, f, w);
      } else {
#pragma unroll
        for (int k = 0; k < kRowWords; ++k) w[k] = 0u;   // padding rows: no bias input either
      }
#pragma unroll
      for (int k = 0; k < kRowWords; ++k) {
        S.X[tid * kS32 + 2 * k] = (uint16_t)(w[k] & 0xffffu);
        S.X[tid * kS32 + 2 * k + 1] = (uint16_t)(w[k] >> 16);
        S.Xt[(2 * k) * kS64 + tid] = (uint16_t)(w[k] & 0xffffu);
        S.Xt[(2 * k + 1) * kS64 + tid] = (uint16_t)(w[k] >> 16);
      }
#pragma unroll
      for (int o = 0; o < 3; ++o) S.T[tid * 4 + o] = row < n ? targets[(size_t)row * 3 + o] : 0.f;
    }
    __syncthreads();

    // ---- forward layer 1: Z1[p][h] for h-tiles 2w, 2w+1 ----
    f32x4 z1[2][4], z2[2][4];
#pragma unroll
    for (int hs = 0; hs < 2; ++hs) {
      const int h0 = 16 * (2 * wave + hs);
      const bf16x8 b = glb8(tr + kTrW1t + (h0 + r) * 32 + 8 * g);
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) {
        const bf16x8 a = lds8(S.X + (16 * pt + r) * kS32 + 8 * g);
        z1[hs][pt] = mfma(a, b, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int p = 16 * pt + 4 * g + i, h = h0 + r;
          const uint16_t hb = (uint16_t)bf16_bits(gelu(z1[hs][pt][i]));
          S.H1[p * kS128 + h] = hb;
          S.H1t[h * kS64 + p] = hb;
        }
      }
    }
    __syncthreads();
    // ---- forward layer 2 ----
#pragma unroll
    for (int hs = 0; hs < 2; ++hs) {
      const int h0 = 16 * (2 * wave + hs);
      const float bias = trb[h0 + r];
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) z2[hs][pt] = f32x4{bias, bias, bias, bias};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 b = glb8(tr + kTrW2t + (h0 + r) * 128 + 32 * kb + 8 * g);
#pragma unroll
        for (int pt = 0; pt < 4; ++pt) {
          const bf16x8 a = lds8(S.H1 + (16 * pt + r) * kS128 + 32 * kb + 8 * g);
          z2[hs][pt] = mfma(a, b, z2[hs][pt]);
        }
      }
#pragma unroll
      for (int pt = 0; pt < 4; ++pt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int p = 16 * pt + 4 * g + i, h = h0 + r;
          const uint16_t hb = (uint16_t)bf16_bits(gelu(z2[hs][pt][i]));
          S.H2[p * kS128 + h] = hb;
          S.H2t[h * kS64 + p] = hb;
        }
    }
    __syncthreads();
    // ---- output layer and loss: wave w owns rows 16w..16w+15 ----
    {
      const float b3v = r < kOut ? trb[kHidden + r] : 0.f;
      f32x4 y = f32x4{b3v, b3v, b3v, b3v};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 a = lds8(S.H2 + (16 * wave + r) * kS128 + 32 * kb + 8 * g);
        const bf16x8 b = glb8(tr + kTrW3t + r * 128 + 32 * kb + 8 * g);
        y = mfma(a, b, y);
      }
      // lane (g, r) holds y[p = 16w + 4g + i][o = r]
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = 16 * wave + 4 * g + i;
        float d = 0.f;
        if (r < kOut && c * kChunk + p < n) {
          const float e = y[i] - S.T[p * 4 + r];
          lsum += e * e;
          d = 2.f * e * inv_rows;
        }
        if (r < kOut) S.dY[p * 4 + r] = d;
        S.dYt[r * kS64 + p] = (uint16_t)bf16_bits(d);
        db3 += d;
      }
    }
    __syncthreads();
    // ---- dZ2 = (dY W3^T) * gelu'(z2), same tiles as layer 2 ----
#pragma unroll
    for (int hs = 0; hs < 2; ++hs) {
      const int h = 16 * (2 * wave + hs) + r;
      const float w30 = rbf(P[kOffW3 + h * 3]), w31 = rbf(P[kOffW3 + h * 3 + 1]), w32 = rbf(P[kOffW3 + h * 3 + 2]);
#pragma unroll
      for (int pt = 0; pt < 4; ++pt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int p = 16 * pt + 4 * g + i;
          const float dh = S.dY[p * 4] * w30 + S.dY[p * 4 + 1] * w31 + S.dY[p * 4 + 2] * w32;
          const float dz = dh * gelu_grad(z2[hs][pt][i]);
          db2[hs] += dz;
          const uint16_t b = (uint16_t)bf16_bits(dz);
          S.dZ2[p * kS128 + h] = b;
          S.dZ2t[h * kS64 + p] = b;
        }
    }
    __syncthreads();
    // ---- dW3[h][o] += H2t[h][:] . dYt[o][:] ----
#pragma unroll
    for (int hs = 0; hs < 2; ++hs) {
      const int h0 = 16 * (2 * wave + hs);
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 a = lds8(S.H2t + (h0 + r) * kS64 + 32 * kb + 8 * g);
        const bf16x8 b = lds8(S.dYt + r * kS64 + 32 * kb + 8 * g);
        aW3[hs] = mfma(a, b, aW3[hs]);
      }
    }
    // ---- dZ1 = (dZ2 W2^T) * gelu'(z1), same tiles as layer 1 ----
#pragma unroll
    for (int is = 0; is < 2; ++is) {
      const int i0 = 16 * (2 * wave + is);
      f32x4 acc[4];
#pragma unroll
      for (int pt = 0; pt < 4; ++pt) acc[pt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const bf16x8 b = glb8(tr + kTrW2n + (i0 + r) * 128 + 32 * kb + 8 * g);
#pragma unroll
        for (int pt = 0; pt < 4; ++pt) {
          const bf16x8 a = lds8(S.dZ2 + (16 * pt + r) * kS128 + 32 * kb + 8 * g);
          acc[pt] = mfma(a, b, acc[pt]);
        }
      }
#pragma unroll
      for (int pt = 0; pt < 4; ++pt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int p = 16 * pt + 4 * g + i;
          S.dZ1t[(i0 + r) * kS64 + p] = (uint16_t)bf16_bits(acc[pt][i] * gelu_grad(z1[is][pt][i]));
        }
    }
    __syncthreads();
    // ---- dW2[i][h] += H1t[i][:] . dZ2t[h][:];  dW1aug[k][i] += Xt[k][:] . dZ1t[i][:] ----
#pragma unroll
    for (int is = 0; is < 2; ++is) {
      const int i0 = 16 * (2 * wave + is);
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 a = lds8(S.H1t + (i0 + r) * kS64 + 32 * kb + 8 * g);
#pragma unroll
        for (int ht = 0; ht < 8; ++ht) {
          const bf16x8 b = lds8(S.dZ2t + (16 * ht + r) * kS64 + 32 * kb + 8 * g);
          aW2[is][ht] = mfma(a, b, aW2[is][ht]);
        }
      }
    }
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const bf16x8 a = lds8(S.Xt + (16 * kt + r) * kS64 + 32 * kb + 8 * g);
#pragma unroll
        for (int hs = 0; hs < 2; ++hs) {
          const bf16x8 b = lds8(S.dZ1t + (16 * (2 * wave + hs) + r) * kS64 + 32 * kb + 8 * g);
          aW1[kt][hs] = mfma(a, b, aW1[kt][hs]);
        }
      }
    }
    __syncthreads();
  }

  // ---- write this workgroup's partial gradient ----
  float* out = partial + (size_t)blockIdx.x * (kTrainable + 1);
  // dW1aug tile (kt, h-tile 2w+hs): lane holds rows k = 16kt + 4g + i, column h = 16(2w+hs) + r
#pragma unroll
  for (int kt = 0; kt < 2; ++kt)
#pragma unroll
    for (int hs = 0; hs < 2; ++hs)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 16 * kt + 4 * g + i, h = 16 * (2 * wave + hs) + r;
        if (k < kFeat) out[kOffW1 + k * kHidden + h] = aW1[kt][hs][i];
        else if (k == kFeat) out[kOffB1 + h] = aW1[kt][hs][i];
      }
#pragma unroll
  for (int is = 0; is < 2; ++is)
#pragma unroll
    for (int ht = 0; ht < 8; ++ht)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int in = 16 * (2 * wave + is) + 4 * g + i, h = 16 * ht + r;
        out[kOffW2 + in * kHidden + h] = aW2[is][ht][i];
      }
#pragma unroll
  for (int hs = 0; hs < 2; ++hs)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * (2 * wave + hs) + 4 * g + i;
      if (r < kOut) out[kOffW3 + h * kOut + r] = aW3[hs][i];
    }
  // db2: lanes (g, r) of one wave hold partial sums of the same column; fold the 4 groups
#pragma unroll
  for (int hs = 0; hs < 2; ++hs) {
    float s = db2[hs];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (g == 0) out[kOffB2 + 16 * (2 * wave + hs) + r] = s;
  }
  {
    float s = db3;
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    // every wave saw its own rows: combine the four waves through LDS
    if (g == 0 && r < kOut) S.dY[wave * 4 + r] = s;
    float l = lsum;
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if (lane == 0) S.loss[wave] = l;
  }
  __syncthreads();
  if (tid < kOut) out[kOffB3 + tid] = S.dY[tid] + S.dY[4 + tid] + S.dY[8 + tid] + S.dY[12 + tid];
  if (tid == 0) out[kTrainable] = S.loss[0] + S.loss[1] + S.loss[2] + S.loss[3];
}

__global__ void mlp_reduce_kernel(const float* __restrict__ partial, int nparts, int n, float* __restrict__ grad,
                                  float* __restrict__ loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kTrainable) return;
  float s = 0.f;
  for (int k = 0; k < nparts; ++k) s += partial[(size_t)k * (kTrainable + 1) + i];
  if (i < kTrainable) grad[i] = s;
  else if (loss) *loss = s / (3.f * (float)n);
}

__global__ void mlp_adamw_kernel(float* __restrict__ P, const float* __restrict__ grad, float* __restrict__ m,
                                 float* __restrict__ v, float lr, float b1, float b2, float eps, float wd,
                                 float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kTrainable) return;
  const float gi = grad[i];
  float p = P[i] * (1.f - lr * wd);
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  P[i] = p;
}

int grad_blocks(int n) {
  const int nchunks = (n + kChunk - 1) / kChunk;
  return nchunks < 256 ? (nchunks > 0 ? nchunks : 1) : 256;
}

}  // namespace

size_t packed_bytes() { return kPackedBytes; }

hipError_t launch_pack(const float* params, void* packed, hipStream_t s) {
  constexpr int threads = (kPkB2 - kPkW1) * 8 > 128 * 128 ? (kPkB2 - kPkW1) * 8 : 128 * 128;
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((threads + 255) / 256), dim3(256), 0, s, params, (uint4*)packed);
  return hipGetLastError();
}

hipError_t launch_infer(const void* packed, const float* feats, int n, float* y, hipStream_t s) {
  const int nchunks = (n + kChunk - 1) / kChunk;
  if (nchunks == 0) return hipSuccess;
  const int grid = nchunks < 4096 ? nchunks : 4096;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3(grid), dim3(64), 0, s, (const uint4*)packed, feats, n, y);
  return hipGetLastError();
}

size_t grad_workspace_bytes(int n) { return (size_t)grad_blocks(n) * (kTrainable + 1) * sizeof(float); }

hipError_t launch_grad(const float* params, const void* packed, const float* feats, const float* targets, int n,
                       float* grad, float* loss, void* workspace, hipStream_t s) {
  // the kernel's dynamic-LDS limit, once per device (the current one)
  constexpr int kMaxDevices = 64;
  static std::mutex attr_mutex;
  static bool attr[kMaxDevices] = {};
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  {
    std::lock_guard<std::mutex> lock(attr_mutex);
    if (!attr[dev]) {
      hipError_t e = hipFuncSetAttribute((const void*)mlp_grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)sizeof(TrainLds));
      if (e != hipSuccess) return e;
      attr[dev] = true;
    }
  }
  const int blocks = grad_blocks(n);
  float* part = (float*)workspace;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(blocks), dim3(kTrainThreads), sizeof(TrainLds), s, params,
                     (const uint4*)packed, feats, targets, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kTrainable + 1 + 255) / 256), dim3(256), 0, s, part, blocks, n, grad,
                     loss);
  return hipGetLastError();
}

hipError_t launch_adamw(float* params, const float* grad, float* m, float* v, int step, float lr, float b1, float b2,
                        float eps, float wd, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp_adamw_kernel, dim3((kTrainable + 255) / 256), dim3(256), 0, s, params, grad, m, v, lr, b1,
                     b2, eps, wd, c1, c2);
  return hipGetLastError();
}

}  // namespace mlp
}  // namespace jg

// Scratch of jg_mlp_grad_noalloc: the per-workgroup partial gradients of one call, at most
// kGradScratchParts rows of JG_MLP_TRAINABLE + 1 floats (256 x 20100 x 4 B = 20.6 MB; the
// gradient launch never uses more workgroups).  Each device the library runs on holds its own
// copy until the process ends.  Every row a call reads is written earlier in the same call.
constexpr int kGradScratchParts = 256;
static __device__ __align__(256) float scratch[(size_t)kGradScratchParts * (JG_MLP_TRAINABLE + 1)];

// ------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------
namespace {
int32_t hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return JG_OK;
  return jg::set_error(JG_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// The device address of `scratch` on the current device, looked up on the first call there
// (the array's name is only a host-side stand-in; kernels get this address).
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
float* g_scratch_ptr[kScratchDevices] = {};

int32_t scratch_on_current_device(float** out) {
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return hip_status(e, "jg_mlp_grad_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices) return jg::set_error(JG_EDEVICE, "jg_mlp_grad_noalloc: device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)))
      return hip_status(e, "jg_mlp_grad_noalloc: hipGetSymbolAddress(scratch)");
    if (!p) return jg::set_error(JG_EDEVICE, "jg_mlp_grad_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = static_cast<float*>(p);
  }
  *out = g_scratch_ptr[dev];
  return JG_OK;
}
}  // namespace

extern "C" {

int32_t jg_mlp_packed_bytes(size_t* bytes) {
  if (!bytes) return jg::set_error(JG_EINVAL, "jg_mlp_packed_bytes: null pointer");
  *bytes = jg::mlp::packed_bytes();
  return JG_OK;
}

int32_t jg_mlp_pack(const float* params, void* packed, void* stream) {
  if (!params || !packed) return jg::set_error(JG_EINVAL, "jg_mlp_pack: null pointer");
  return hip_status(jg::mlp::launch_pack(params, packed, (hipStream_t)stream), "jg_mlp_pack");
}

int32_t jg_mlp_forward(const void* packed, const float* feats, int32_t n, float* y, void* stream) {
  if (n < 0) return jg::set_error(JG_EINVAL, "jg_mlp_forward: negative row count");
  if (n == 0) return JG_OK;
  if (!packed || !feats || !y) return jg::set_error(JG_EINVAL, "jg_mlp_forward: null pointer");
  return hip_status(jg::mlp::launch_infer(packed, feats, n, y, (hipStream_t)stream), "jg_mlp_forward");
}

int32_t jg_mlp_grad_workspace_bytes(int32_t n, size_t* bytes) {
  if (n < 0 || !bytes) return jg::set_error(JG_EINVAL, "jg_mlp_grad_workspace_bytes: bad argument");
  *bytes = jg::mlp::grad_workspace_bytes(n);
  return JG_OK;
}

int32_t jg_mlp_grad(const float* params, const void* packed, const float* feats, const float* targets, int32_t n,
                    float* grad, float* loss, void* workspace, size_t workspace_bytes, void* stream) {
  if (n <= 0) return jg::set_error(JG_EINVAL, "jg_mlp_grad: the batch must hold at least one row");
  if (!params || !packed || !feats || !targets || !grad || !workspace)
    return jg::set_error(JG_EINVAL, "jg_mlp_grad: null pointer");
  if (workspace_bytes < jg::mlp::grad_workspace_bytes(n))
    return jg::set_error(JG_EINVAL, "jg_mlp_grad: workspace smaller than jg_mlp_grad_workspace_bytes(n)");
  return hip_status(jg::mlp::launch_grad(params, packed, feats, targets, n, grad, loss, workspace, (hipStream_t)stream),
                    "jg_mlp_grad");
}

int32_t jg_mlp_grad_noalloc(const float* params, const void* packed, const float* feats, const float* targets,
                            int32_t n, float* grad, float* loss, void* stream) {
  if (n <= 0) return jg::set_error(JG_EINVAL, "jg_mlp_grad_noalloc: the batch must hold at least one row");
  if (!params || !packed || !feats || !targets || !grad)
    return jg::set_error(JG_EINVAL, "jg_mlp_grad_noalloc: null pointer");
  if (jg::mlp::grad_workspace_bytes(n) > sizeof(scratch))
    return jg::set_error(JG_ECAPACITY, "jg_mlp_grad_noalloc: the batch needs " +
                                       std::to_string(jg::mlp::grad_workspace_bytes(n)) +
                                       " bytes of partial sums, more than the static scratch holds (" +
                                       std::to_string(sizeof(scratch)) + ")");
  float* ws = nullptr;
  if (int32_t r = scratch_on_current_device(&ws)) return r;
  return hip_status(jg::mlp::launch_grad(params, packed, feats, targets, n, grad, loss, ws, (hipStream_t)stream),
                    "jg_mlp_grad_noalloc");
}

int32_t jg_mlp_adamw(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                     float beta2, float eps, float weight_decay, void* stream) {
  if (!params || !grad || !m || !v) return jg::set_error(JG_EINVAL, "jg_mlp_adamw: null pointer");
  if (step < 1) return jg::set_error(JG_EINVAL, "jg_mlp_adamw: step counts from 1");
  return hip_status(jg::mlp::launch_adamw(params, grad, m, v, step, lr, beta1, beta2, eps, weight_decay,
                                          (hipStream_t)stream),
                    "jg_mlp_adamw");
}

}  // extern "C"
