// HIP kernels (gfx950) of the learned SGS closure: features, BF16-MFMA MLP forward and
// backward, split-K weight gradients, Adam, and inference over a field with the gradient
// model as fallback outside the training envelope.
//
// Network 14 -> 64 -> 64 -> 64 -> 6 with GELU (tanh form) after the hidden layers.
// Every product runs transposed, Z^T = W A^T, so a 16x16 MFMA tile holds 16 output
// features of 16 points: lane l = 16 g + p owns features 4 g + i (i = 0..3) of point p.
// That is exactly the B-operand layout of v_mfma_f32_16x16x16_bf16 (K slots 4 g + j), and
// for v_mfma_f32_16x16x32_bf16 two such tiles are concatenated; the matching input-feature
// permutation is folded into how the weights are packed, so no lane shuffles are needed
// between layers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kcf_mlp_internal.h"

namespace kcf {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace {

constexpr float kGeluC = 0.7978845608028654f;  // sqrt(2/pi)
constexpr float kGeluA = 0.044715f;

__device__ __forceinline__ __bf16 to_bf16(float f) { return static_cast<__bf16>(f); }

// exp(-u) for u = 2 c (x + a x^3) as 2^(x (k0 + k1 x^2)), k0 = -2 c log2(e), k1 = a k0:
// one multiply less than forming u first
constexpr float kGeluK0 = (float)(-2.0 * 0.7978845608028654 * 1.4426950408889634);
constexpr float kGeluK1 = (float)(-2.0 * 0.7978845608028654 * 1.4426950408889634 * 0.044715);

__device__ __forceinline__ float gelu_exp(float x) {
  return __builtin_amdgcn_exp2f(x * fmaf(kGeluK1, x * x, kGeluK0));
}

// x * sigmoid(u): the tanh form 0.5 x (1 + tanh(c (x + a x^3))).
__device__ __forceinline__ float gelu(float x) {
  return x * __builtin_amdgcn_rcpf(1.f + gelu_exp(x));
}

__device__ __forceinline__ float gelu_grad(float x) {
  const float s = __builtin_amdgcn_rcpf(1.f + gelu_exp(x));
  const float du = 2.f * kGeluC * fmaf(3.f * kGeluA, x * x, 1.f);
  return fmaf(x * s * (1.f - s), du, s);
}

// Input feature held in K slot j of lane group g for K step s of a 64-wide layer input.
__host__ __device__ __forceinline__ int perm64(int s, int g, int j) {
  return 16 * (2 * s + (j >> 2)) + 4 * g + (j & 3);
}

__device__ __forceinline__ floatx4 mfma16(short4v a, short4v b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma32(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ short4v pack4(float a, float b, float c, float d) {
  short4v r;
  r[0] = __builtin_bit_cast(short, to_bf16(a));
  r[1] = __builtin_bit_cast(short, to_bf16(b));
  r[2] = __builtin_bit_cast(short, to_bf16(c));
  r[3] = __builtin_bit_cast(short, to_bf16(d));
  return r;
}

__device__ __forceinline__ bf16x8 pack8(const floatx4& lo, const floatx4& hi) {
  bf16x8 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i] = to_bf16(lo[i]);
    r[4 + i] = to_bf16(hi[i]);
  }
  return r;
}

// ---------------------------------------------------------------- operand packing
// One thread per packed bf16 entry (kPackTotal).
__global__ void k_pack(const float* __restrict__ P, __bf16* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kPackTotal) return;
  float v = 0.f;
  if (e < kPF1) {  // W1, 16x16x16: [mt][lane][j]
    const int j = e & 3, L = (e >> 2) & 63, mt = e >> 8;
    const int g = L >> 4, r = L & 15;
    const int o = 16 * mt + r, i = 4 * g + j;
    v = (i < 14) ? P[kOffW1 + o * 14 + i] : 0.f;
  } else if (e < kPF3) {  // W2, W3, 16x16x32: [mt][s][lane][j]
    const int base = e < kPF2 ? kPF1 : kPF2;
    const int off = e < kPF2 ? kOffW2 : kOffW3;
    const int q = e - base;
    const int j = q & 7, L = (q >> 3) & 63, s = (q >> 9) & 1, mt = q >> 10;
    const int g = L >> 4, r = L & 15;
    v = P[off + (16 * mt + r) * 64 + perm64(s, g, j)];
  } else if (e < kPB3) {  // W4, 16x16x32: [s][lane][j], 6 real output rows
    const int q = e - kPF3;
    const int j = q & 7, L = (q >> 3) & 63, s = q >> 9;
    const int g = L >> 4, r = L & 15;
    v = (r < 6) ? P[kOffW4 + r * 64 + perm64(s, g, j)] : 0.f;
  } else if (e < kPB2) {  // W4^T, 16x16x16: [mt][lane][j]: rows = inputs, K = outputs
    const int q = e - kPB3;
    const int j = q & 3, L = (q >> 2) & 63, mt = q >> 8;
    const int g = L >> 4, r = L & 15;
    const int o = 4 * g + j;
    v = (o < 6) ? P[kOffW4 + o * 64 + 16 * mt + r] : 0.f;
  } else {  // W3^T then W2^T, 16x16x32: [mt][s][lane][j]
    const int base = e < kPB1 ? kPB2 : kPB1;
    const int off = e < kPB1 ? kOffW3 : kOffW2;
    const int q = e - base;
    const int j = q & 7, L = (q >> 3) & 63, s = (q >> 9) & 1, mt = q >> 10;
    const int g = L >> 4, r = L & 15;
    v = P[off + perm64(s, g, j) * 64 + 16 * mt + r];
  }
  out[e] = to_bf16(v);
}

// Copies packed operands and biases into LDS.
__device__ __forceinline__ void stage_params(const MlpArgs& M, __bf16* sW, float* sB, int n_pack) {
  const uint4* src = reinterpret_cast<const uint4*>(M.packed);
  uint4* dst = reinterpret_cast<uint4*>(sW);
  for (int i = threadIdx.x; i < n_pack / 8; i += blockDim.x) dst[i] = src[i];
  for (int i = threadIdx.x; i < 64; i += blockDim.x) {
    sB[i] = M.params[kOffB1 + i];
    sB[64 + i] = M.params[kOffB2 + i];
    sB[128 + i] = M.params[kOffB3 + i];
  }
  if (threadIdx.x < 16) sB[192 + threadIdx.x] = threadIdx.x < 6 ? M.params[kOffB4 + threadIdx.x] : 0.f;
}

// Forward pass of one 16-point tile. x: the lane's four standardised inputs (features
// 4g..4g+3). Keeps pre-activations z1..z3 (FP32) and the BF16 operands a1..a3.
struct Fwd {
  floatx4 z[3][4];   // pre-activations of hidden layers (tile t, rows 4g+i)
  bf16x8 a[3][2];    // BF16 activations as K-step operands of the next layer
  floatx4 y;         // network output rows 4g+i (rows < 6 valid)
};

__device__ __forceinline__ void forward(const __bf16* sW, const float* sB, short4v x, Fwd& F) {
  const int lane = __lane_id();
  const int g = lane >> 4;
  // layer 1: 16x16x16, 4 output tiles
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    floatx4 c;
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = sB[16 * mt + 4 * g + i];
    const short4v w = *reinterpret_cast<const short4v*>(sW + (mt * 64 + lane) * 4);
    F.z[0][mt] = mfma16(w, x, c);
  }
  // layers 2, 3: 16x16x32 over two K steps
#pragma unroll
  for (int l = 1; l <= 2; ++l) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      floatx4 lo, hi;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        lo[i] = gelu(F.z[l - 1][2 * s][i]);
        hi[i] = gelu(F.z[l - 1][2 * s + 1][i]);
      }
      F.a[l - 1][s] = pack8(lo, hi);
    }
    const int base = (l == 1) ? kPF1 : kPF2;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      floatx4 c;
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = sB[64 * l + 16 * mt + 4 * g + i];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 w = *reinterpret_cast<const bf16x8*>(sW + base + ((mt * 2 + s) * 64 + lane) * 8);
        c = mfma32(w, F.a[l - 1][s], c);
      }
      F.z[l][mt] = c;
    }
  }
  // layer 4
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    floatx4 lo, hi;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      lo[i] = gelu(F.z[2][2 * s][i]);
      hi[i] = gelu(F.z[2][2 * s + 1][i]);
    }
    F.a[2][s] = pack8(lo, hi);
  }
  floatx4 c;
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] = sB[192 + 4 * g + i];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bf16x8 w = *reinterpret_cast<const bf16x8*>(sW + kPF3 + (s * 64 + lane) * 8);
    c = mfma32(w, F.a[2][s], c);
  }
  F.y = c;
}

// Forward pass of NT 16-point tiles at once (inference): every weight operand is read from
// LDS once and applied to the NT tiles, which also gives the matrix cores NT independent
// accumulation chains. Per tile the operations and their order are those of forward().
template <int NT>
__device__ __forceinline__ void forward_tiles(const __bf16* sW, const float* sB,
                                              const short4v (&x)[NT], floatx4 (&y)[NT]) {
  const int lane = __lane_id();
  const int g = lane >> 4;
  floatx4 z[NT][4];
  bf16x8 a[NT][2];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    floatx4 c;
#pragma unroll
    for (int i = 0; i < 4; ++i) c[i] = sB[16 * mt + 4 * g + i];
    const short4v w = *reinterpret_cast<const short4v*>(sW + (mt * 64 + lane) * 4);
#pragma unroll
    for (int t = 0; t < NT; ++t) z[t][mt] = mfma16(w, x[t], c);
  }
#pragma unroll
  for (int l = 1; l <= 3; ++l) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        floatx4 lo, hi;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          lo[i] = gelu(z[t][2 * s][i]);
          hi[i] = gelu(z[t][2 * s + 1][i]);
        }
        a[t][s] = pack8(lo, hi);
      }
    }
    if (l == 3) break;
    const int base = (l == 1) ? kPF1 : kPF2;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      floatx4 c;
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] = sB[64 * l + 16 * mt + 4 * g + i];
      const bf16x8 w0 = *reinterpret_cast<const bf16x8*>(sW + base + ((mt * 2) * 64 + lane) * 8);
      const bf16x8 w1 = *reinterpret_cast<const bf16x8*>(sW + base + ((mt * 2 + 1) * 64 + lane) * 8);
#pragma unroll
      for (int t = 0; t < NT; ++t) z[t][mt] = mfma32(w1, a[t][1], mfma32(w0, a[t][0], c));
    }
  }
  floatx4 c;
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] = sB[192 + 4 * g + i];
  const bf16x8 w0 = *reinterpret_cast<const bf16x8*>(sW + kPF3 + lane * 8);
  const bf16x8 w1 = *reinterpret_cast<const bf16x8*>(sW + kPF3 + (64 + lane) * 8);
#pragma unroll
  for (int t = 0; t < NT; ++t) y[t] = mfma32(w1, a[t][1], mfma32(w0, a[t][0], c));
}

// ---------------------------------------------------------------- training: forward + backward
// Each wave handles kTilesPerWave tiles of 16 samples. Writes BF16 activations and deltas
// feature-major ([feature][batch]) for the weight-gradient GEMM, and per-block FP32 bias
// gradient and FP64 loss partials.
__global__ void __launch_bounds__(256) k_fwdbwd(MlpArgs M, TrainArgs T) {
  __shared__ __attribute__((aligned(16))) __bf16 sW[kPackTotal];
  __shared__ float sB[208];
  __shared__ float sNorm[40];
  __shared__ float sRed[4][208];
  __shared__ double sLoss[4];
  stage_params(M, sW, sB, kPackTotal);
  if (threadIdx.x < 14) {
    sNorm[threadIdx.x] = M.x_mu[threadIdx.x];
    sNorm[14 + threadIdx.x] = 1.f / M.x_sd[threadIdx.x];
  }
  if (threadIdx.x < 6) {
    sNorm[28 + threadIdx.x] = M.y_mu[threadIdx.x];
    sNorm[34 + threadIdx.x] = 1.f / M.y_sd[threadIdx.x];
  }
  __syncthreads();
  const int lane = __lane_id();
  const int g = lane >> 4, p = lane & 15;
  const int wave = threadIdx.x >> 6;
  const int B = T.batch;
  float db[3][16];
  float db4[4];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int k = 0; k < 16; ++k) db[l][k] = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) db4[i] = 0.f;
  double loss = 0.0;
  const float scale = 2.f / ((float)B * 6.f);

  const int tiles_total = B / 16;
  const int wave_global = blockIdx.x * 4 + wave;
  // the rows of every tile of the wave, then the raw inputs and targets of one tile ahead,
  // requested before the work on the current tile (the gathers are random reads)
  int64_t smpv[kTilesPerWave];
#pragma unroll
  for (int tt = 0; tt < kTilesPerWave; ++tt) {
    const int tile = wave_global * kTilesPerWave + tt;
    const int b = tile * 16 + p;
    int64_t smp = 0;
    if (tile < tiles_total) smp = T.idx ? (int64_t)T.idx[b] : (int64_t)b;
    smpv[tt] = smp < 0 ? 0 : (smp >= T.n_rows ? T.n_rows - 1 : smp);
  }
  float xr[4], yr[4];
  auto fetch = [&](int64_t smp) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = 4 * g + j;
      xr[j] = (f < 14) ? T.x[smp * 14 + f] : 0.f;
      const int o = 4 * g + j;
      yr[j] = (o < 6) ? T.y[smp * 6 + o] : 0.f;
    }
  };
  if (wave_global * kTilesPerWave < tiles_total) fetch(smpv[0]);
  for (int tt = 0; tt < kTilesPerWave; ++tt) {
    const int tile = wave_global * kTilesPerWave + tt;
    if (tile >= tiles_total) break;  // uniform per wave
    const int b = tile * 16 + p;
    float xc[4], yc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      xc[j] = xr[j];
      yc[j] = yr[j];
    }
    if (tt + 1 < kTilesPerWave && tile + 1 < tiles_total) fetch(smpv[tt + 1]);
    // inputs: features 4g..4g+3 (14 real), standardised
    float xs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = 4 * g + j;
      xs[j] = (f < 14) ? (xc[j] - sNorm[f]) * sNorm[14 + f] : 0.f;
    }
    const short4v x = pack4(xs[0], xs[1], xs[2], xs[3]);
    Fwd F;
    forward(sW, sB, x, F);
    // loss and output delta (rows 4g+i < 6)
    floatx4 dz4;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * g + i;
      float d = 0.f;
      if (o < 6) {
        const float t = (yc[i] - sNorm[28 + o]) * sNorm[34 + o];
        d = F.y[i] - t;
        loss += (double)d * (double)d;
      }
      dz4[i] = d * scale;
      db4[i] += dz4[i];
    }
    // store A0 (16 rows), A1..A3, dZ4 feature-major
    {
      __bf16* A0 = T.act0;
#pragma unroll
      for (int j = 0; j < 4; ++j) A0[(4 * g + j) * (int64_t)B + b] = to_bf16(xs[j]);
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        __bf16* Al = T.act[l];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int j = 0; j < 8; ++j) Al[perm64(s, g, j) * (int64_t)B + b] = F.a[l][s][j];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) T.dz4[(4 * g + i) * (int64_t)B + b] = to_bf16(dz4[i]);
    }
    // dA3 = W4^T dZ4 (16x16x16, K = outputs)
    const short4v dz4b = pack4(dz4[0], dz4[1], dz4[2], dz4[3]);
    floatx4 dz[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      floatx4 c = {0.f, 0.f, 0.f, 0.f};
      const short4v w = *reinterpret_cast<const short4v*>(sW + kPB3 + (mt * 64 + lane) * 4);
      c = mfma16(w, dz4b, c);
#pragma unroll
      for (int i = 0; i < 4; ++i) c[i] *= gelu_grad(F.z[2][mt][i]);
      dz[mt] = c;
    }
    // layers 3 and 2 backward: dZ_l stored, dA_{l-1} = W_l^T dZ_l, then times gelu'
#pragma unroll
    for (int l = 2; l >= 1; --l) {
      __bf16* Dl = T.dz[l];  // dz[2] = dZ3, dz[1] = dZ2
      bf16x8 ops[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        ops[s] = pack8(dz[2 * s], dz[2 * s + 1]);
#pragma unroll
        for (int j = 0; j < 8; ++j) Dl[perm64(s, g, j) * (int64_t)B + b] = ops[s][j];
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) db[l][4 * mt + i] += dz[mt][i];
      const int base = (l == 2) ? kPB2 : kPB1;
      floatx4 nd[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) {
        floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const bf16x8 w = *reinterpret_cast<const bf16x8*>(sW + base + ((mt * 2 + s) * 64 + lane) * 8);
          c = mfma32(w, ops[s], c);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) c[i] *= gelu_grad(F.z[l - 1][mt][i]);
        nd[mt] = c;
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) dz[mt] = nd[mt];
    }
    // dZ1 stored
    {
      __bf16* D0 = T.dz[0];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 o = pack8(dz[2 * s], dz[2 * s + 1]);
#pragma unroll
        for (int j = 0; j < 8; ++j) D0[perm64(s, g, j) * (int64_t)B + b] = o[j];
      }
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) db[0][4 * mt + i] += dz[mt][i];
    }
  }
  // bias-gradient partials: sum over the 16 points of each lane row, then over waves
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      float v = db[l][k];
#pragma unroll
      for (int d = 1; d < 16; d <<= 1) v += __shfl_xor(v, d);
      db[l][k] = v;
    }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float v = db4[i];
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) v += __shfl_xor(v, d);
    db4[i] = v;
  }
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) loss += __shfl_xor(loss, d);
  if (p == 0) {
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) sRed[wave][64 * l + 16 * mt + 4 * g + i] = db[l][4 * mt + i];
#pragma unroll
    for (int i = 0; i < 4; ++i) sRed[wave][192 + 4 * g + i] = db4[i];
  }
  if (lane == 0) sLoss[wave] = loss;
  __syncthreads();
  if (threadIdx.x < 198) {
    const int k = threadIdx.x;
    const float v = sRed[0][k] + sRed[1][k] + sRed[2][k] + sRed[3][k];
    T.db_part[(int64_t)blockIdx.x * 198 + k] = v;
  }
  if (threadIdx.x == 0) T.loss_part[blockIdx.x] = sLoss[0] + sLoss[1] + sLoss[2] + sLoss[3];
}

// ---------------------------------------------------------------- weight gradients (split K)
// Tile pairs (layer, m tile, n tile): W1 4x1, W2 4x4, W3 4x4, W4 1x4 = 40 pairs, 10 per wave.
__device__ __forceinline__ void pair_info(int tp, int& layer, int& mt, int& nt) {
  if (tp < 4) { layer = 0; mt = tp; nt = 0; return; }
  if (tp < 20) { layer = 1; mt = (tp - 4) >> 2; nt = (tp - 4) & 3; return; }
  if (tp < 36) { layer = 2; mt = (tp - 20) >> 2; nt = (tp - 20) & 3; return; }
  layer = 3; mt = 0; nt = tp - 36;
}

__global__ void __launch_bounds__(256) k_wgrad(TrainArgs T, int chunk) {
  const int lane = __lane_id();
  const int g = lane >> 4, r = lane & 15;
  const int wave = threadIdx.x >> 6;
  const int64_t B = T.batch;
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  floatx4 acc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) acc[k] = floatx4{0.f, 0.f, 0.f, 0.f};
  // operands of the next K step are requested before the products of the current one
  const __bf16* rowD[10];
  const __bf16* rowA[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    int layer, mt, nt;
    pair_info(wave * 10 + k, layer, mt, nt);
    const __bf16* D = layer == 0 ? T.dz[0] : layer == 1 ? T.dz[1] : layer == 2 ? T.dz[2] : T.dz4;
    const __bf16* Aprev = layer == 0 ? T.act0 : T.act[layer - 1];
    rowD[k] = D + (16 * mt + r) * B + 8 * g;
    rowA[k] = Aprev + (16 * nt + r) * B + 8 * g;
  }
  bf16x8 na[10], nb[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    na[k] = *reinterpret_cast<const bf16x8*>(rowD[k] + p0);
    nb[k] = *reinterpret_cast<const bf16x8*>(rowA[k] + p0);
  }
  for (int64_t ks = p0; ks < p0 + chunk; ks += 32) {
    bf16x8 ca[10], cb[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) {
      ca[k] = na[k];
      cb[k] = nb[k];
    }
    if (ks + 32 < p0 + chunk) {
#pragma unroll
      for (int k = 0; k < 10; ++k) {
        na[k] = *reinterpret_cast<const bf16x8*>(rowD[k] + ks + 32);
        nb[k] = *reinterpret_cast<const bf16x8*>(rowA[k] + ks + 32);
      }
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[k] = mfma32(ca[k], cb[k], acc[k]);
  }
  float* out = T.w_part + (int64_t)blockIdx.x * kNParams;
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    int layer, mt, nt;
    pair_info(wave * 10 + k, layer, mt, nt);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 16 * mt + 4 * g + i;  // output feature (row)
      const int in = 16 * nt + r;          // input feature (column)
      if (layer == 0) {
        if (in < 14) out[kOffW1 + o * 14 + in] = acc[k][i];
      } else if (layer == 1) {
        out[kOffW2 + o * 64 + in] = acc[k][i];
      } else if (layer == 2) {
        out[kOffW3 + o * 64 + in] = acc[k][i];
      } else {
        if (o < 6) out[kOffW4 + o * 64 + in] = acc[k][i];
      }
    }
  }
}

// ---------------------------------------------------------------- reduce + Adam
__device__ __forceinline__ int bias_slot(int i) {
  if (i >= kOffB1 && i < kOffB1 + 64) return i - kOffB1;
  if (i >= kOffB2 && i < kOffB2 + 64) return 64 + i - kOffB2;
  if (i >= kOffB3 && i < kOffB3 + 64) return 128 + i - kOffB3;
  if (i >= kOffB4 && i < kOffB4 + 6) return 192 + i - kOffB4;
  return -1;
}

// Gradient of every parameter from the partials of the split-K weight pass and of the
// forward/backward blocks. A block owns kRedCols consecutive parameters; thread slice k of
// a column sums partials k, k + kRedSlices, ... and the slices are then added in order, so
// the result does not depend on timing.
constexpr int kRedCols = 32, kRedSlices = 8;

// The gradient of parameter i = blockIdx.x * kRedCols + threadIdx.x % kRedCols, valid in the
// threads of slice 0 (the others return 0).
__device__ __forceinline__ float reduce_param(const TrainArgs& T, int nw_part, int ndb_part,
                                              float (&sp)[kRedSlices][kRedCols]) {
  static_assert(kRedCols * kRedSlices == 256, "one thread per (column, slice)");
  const int col = threadIdx.x % kRedCols, slice = threadIdx.x / kRedCols;
  const int i = blockIdx.x * kRedCols + col;
  float s = 0.f;
  if (i < kNParams) {
    const int bs = bias_slot(i);
    // unrolled so that several loads are in flight; the additions stay in partial order
    if (bs < 0) {
#pragma unroll 8
      for (int c = slice; c < nw_part; c += kRedSlices) s += T.w_part[(int64_t)c * kNParams + i];
    } else {
#pragma unroll 8
      for (int c = slice; c < ndb_part; c += kRedSlices) s += T.db_part[(int64_t)c * 198 + bs];
    }
  }
  sp[slice][col] = s;
  __syncthreads();
  float t = 0.f;
  if (slice == 0 && i < kNParams) {
    t = sp[0][col];
#pragma unroll
    for (int k = 1; k < kRedSlices; ++k) t += sp[k][col];
  }
  return t;
}

__global__ void __launch_bounds__(256) k_grad_reduce(TrainArgs T, int nw_part, int ndb_part,
                                                     float* __restrict__ grad) {
  __shared__ float sp[kRedSlices][kRedCols];
  const float t = reduce_param(T, nw_part, ndb_part, sp);
  const int i = blockIdx.x * kRedCols + threadIdx.x % kRedCols;
  if (threadIdx.x < kRedCols && i < kNParams) grad[i] = t;
}

// Adam update of one parameter from its gradient g (bias-corrected moments, c1 and c2).
__device__ __forceinline__ void adam_param(const MlpArgs& M, const AdamArgs& A, int i, float g) {
  const float m = A.b1 * M.m[i] + (1.f - A.b1) * g;
  const float v = A.b2 * M.v[i] + (1.f - A.b2) * g * g;
  M.m[i] = m;
  M.v[i] = v;
  const float mh = m * A.c1;  // 1 / (1 - b1^t)
  const float vh = v * A.c2;  // 1 / (1 - b2^t)
  M.params[i] -= A.lr * mh / (sqrtf(vh) + A.eps);
}

// The BF16 operand entries of a weight (k_pack's layouts, inverted): after an Adam update
// the thread that changed parameter i writes them, so a training step needs no packing pass.
// Biases are not packed. Padding entries never change.
__device__ __forceinline__ void repack_param(__bf16* __restrict__ out, int i, float v) {
  const __bf16 b = to_bf16(v);
  // (s, g, j) of input column c in the 16x16x32 operands: c = perm64(s, g, j)
  auto inv64 = [](int c, int& sv, int& gv, int& jv) {
    sv = c >> 5;
    gv = (c >> 2) & 3;
    jv = 4 * ((c >> 4) & 1) + (c & 3);
  };
  if (i < kOffB1) {  // W1 [64][14]: 16x16x16 [mt][lane][j]
    const int o = i / 14, in = i % 14;
    out[((o >> 4) * 64 + 16 * (in >> 2) + (o & 15)) * 4 + (in & 3)] = b;
  } else if ((i >= kOffW2 && i < kOffB2) || (i >= kOffW3 && i < kOffB3)) {  // W2, W3 [64][64]
    const bool w2 = i < kOffB2;
    const int k = i - (w2 ? kOffW2 : kOffW3);
    const int o = k >> 6, c = k & 63;
    int sv, gv, jv;
    inv64(c, sv, gv, jv);  // forward: rows o, K = inputs
    out[(w2 ? kPF1 : kPF2) + (o >> 4) * 1024 + sv * 512 + (16 * gv + (o & 15)) * 8 + jv] = b;
    inv64(o, sv, gv, jv);  // transposed: rows = inputs, K = outputs
    out[(w2 ? kPB1 : kPB2) + (c >> 4) * 1024 + sv * 512 + (16 * gv + (c & 15)) * 8 + jv] = b;
  } else if (i >= kOffW4 && i < kOffB4) {  // W4 [6][64]
    const int k = i - kOffW4;
    const int o = k >> 6, c = k & 63;
    int sv, gv, jv;
    inv64(c, sv, gv, jv);  // forward 16x16x32 [s][lane][j], rows = outputs
    out[kPF3 + sv * 512 + (16 * gv + o) * 8 + jv] = b;
    // transposed 16x16x16 [mt][lane][j]: rows = inputs, K = outputs
    out[kPB3 + (c >> 4) * 256 + (16 * (o >> 2) + (c & 15)) * 4 + (o & 3)] = b;
  }
}

// Mean loss of the batch from its partials: the first wave of the calling block, in a fixed
// order.
__device__ __forceinline__ void loss_mean(const double* __restrict__ loss_part, int nloss,
                                          double den, float* loss_out) {
  const int t = threadIdx.x;
  if (t < 64) {
    double s = 0;
    for (int c = t; c < nloss; c += 64) s += loss_part[c];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (t == 0) *loss_out = (float)(s / den);
  }
}

// The gradient reduction and the Adam step in one launch for a training step: each parameter
// is updated by the thread that sums its gradient.
__global__ void __launch_bounds__(256) k_grad_adam(TrainArgs T, int nw_part, int ndb_part,
                                                   MlpArgs M, AdamArgs A,
                                                   const double* __restrict__ loss_part, int nloss,
                                                   float* __restrict__ loss_out,
                                                   __bf16* __restrict__ packed) {
  __shared__ float sp[kRedSlices][kRedCols];
  const float g = reduce_param(T, nw_part, ndb_part, sp);
  const int i = blockIdx.x * kRedCols + threadIdx.x % kRedCols;
  if (threadIdx.x < kRedCols && i < kNParams) {
    adam_param(M, A, i, g);
    repack_param(packed, i, M.params[i]);
  }
  if (blockIdx.x == 0 && loss_out) loss_mean(loss_part, nloss, A.loss_den, loss_out);
}


// ---------------------------------------------------------------- forward on feature rows
__global__ void __launch_bounds__(256) k_predict(MlpArgs M, const float* __restrict__ x,
                                                 int64_t n, float* __restrict__ y_out) {
  __shared__ __attribute__((aligned(16))) __bf16 sW[kPF3 + 1024];
  __shared__ float sB[208];
  __shared__ float sNorm[28];
  stage_params(M, sW, sB, kPF3 + 1024);
  if (threadIdx.x < 14) {
    sNorm[threadIdx.x] = M.x_mu[threadIdx.x];
    sNorm[14 + threadIdx.x] = 1.f / M.x_sd[threadIdx.x];
  }
  __syncthreads();
  const int lane = __lane_id();
  const int g = lane >> 4, p = lane & 15;
  const int64_t tiles = (n + 15) / 16;
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= tiles) return;
  const int64_t b = tile * 16 + p;
  float xs[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int f = 4 * g + j;
    xs[j] = (f < 14 && b < n) ? (x[b * 14 + f] - sNorm[f]) * sNorm[14 + f] : 0.f;
  }
  Fwd F;
  forward(sW, sB, pack4(xs[0], xs[1], xs[2], xs[3]), F);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (4 * g + i < 6 && b < n) y_out[b * 6 + 4 * g + i] = F.y[i];
}

// ---------------------------------------------------------------- features from fields
__device__ __forceinline__ void grad_at(const float* __restrict__ ut, int64_t g, int x, int y,
                                        int z, int nx, int ny, int nz, int64_t ntot, float inv2h,
                                        float (&G)[3][3]) {
  const int64_t plane = (int64_t)nx * ny;
  const int64_t xp = g - x + (x + 1 == nx ? 0 : x + 1), xm = g - x + (x == 0 ? nx - 1 : x - 1);
  const int64_t yp = g + (int64_t)((y + 1 == ny ? 0 : y + 1) - y) * nx;
  const int64_t ym = g + (int64_t)((y == 0 ? ny - 1 : y - 1) - y) * nx;
  const int64_t zp = g + (int64_t)((z + 1 == nz ? 0 : z + 1) - z) * plane;
  const int64_t zm = g + (int64_t)((z == 0 ? nz - 1 : z - 1) - z) * plane;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float* u = ut + i * ntot;
    G[i][0] = (u[xp] - u[xm]) * inv2h;
    G[i][1] = (u[yp] - u[ym]) * inv2h;
    G[i][2] = (u[zp] - u[zm]) * inv2h;
  }
}

// The 14 inputs: g = Delta G (9, row-major) and tr(s^2), tr(r^2), tr(s^3), tr(s r^2),
// tr(s^2 r^2) with s, r the symmetric and antisymmetric parts of g.
__device__ __forceinline__ void features14(const float (&G)[3][3], float delta, float (&f)[14]) {
  float gg[3][3], s[3][3], r[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) gg[i][j] = delta * G[i][j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      s[i][j] = 0.5f * (gg[i][j] + gg[j][i]);
      r[i][j] = 0.5f * (gg[i][j] - gg[j][i]);
    }
  float ss[3][3], rr[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      ss[i][j] = s[i][0] * s[0][j] + s[i][1] * s[1][j] + s[i][2] * s[2][j];
      rr[i][j] = r[i][0] * r[0][j] + r[i][1] * r[1][j] + r[i][2] * r[2][j];
    }
  float l1 = 0, l2 = 0, l3 = 0, l4 = 0, l5 = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    l1 += ss[i][i];
    l2 += rr[i][i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      l3 += ss[i][k] * s[k][i];
      l4 += s[i][k] * rr[k][i];
      l5 += ss[i][k] * rr[k][i];
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) f[3 * i + j] = gg[i][j];
  f[9] = l1;
  f[10] = l2;
  f[11] = l3;
  f[12] = l4;
  f[13] = l5;
}

__global__ void __launch_bounds__(256) k_features(FeatArgs A) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t plane = (int64_t)A.nx * A.ny;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < A.ntot; g += stride) {
    const int x = (int)(g % A.nx), y = (int)((g / A.nx) % A.ny), z = (int)(g / plane);
    float G[3][3];
    grad_at(A.ut, g, x, y, z, A.nx, A.ny, A.nz, A.ntot, A.inv2h, G);
    float f[14];
    features14(G, A.delta, f);
#pragma unroll
    for (int k = 0; k < 14; ++k) A.x[g * 14 + k] = f[k];
    if (A.y) {
      const float inv = 1.f / A.rho_bar[g];
#pragma unroll
      for (int c = 0; c < 6; ++c) A.y[g * 6 + c] = A.tau[c * A.ntot + g] * inv;
    }
  }
}

// Column sums, sums of squares (FP64), minima and maxima of an n x ncol row-major matrix.
__global__ void __launch_bounds__(256) k_colstats(const float* __restrict__ X, int64_t n, int ncol,
                                                  double* __restrict__ part) {
  // block b handles rows [b*chunk, ...); thread t handles column t % ncol on rows t / ncol + k*step
  __shared__ double sh[256][2];
  __shared__ float sm[256][2];
  const int t = threadIdx.x;
  const int rows_per_iter = 256 / ncol;
  const int col = t % ncol, r0 = t / ncol;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t a = (int64_t)blockIdx.x * chunk;
  const int64_t e = a + chunk < n ? a + chunk : n;
  double s = 0, s2 = 0;
  float mn = INFINITY, mx = -INFINITY;
  if (r0 < rows_per_iter) {
    for (int64_t i = a + r0; i < e; i += rows_per_iter) {
      const float v = X[i * ncol + col];
      s += v;
      s2 += (double)v * v;
      mn = fminf(mn, v);
      mx = fmaxf(mx, v);
    }
  }
  sh[t][0] = s;
  sh[t][1] = s2;
  sm[t][0] = mn;
  sm[t][1] = mx;
  __syncthreads();
  if (t < ncol) {
    double S = 0, S2 = 0;
    float MN = INFINITY, MX = -INFINITY;
    for (int k = t; k < rows_per_iter * ncol; k += ncol) {
      S += sh[k][0];
      S2 += sh[k][1];
      MN = fminf(MN, sm[k][0]);
      MX = fmaxf(MX, sm[k][1]);
    }
    double* o = part + ((int64_t)blockIdx.x * ncol + t) * 4;
    o[0] = S;
    o[1] = S2;
    o[2] = MN;
    o[3] = MX;
  }
}

// ---------------------------------------------------------------- inference over a field
// Makes LDS writes of this wave visible to its other lanes (LDS only: outstanding global
// memory operations are not waited for).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int kXS = 17;  // LDS row stride of one point's 16 standardised inputs (odd: no conflicts)
constexpr int kYS = 9;   // LDS row stride of one point's outputs

// What the gradient of one point needs: ut_i at the six neighbours (x+, x-, y+, y-, z+, z-)
// and rho_bar of the point.
struct InferLoads {
  float u[3][6];
  float rb;
};

// Coordinates of point gi (clamped to the last point past the end) and its loads.
__device__ __forceinline__ void infer_load(const InferArgs& I, int64_t base, int lane,
                                           InferLoads& L, int64_t& gc, bool& inside) {
  const int64_t row = base / I.nx;
  int x = (int)(base - row * I.nx) + lane;
  int y = (int)(row % I.ny), z = (int)(row / I.ny);
  while (x >= I.nx) {
    x -= I.nx;
    if (++y == I.ny) {
      y = 0;
      ++z;
    }
  }
  const int64_t gi = base + lane;
  inside = gi < I.ntot;
  if (!inside) {
    x = I.nx - 1;
    y = I.ny - 1;
    z = I.nz - 1;
  }
  gc = inside ? gi : I.ntot - 1;
  const int64_t plane = (int64_t)I.nx * I.ny;
  const int64_t o[6] = {gc - x + (x + 1 == I.nx ? 0 : x + 1), gc - x + (x == 0 ? I.nx - 1 : x - 1),
                        gc + (int64_t)((y + 1 == I.ny ? 0 : y + 1) - y) * I.nx,
                        gc + (int64_t)((y == 0 ? I.ny - 1 : y - 1) - y) * I.nx,
                        gc + (int64_t)((z + 1 == I.nz ? 0 : z + 1) - z) * plane,
                        gc + (int64_t)((z == 0 ? I.nz - 1 : z - 1) - z) * plane};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int d = 0; d < 6; ++d) L.u[i][d] = I.ut[i * I.ntot + o[d]];
  L.rb = I.rho_bar[gc];
}

// One wave per 64 consecutive points. Every lane derives the gradient, the 14 inputs and the
// envelope test of its own point; the standardised inputs go through LDS into the MFMA
// layout of four 16-point tiles, which run through the network together, and the network
// outputs come back through the same LDS rows to the lane of their point, which applies the
// unstandardisation, or the gradient model tau_gm = rho_bar C2 G G^T where the inputs leave
// the training box or are not finite, and stores tau (64 consecutive points per store).
__global__ void __launch_bounds__(256) k_infer(MlpArgs M, InferArgs I) {
  __shared__ __attribute__((aligned(16))) __bf16 sW[kPF3 + 1024];
  __shared__ float sB[208];
  __shared__ float sNorm[68];
  __shared__ float sX[4 * 64 * kXS];
  static_assert(kYS <= kXS, "outputs reuse the input rows");
  stage_params(M, sW, sB, kPF3 + 1024);
  if (threadIdx.x < 14) {
    sNorm[threadIdx.x] = M.x_mu[threadIdx.x];
    sNorm[14 + threadIdx.x] = 1.f / M.x_sd[threadIdx.x];
    sNorm[40 + threadIdx.x] = M.x_lo[threadIdx.x];
    sNorm[54 + threadIdx.x] = M.x_hi[threadIdx.x];
  }
  if (threadIdx.x < 6) {
    sNorm[28 + threadIdx.x] = M.y_mu[threadIdx.x];
    sNorm[34 + threadIdx.x] = M.y_sd[threadIdx.x];
  }
  __syncthreads();
  const int lane = __lane_id();
  const int g = lane >> 4, p = lane & 15;
  const int wv = threadIdx.x >> 6;
  float* xw = sX + wv * 64 * kXS;  // this wave's 64 rows: inputs, then outputs
  const int64_t ntiles = (I.ntot + 15) / 16;
  const int64_t nchunks = (I.ntot + 63) / 64;
  const int64_t cstep = (int64_t)gridDim.x * 4;
  int64_t fallback = 0;
  for (int64_t chunk = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + wv); chunk < nchunks;
       chunk += cstep) {
    const int64_t gi = chunk * 64 + lane;
    InferLoads L;
    int64_t gc;
    bool in_cur;
    infer_load(I, chunk * 64, lane, L, gc, in_cur);
    const float rb = L.rb;
    float G[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) G[i][j] = (L.u[i][2 * j] - L.u[i][2 * j + 1]) * I.inv2h;
    float f[14];
    features14(G, I.delta, f);
    bool out = false;
    float* xr = xw + lane * kXS;
#pragma unroll
    for (int k = 0; k < 14; ++k) {
      const float v = (f[k] - sNorm[k]) * sNorm[14 + k];
      out = out || !(v >= sNorm[40 + k] && v <= sNorm[54 + k]);
      xr[k] = isfinite(v) ? v : 0.f;
    }
    xr[14] = 0.f;
    xr[15] = 0.f;
    wave_lds_sync();
    // the four tiles through the network together; their outputs go to the rows of their
    // points after every input row has been read
    short4v xin[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const float* src = xw + (16 * t + p) * kXS + 4 * g;
      xin[t] = pack4(src[0], src[1], src[2], src[3]);
    }
    floatx4 yv[4];
    forward_tiles<4>(sW, sB, xin, yv);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float* dst = xw + (16 * t + p) * kXS + 4 * g;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (4 * g + i < 6) dst[i] = yv[t][i];
    }
    wave_lds_sync();
    const float* yr = xw + lane * kXS;
    const int ii[6] = {0, 0, 0, 1, 1, 2};
    const int jj[6] = {0, 1, 2, 1, 2, 2};
    if (in_cur) {
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        float v;
        if (out) {
          const int a = ii[c], bb = jj[c];
          v = I.gm_coef * rb * (G[a][0] * G[bb][0] + G[a][1] * G[bb][1] + G[a][2] * G[bb][2]);
        } else {
          v = rb * fmaf(sNorm[34 + c], yr[c], sNorm[28 + c]);
        }
        I.tau[c * I.ntot + gi] = v;
      }
    }
    const unsigned long long bal = __ballot(out && in_cur);
    if (I.mask && lane < 4 && chunk * 4 + lane < ntiles)
      I.mask[chunk * 4 + lane] = (uint16_t)((bal >> (16 * lane)) & 0xFFFFull);
    fallback += __popcll(bal);
    // the outputs of this chunk are read before the next chunk overwrites them
    wave_lds_sync();
  }
  if (I.fallback_part && lane == 0)
    I.fallback_part[(int64_t)blockIdx.x * 4 + wv] = fallback;
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_pack(const float* params, __bf16* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((kPackTotal + 255) / 256), dim3(256), 0, s, params, packed);
  return hipGetLastError();
}

hipError_t launch_train_passes(const MlpArgs& M, const TrainArgs& T, int* n_fb_blocks,
                               int* n_w_parts, hipStream_t s) {
  const int tiles = T.batch / 16;
  const int waves = (tiles + kTilesPerWave - 1) / kTilesPerWave;
  const int blocks = (waves + 3) / 4;
  hipLaunchKernelGGL(k_fwdbwd, dim3(blocks), dim3(256), 0, s, M, T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int chunk = wgrad_chunk(T.batch);
  hipLaunchKernelGGL(k_wgrad, dim3(T.batch / chunk), dim3(256), 0, s, T, chunk);
  *n_fb_blocks = blocks;
  *n_w_parts = T.batch / chunk;
  return hipGetLastError();
}

int fwdbwd_blocks(int batch) {
  const int tiles = batch / 16;
  const int waves = (tiles + kTilesPerWave - 1) / kTilesPerWave;
  return (waves + 3) / 4;
}

// Samples per block of the split-K weight pass: small enough that a batch of 65 536 spreads
// over 256 blocks (one per CU), at least one 32-sample K step.
int wgrad_chunk(int batch) {
  int chunk = 1024;
  while (chunk > 32 && batch / chunk < 256) chunk /= 2;
  while (batch % chunk) chunk /= 2;
  return chunk;
}

hipError_t launch_grad_reduce(const TrainArgs& T, int nw_part, int ndb_part, float* grad,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_grad_reduce, dim3((kNParams + kRedCols - 1) / kRedCols), dim3(256), 0, s,
                     T, nw_part, ndb_part, grad);
  return hipGetLastError();
}

hipError_t launch_grad_adam(const TrainArgs& T, int nw_part, int ndb_part, const MlpArgs& M,
                           const AdamArgs& A, const double* loss_part, int nloss, float* loss_out,
                           __bf16* packed, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_adam, dim3((kNParams + kRedCols - 1) / kRedCols), dim3(256), 0, s, T,
                     nw_part, ndb_part, M, A, loss_part, nloss, loss_out, packed);
  return hipGetLastError();
}


hipError_t launch_predict(const MlpArgs& M, const float* x, int64_t n, float* y, hipStream_t s) {
  const int64_t tiles = (n + 15) / 16;
  hipLaunchKernelGGL(k_predict, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, M, x, n, y);
  return hipGetLastError();
}

hipError_t launch_features(const FeatArgs& A, hipStream_t s) {
  int64_t b = (A.ntot + 255) / 256;
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(k_features, dim3((unsigned)b), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_colstats(const float* X, int64_t n, int ncol, double* part, int blocks,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_colstats, dim3(blocks), dim3(256), 0, s, X, n, ncol, part);
  return hipGetLastError();
}

hipError_t launch_infer(const MlpArgs& M, const InferArgs& I, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_infer, dim3(blocks), dim3(256), 0, s, M, I);
  return hipGetLastError();
}

}  // namespace mlp
}  // namespace kcf
