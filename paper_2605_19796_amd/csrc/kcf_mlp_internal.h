// Internal declarations of the learned-closure kernels (network 14-64-64-64-6).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kcf {
namespace mlp {

// Parameter vector (float32): W1 (64x14), b1, W2 (64x64), b2, W3 (64x64), b3, W4 (6x64), b4.
constexpr int kOffW1 = 0, kOffB1 = 896, kOffW2 = 960, kOffB2 = 5056, kOffW3 = 5120,
              kOffB3 = 9216, kOffW4 = 9280, kOffB4 = 9664, kNParams = 9670;

// Packed BF16 MFMA operands (lane-ordered): forward W1 (16x16x16), W2, W3 (16x16x32), W4,
// backward W4^T (16x16x16), W3^T, W2^T (16x16x32).
constexpr int kPF1 = 1024, kPF2 = 5120, kPF3 = 9216, kPB3 = 10240, kPB2 = 11264, kPB1 = 15360,
              kPackTotal = 19456;

constexpr int kTilesPerWave = 4;  // 16-sample tiles per wave in the training pass

struct MlpArgs {
  float* params;            // FP32 master parameters (kNParams)
  float* m;                 // Adam first moment
  float* v;                 // Adam second moment
  const __bf16* packed;     // packed BF16 operands (kPackTotal)
  const float* x_mu;        // 14 input means
  const float* x_sd;        // 14 input standard deviations
  const float* y_mu;        // 6 target means
  const float* y_sd;        // 6 target standard deviations
  const float* x_lo;        // 14 lower bounds of standardised inputs (envelope)
  const float* x_hi;        // 14 upper bounds
};

struct TrainArgs {
  const float* x;           // dataset inputs, row-major [n][14] (raw)
  const float* y;           // dataset targets, row-major [n][6] (raw)
  const int32_t* idx;       // batch sample indices (NULL: rows 0..batch-1)
  int64_t n_rows;           // dataset rows; indices are clamped to [0, n_rows)
  int batch;                // multiple of 32
  __bf16* act0;             // [16][batch] standardised inputs (BF16)
  __bf16* act[3];           // [64][batch] hidden activations (BF16)
  __bf16* dz[3];            // [64][batch] hidden pre-activation deltas (BF16)
  __bf16* dz4;              // [16][batch] output deltas (BF16)
  float* db_part;           // [blocks][198] bias-gradient partials
  double* loss_part;        // [blocks] squared-error partials
  float* w_part;            // [chunks][kNParams] weight-gradient partials
};

struct AdamArgs {
  float lr, b1, b2, eps, c1, c2;  // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
  double loss_den;                // batch * 6
};

struct FeatArgs {
  const float* rho_bar;
  const float* ut;
  const float* tau;         // may be NULL when only inputs are wanted
  int nx, ny, nz;
  int64_t ntot;
  float inv2h, delta;
  float* x;                 // [ntot][14]
  float* y;                 // [ntot][6] or NULL
};

struct InferArgs {
  const float* rho_bar;
  const float* ut;
  int nx, ny, nz;
  int64_t ntot;
  float inv2h, delta, gm_coef;
  float* tau;               // [6][ntot]
  uint16_t* mask;           // [ceil(ntot/16)] fallback bits, or NULL
  int64_t* fallback_part;   // [blocks*4] fallback counts, or NULL
};

hipError_t launch_pack(const float* params, __bf16* packed, hipStream_t s);
hipError_t launch_train_passes(const MlpArgs& M, const TrainArgs& T, int* n_fb_blocks,
                               int* n_w_parts, hipStream_t s);
int fwdbwd_blocks(int batch);
int wgrad_chunk(int batch);
hipError_t launch_grad_reduce(const TrainArgs& T, int nw_part, int ndb_part, float* grad,
                              hipStream_t s);
// The gradient reduction, the Adam step and the BF16 operand entries of the updated weights
// (packed: the layouts of launch_pack) in one launch.
hipError_t launch_grad_adam(const TrainArgs& T, int nw_part, int ndb_part, const MlpArgs& M,
                           const AdamArgs& A, const double* loss_part, int nloss, float* loss_out,
                           __bf16* packed, hipStream_t s);
hipError_t launch_predict(const MlpArgs& M, const float* x, int64_t n, float* y, hipStream_t s);
hipError_t launch_features(const FeatArgs& A, hipStream_t s);
hipError_t launch_colstats(const float* X, int64_t n, int ncol, double* part, int blocks,
                           hipStream_t s);
hipError_t launch_infer(const MlpArgs& M, const InferArgs& I, int blocks, hipStream_t s);

}  // namespace mlp
}  // namespace kcf
