// sa_mlp.h -- the proposal network (32 inputs -> 256 ReLU units -> 1 score)
// on bf16 MFMA with float32 accumulation: fragment layouts, the inference
// tile shared by the forward kernel and the learned annealing kernel, and the
// training kernels' launch wrappers.  The learned proposal is an extension of
// Table 1's GetCandidate (not in the paper).
//
// Parameters (float32 masters, one flat array of kMlpParams):
//   W1[k][h] (k < 32 inputs, h < 256 hidden; input 31 is the constant 1, so
//   W1[31][.] is the hidden bias), then w2[h], then b2.
// Network:  z_h = sum_k bf16(W1[k][h]) bf16(f_k);  a_h = bf16(max(z_h, 0));
//           logit = sum_h bf16(w2[h]) a_h + b2.
//
// MFMA v_mfma_f32_16x16x32_bf16 (D = A B + C, A 16x32, B 32x16): lane l holds
// row/column l%16 of A/B and the eight k = 8(l/16) .. 8(l/16)+7; D lane l
// holds column l%16, rows 4(l/16) .. 4(l/16)+3.
//   W1 fragments  w1f[ht][lane] (8 bf16): W1[8g + j][16 ht + r]   (g = lane/16, r = lane%16)
//   w2 fragments  w2f[u][g]     (8 bf16): w2[16 (2u + j/4) + 4g + j%4]
// Inference scores 16 moves per tile as Z^T = W1^T F^T (16 MFMAs, lane l then
// holds hidden units 16 ht + 4g + i of move l%16), and the second layer as
// one more MFMA per 32 hidden units whose k-order is exactly the order in
// which a lane already holds them, with w2 replicated over the 16 rows, so
// every lane ends with the score of its move: no cross-lane reduction.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sa {

constexpr int kMlpIn = 32, kMlpHidden = 256;
constexpr int kMlpW1 = kMlpIn * kMlpHidden;         // 8192
constexpr int kMlpParams = kMlpW1 + kMlpHidden + 1;  // 8449
constexpr int kW1FragU4 = 16 * 64;                   // uint4 (8 bf16) per W1 fragment set
constexpr int kW2FragU4 = 8 * 4;
constexpr int kMlpMaxWaves = 1024;                   // partial-gradient slots of a training step

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v8bf as_v8bf(uint4 u) { return __builtin_bit_cast(v8bf, u); }

__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// max(z, 0) for finite z in one v_med3_f32 (fmaxf also canonicalises its
// operand, a second instruction per value)
__device__ __forceinline__ float relu(float z) { return __builtin_amdgcn_fmed3f(z, 0.f, 3.0e38f); }

// Score of move l%16 (every lane) from its features 8g .. 8g+7 (feat), with
// the fragments in LDS.
__device__ __forceinline__ float mlp_tile_logit(v8bf feat, const uint4 *w1f, const uint4 *w2f, int lane, float b2) {
  const int g = lane >> 4;
  v4f out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int u = 0; u < 8; ++u) {
    const v4f zero = {0.f, 0.f, 0.f, 0.f};
    const v4f z0 = mfma_bf16(as_v8bf(w1f[(2 * u) * 64 + lane]), feat, zero);
    const v4f z1 = mfma_bf16(as_v8bf(w1f[(2 * u + 1) * 64 + lane]), feat, zero);
    v8bf h;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      h[i] = (__bf16)relu(z0[i]);
      h[4 + i] = (__bf16)relu(z1[i]);
    }
    out = mfma_bf16(as_v8bf(w2f[u * 4 + g]), h, out);
  }
  return out[0] + b2;
}

// Copies the fragment sets (16.5 KB) from global memory into LDS; every
// thread of the block takes part, the caller synchronizes.
__device__ __forceinline__ void stage_mlp_fragments(uint4 *lds_w1f, uint4 *lds_w2f, const uint4 *w1f, const uint4 *w2f,
                                                    int tid, int nthreads) {
  for (int i = tid; i < kW1FragU4; i += nthreads) lds_w1f[i] = w1f[i];
  for (int i = tid; i < kW2FragU4; i += nthreads) lds_w2f[i] = w2f[i];
}

struct MlpTrainArgs {
  const uint4 *x;      // [n][32] bf16 rows (4 uint4 per row)
  const float *y;      // [n] labels in [0, 1]
  int64_t n;
  int tiles_per_wave;  // 32-row tiles per wave
  int waves;
  const float *master; // parameters (float32)
  const uint4 *w1f;    // W1 fragments (bf16)
  float *partial;      // [waves][kMlpParams] gradient partials
  float *loss_partial; // [waves]
};

struct MlpUpdateArgs {
  const float *partial;
  const float *loss_partial;
  int waves;           // 0: only rewrite the bf16 fragments from the masters
  float *grad_out;     // gradients mode: sums written here (no update)
  float *loss_out;     // optional: mean loss of the batch
  int adam;            // 1: Adam step on the masters
  // beta, 1 - beta and the bias corrections 1 - beta^t, each the float32
  // rounding of its exact decimal value (1 - beta is not taken in float32:
  // 1 - 0.999f is 1.3e-5 off in relative terms)
  float lr, beta1, beta2, omb1, omb2, eps, bc1, bc2;
  float *master, *m, *v;
  uint4 *w1f, *w2f;
};

hipError_t launch_mlp_forward(const uint4 *x, int64_t n, float *logit, const uint4 *w1f, const uint4 *w2f,
                              const float *master, hipStream_t stream);
hipError_t launch_mlp_train(const MlpTrainArgs &a, hipStream_t stream);
hipError_t launch_mlp_update(const MlpUpdateArgs &a, hipStream_t stream);

}  // namespace sa
