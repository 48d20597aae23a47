// sa_k_mlp.hip -- kernels of the proposal network: batched forward (the
// inference tile of the learned annealing kernel), the training step's
// forward + backward with per-wave gradient partials, and the deterministic
// reduction that applies Adam and rewrites the bf16 fragments.
//
// Training (binary cross-entropy with logits, mean over the batch):
//   dlogit = (sigmoid(logit) - y) / n,  dW2[h] = sum_rows a_h dlogit,
//   dZ = dlogit w2 [z > 0],  dW1 = X^T dZ (the hidden bias is row 31 of W1,
//   fed by the constant input), db2 = sum dlogit.
// Per 32-row tile a wave computes Z = X W1 as two 16-row halves (lane l:
// hidden 16 ht + l%16, rows 4g .. 4g+3 of each half).  Those eight rows are
// exactly the k-slice a lane supplies to dW1^T = dZ^T X when the 32 rows of
// the tile are the MFMA's k in the order (half, 4g + i): dZ never leaves the
// lane that computed it.
#include "sa_device.h"
#include "sa_mlp.h"

namespace sa {

namespace {

__device__ __forceinline__ uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_round(float f) { return (float)(__bf16)f; }

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const uint4 *__restrict__ x, int64_t n,
                                                          float *__restrict__ logit, const uint4 *__restrict__ w1f,
                                                          const uint4 *__restrict__ w2f, const float *__restrict__ master) {
  __shared__ uint4 s_w1f[kW1FragU4];
  __shared__ uint4 s_w2f[kW2FragU4];
  stage_mlp_fragments(s_w1f, s_w2f, w1f, w2f, threadIdx.x, blockDim.x);
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  const float b2 = master[kMlpParams - 1];
  const int64_t tiles = (n + 15) / 16;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t t = wave; t < tiles; t += nwaves) {
    const int64_t row = t * 16 + r;
    const uint4 f = row < n ? x[row * 4 + g] : make_uint4(0u, 0u, 0u, 0u);
    const float l = mlp_tile_logit(as_v8bf(f), s_w1f, s_w2f, lane, b2);
    if (g == 0 && row < n) logit[row] = l;
  }
}

__global__ __launch_bounds__(256) void mlp_train_kernel(MlpTrainArgs a) {
  __shared__ uint4 s_w1f[kW1FragU4];
  __shared__ uint4 s_x[4][32 * 4];  // per wave: one 32-row tile, 4 uint4 per row
  for (int i = threadIdx.x; i < kW1FragU4; i += blockDim.x) s_w1f[i] = a.w1f[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  const int wave = blockIdx.x * 4 + wid;
  if (wave >= a.waves) return;  // no block-level barrier below
  const uint16_t *sx = reinterpret_cast<const uint16_t *>(s_x[wid]);
  const float inv_n = 1.0f / (float)a.n;
  const float b2 = a.master[kMlpParams - 1];
  float w2c[16];
#pragma unroll
  for (int ht = 0; ht < 16; ++ht) w2c[ht] = bf16_round(a.master[kMlpW1 + 16 * ht + r]);

  v4f dw1[16][2];
  float dw2[16];
#pragma unroll
  for (int ht = 0; ht < 16; ++ht) {
    dw1[ht][0] = dw1[ht][1] = v4f{0.f, 0.f, 0.f, 0.f};
    dw2[ht] = 0.f;
  }
  float db2 = 0.f, loss = 0.f;

  for (int t = 0; t < a.tiles_per_wave; ++t) {
    const int64_t row0 = ((int64_t)wave * a.tiles_per_wave + t) * 32;
    if (row0 >= a.n) break;
    uint4 xa[2];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      const int64_t row = row0 + hf * 16 + r;
      xa[hf] = row < a.n ? a.x[row * 4 + g] : make_uint4(0u, 0u, 0u, 0u);
      s_x[wid][(hf * 16 + r) * 4 + g] = xa[hf];
    }
    // pass 1: scores of the 32 rows
    float part[2][4] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    const v4f zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ht = 0; ht < 16; ++ht) {
      const v8bf w = as_v8bf(s_w1f[ht * 64 + lane]);
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const v4f z = mfma_bf16(as_v8bf(xa[hf]), w, zero);
#pragma unroll
        for (int i = 0; i < 4; ++i) part[hf][i] += bf16_round(relu(z[i])) * w2c[ht];
      }
    }
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = part[hf][i];
        v += __shfl_xor(v, 1, kWave);
        v += __shfl_xor(v, 2, kWave);
        v += __shfl_xor(v, 4, kWave);
        v += __shfl_xor(v, 8, kWave);
        part[hf][i] = v;
      }
    float dl[2][4];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + hf * 16 + 4 * g + i;
        const bool valid = row < a.n;
        const float l = part[hf][i] + b2;
        const float yv = valid ? a.y[row] : 0.f;
        const float p = 1.0f / (1.0f + expf(-l));
        dl[hf][i] = valid ? (p - yv) * inv_n : 0.f;
        if (valid && r == 0) {
          loss += (fmaxf(l, 0.f) + log1pf(expf(-fabsf(l))) - yv * l) * inv_n;
          db2 += dl[hf][i];
        }
      }
    wave_sync();
    // X as the B operand of dW1^T: feature 16 ft + r, rows (j/4)*16 + 4g + j%4
    v8bf xb[2];
#pragma unroll
    for (int ft = 0; ft < 2; ++ft)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int rho = (j >> 2) * 16 + 4 * g + (j & 3);
        xb[ft][j] = __builtin_bit_cast(__bf16, sx[rho * 32 + ft * 16 + r]);
      }
    // pass 2: gradients
#pragma unroll
    for (int ht = 0; ht < 16; ++ht) {
      const v8bf w = as_v8bf(s_w1f[ht * 64 + lane]);
      const v4f z0 = mfma_bf16(as_v8bf(xa[0]), w, zero);
      const v4f z1 = mfma_bf16(as_v8bf(xa[1]), w, zero);
      v8bf dz;
      float s = 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        s += bf16_round(relu(z0[i])) * dl[0][i] + bf16_round(relu(z1[i])) * dl[1][i];
        dz[i] = (__bf16)(z0[i] > 0.f ? dl[0][i] * w2c[ht] : 0.f);
        dz[4 + i] = (__bf16)(z1[i] > 0.f ? dl[1][i] * w2c[ht] : 0.f);
      }
      dw2[ht] += s;
      dw1[ht][0] = mfma_bf16(dz, xb[0], dw1[ht][0]);
      dw1[ht][1] = mfma_bf16(dz, xb[1], dw1[ht][1]);
    }
    wave_sync();
  }

  float *out = a.partial + (size_t)wave * kMlpParams;
#pragma unroll
  for (int ht = 0; ht < 16; ++ht)
#pragma unroll
    for (int ft = 0; ft < 2; ++ft)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[(ft * 16 + r) * kMlpHidden + ht * 16 + 4 * g + i] = dw1[ht][ft][i];
#pragma unroll
  for (int ht = 0; ht < 16; ++ht) {
    float v = dw2[ht];
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    if (g == 0) out[kMlpW1 + ht * 16 + r] = v;
  }
  db2 = wave_sum_f(db2);
  loss = wave_sum_f(loss);
  if (lane == 0) {
    out[kMlpParams - 1] = db2;
    a.loss_partial[wave] = loss;
  }
}

// One thread per parameter: the batch gradient as the sum of the wave
// partials in wave order (deterministic), then Adam, then the bf16 copy in
// its fragment position.
__global__ __launch_bounds__(256) void mlp_update_kernel(MlpUpdateArgs a) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0 && a.loss_out) {
    float s = 0.f;
    for (int w = 0; w < a.waves; ++w) s += a.loss_partial[w];
    *a.loss_out = s;
  }
  if (q >= kMlpParams) return;
  if (a.waves > 0) {
    float gsum = 0.f;
    for (int w = 0; w < a.waves; ++w) gsum += a.partial[(size_t)w * kMlpParams + q];
    if (a.grad_out) a.grad_out[q] = gsum;
    if (a.adam) {
      const float m = a.beta1 * a.m[q] + a.omb1 * gsum;
      const float v = a.beta2 * a.v[q] + a.omb2 * (gsum * gsum);
      a.m[q] = m;
      a.v[q] = v;
      a.master[q] -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
    }
  }
  const float w = a.master[q];
  if (q < kMlpW1) {
    const int k = q / kMlpHidden, h = q % kMlpHidden;
    const int lane = (h & 15) + 16 * (k >> 3);
    reinterpret_cast<uint16_t *>(a.w1f)[((h >> 4) * 64 + lane) * 8 + (k & 7)] = bf16_bits(w);
  } else if (q < kMlpW1 + kMlpHidden) {
    const int h = q - kMlpW1, u = h >> 5, within = h & 31, rem = within & 15;
    const int j = 4 * (within >> 4) + (rem & 3);
    reinterpret_cast<uint16_t *>(a.w2f)[((u * 4) + (rem >> 2)) * 8 + j] = bf16_bits(w);
  }
}

}  // namespace

hipError_t launch_mlp_forward(const uint4 *x, int64_t n, float *logit, const uint4 *w1f, const uint4 *w2f,
                              const float *master, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t tiles = (n + 15) / 16;
  const unsigned blocks = (unsigned)std::min<int64_t>((tiles + 3) / 4, 4096);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(256), 0, stream, x, n, logit, w1f, w2f, master);
  return hipGetLastError();
}

hipError_t launch_mlp_train(const MlpTrainArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(mlp_train_kernel, dim3((unsigned)((a.waves + 3) / 4)), dim3(256), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_mlp_update(const MlpUpdateArgs &a, hipStream_t stream) {
  hipLaunchKernelGGL(mlp_update_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace sa
