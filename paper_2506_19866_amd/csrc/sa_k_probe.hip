// sa_k_probe.hip -- instruction-throughput probes: the measured peaks that
// the benchmark's roofline figures divide by (the published chip figures
// cover floating-point arithmetic only, and the annealing kernels are bound
// by 32-bit integer VALU issue and the packing conversion).
//
// Every probe runs the whole GPU at full occupancy: each lane keeps 8
// independent dependency chains of one instruction (so issue, not latency,
// limits it), the loop body is unrolled 32 deep, and an empty asm statement
// after every instruction makes its result opaque so the compiler cannot fold
// the chain.  A result is stored only when it equals a value the host never
// passes, which keeps the work alive without memory traffic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sa_anneal.h"

namespace sa {
namespace {

constexpr int kProbeChains = 8;
constexpr int kProbeUnroll = 4;  // x 8 chains = 32 instructions per loop trip

template <int KIND>
__global__ __launch_bounds__(256) void probe_valu_kernel(uint32_t *sink, int iters, uint32_t k0, uint32_t k1,
                                                         uint32_t never) {
  uint32_t a[kProbeChains];
#pragma unroll
  for (int j = 0; j < kProbeChains; ++j) a[j] = threadIdx.x * (2u * j + 1u) + blockIdx.x;
  const float f0 = (float)(threadIdx.x & 7), f1 = -(float)(threadIdx.x & 3);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < kProbeUnroll; ++r)
#pragma unroll
      for (int j = 0; j < kProbeChains; ++j) {
        if constexpr (KIND == SA_PEAK_VALU_XOR) a[j] = a[j] ^ k0;
        if constexpr (KIND == SA_PEAK_VALU_ADD) a[j] = a[j] + k0;
        if constexpr (KIND == SA_PEAK_VALU_BITOP3) a[j] = __builtin_amdgcn_bitop3_b32(a[j], k0, k1, 0xD8);
        if constexpr (KIND == SA_PEAK_CVT_FP4)
          a[j] = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(a[j], f0, f1, 0.125f, 0);
        asm volatile("" : "+v"(a[j]));
      }
  }
  uint32_t x = 0;
#pragma unroll
  for (int j = 0; j < kProbeChains; ++j) x ^= a[j];
  if (x == never) sink[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

typedef int v6i __attribute__((ext_vector_type(6)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// The 32-value fp6 packing conversion (two groups of 16 float32 registers to
// 6 dwords of fp6 codes): 8 conversions per loop trip from two register sets,
// one xor of a result each keeps them alive.
__global__ __launch_bounds__(256) void probe_cvt_fp6_kernel(uint32_t *sink, int iters, uint32_t never) {
  v16f a[2], b[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      a[j][i] = (float)((threadIdx.x + i + j) & 7) - 3.f;
      b[j][i] = (float)((threadIdx.x * i + j) & 5) - 2.f;
    }
  uint32_t acc = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const v6i x = __builtin_amdgcn_cvt_scalef32_2xpk16_fp6_f32(a[r & 1], b[r & 1], 0.25f);
      acc ^= (uint32_t)x[r % 6];
      asm volatile("" : "+v"(a[r & 1]), "+v"(b[r & 1]));
    }
  }
  if (acc == never) sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Dense fp4 (e2m1) x fp4 products of the unscaled 16x16x128 form, the
// instruction the annealing kernels run: 8 independent accumulators per wave
// (FP6: the B operand read as fp6 e2m3 instead).
template <bool FP6>
__global__ __launch_bounds__(256) void probe_mfma_kernel(float *sink, int iters, float never) {
  v8i a = {}, b = {};
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    a[j] = (int)(0x22222222u + threadIdx.x + j);
    b[j] = (int)(0x04104104u - threadIdx.x - j);
  }
  v4f acc[kProbeChains];
#pragma unroll
  for (int j = 0; j < kProbeChains; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < kProbeUnroll; ++r)
#pragma unroll
      for (int j = 0; j < kProbeChains; ++j)
        acc[j] = FP6 ? __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[j], 4, 2, 0, 0, 0, 0)
                     : __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc[j], 4, 4, 0, 0, 0, 0);
  }
  float x = 0.f;
#pragma unroll
  for (int j = 0; j < kProbeChains; ++j) x += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  if (x == never) sink[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

// LDS read bandwidth: the block fills 16 KB of LDS, then every lane reads
// 16-byte words, the 64 lanes of a wave consecutive ones (every bank once
// per quarter of the wave), into 8 independent accumulators; the base index
// alternates between loop trips and is opaque to the compiler, so no read
// can be hoisted or merged (every index stays below 1024).
constexpr int kLdsWords = 1024;  // 16-byte words
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void probe_lds_kernel(uint32_t *sink, int iters, uint32_t never) {
  __shared__ v4u buf[kLdsWords];
  for (int i = threadIdx.x; i < kLdsWords; i += blockDim.x)
    buf[i] = v4u{(uint32_t)i, (uint32_t)i * 3u, (uint32_t)i * 5u, (uint32_t)i * 7u};
  __syncthreads();
  uint32_t acc[kProbeChains];
#pragma unroll
  for (int j = 0; j < kProbeChains; ++j) acc[j] = 0;
  const int lane_word = (int)threadIdx.x & 63;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < kProbeUnroll; ++r) {
      // 8 reads in flight per wave, from one opaque base and immediate offsets
      int base = lane_word + 512 * ((i + r) & 1);
      asm volatile("" : "+v"(base));
      v4u v[kProbeChains];
#pragma unroll
      for (int j = 0; j < kProbeChains; ++j) v[j] = buf[base + 64 * j];
#pragma unroll
      for (int j = 0; j < kProbeChains; ++j) {
        asm volatile("" : : "v"(v[j]));  // all 16 bytes are read
        acc[j] ^= v[j].x;
        asm volatile("" : "+v"(acc[j]));
      }
    }
  }
  uint32_t x = 0;
#pragma unroll
  for (int j = 0; j < kProbeChains; ++j) x ^= acc[j];
  if (x == never) sink[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

}  // namespace

int probe_iters(int kind) {
  switch (kind) {
    case SA_PEAK_MFMA_FP4:
    case SA_PEAK_MFMA_FP4_FP6:
      return 1024;
    case SA_PEAK_CVT_FP4:
      return 2048;
    case SA_PEAK_CVT_FP6:
      return 256;
    case SA_PEAK_LDS_READ:
      return 1024;
    default:
      return 8192;
  }
}

// Work of one launch: lane-ops (VALU), values converted (conversions), flops
// (matrix products), bytes (LDS reads).
double probe_work(int kind, int blocks, int threads) {
  const double waves = (double)blocks * (threads / 64);
  if (kind == SA_PEAK_CVT_FP6) return waves * probe_iters(kind) * 8 * 64 * 32.0;
  const double instr = waves * probe_iters(kind) * kProbeUnroll * kProbeChains;
  if (kind == SA_PEAK_MFMA_FP4 || kind == SA_PEAK_MFMA_FP4_FP6) return instr * 2.0 * 16 * 16 * 128;
  if (kind == SA_PEAK_LDS_READ) return instr * 64.0 * 16.0;
  return instr * 64.0 * (kind == SA_PEAK_CVT_FP4 ? 2.0 : 1.0);
}

int launch_probe(int kind, void *sink, int blocks, int threads, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const int iters = probe_iters(kind);
  const uint32_t k0 = 0x9E3779B9u, k1 = 0x7F4A7C15u, never = 0xFFFFFFFFu;
  uint32_t *u = static_cast<uint32_t *>(sink);
  switch (kind) {
    case SA_PEAK_VALU_XOR:
      probe_valu_kernel<SA_PEAK_VALU_XOR><<<blocks, threads, 0, s>>>(u, iters, k0, k1, never);
      break;
    case SA_PEAK_VALU_ADD:
      probe_valu_kernel<SA_PEAK_VALU_ADD><<<blocks, threads, 0, s>>>(u, iters, k0, k1, never);
      break;
    case SA_PEAK_VALU_BITOP3:
      probe_valu_kernel<SA_PEAK_VALU_BITOP3><<<blocks, threads, 0, s>>>(u, iters, k0, k1, never);
      break;
    case SA_PEAK_CVT_FP4:
      probe_valu_kernel<SA_PEAK_CVT_FP4><<<blocks, threads, 0, s>>>(u, iters, k0, k1, never);
      break;
    case SA_PEAK_CVT_FP6:
      probe_cvt_fp6_kernel<<<blocks, threads, 0, s>>>(u, iters, never);
      break;
    case SA_PEAK_MFMA_FP4:
      probe_mfma_kernel<false><<<blocks, threads, 0, s>>>(static_cast<float *>(sink), iters, -1.0e30f);
      break;
    case SA_PEAK_MFMA_FP4_FP6:
      probe_mfma_kernel<true><<<blocks, threads, 0, s>>>(static_cast<float *>(sink), iters, -1.0e30f);
      break;
    case SA_PEAK_LDS_READ:
      probe_lds_kernel<<<blocks, threads, 0, s>>>(u, iters, never);
      break;
    default:
      return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

}  // namespace sa
