// sa_k_batch.hip -- kernels over batches of vectors (cost, trajectories)
// and the per-stage reduction of Table 1.
#include "sa_device.h"

namespace sa {

// ---------------------------------------------------------------------------
// K3 / K4: cost and trajectories of a batch of vectors (one wave per vector)
// ---------------------------------------------------------------------------
template <int NM, int NK, int D>
__global__ __launch_bounds__(256) void eval_kernel(DevProblem pb, const int8_t *__restrict__ x, int64_t n,
                                                   int32_t *__restrict__ cost) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (i >= n) return;
  const int8_t *xi = x + i * pb.P;
  auto xv = [xi](int p) -> int { return xi[p]; };
  SA_DECLARE_A(A, NM, NK);
  build_a(A, pb, lane, xv);
  const int m = wave_sum(lane_mismatch<NM, NK, D, false>(A, pb, lane, pb.obs_r, pb.obs_w, nullptr));
  const int v = wave_sum(lane_violations(pb, lane, xv, nullptr, nullptr));
  if (lane == 0) cost[i] = m + pb.lambda * v;
}

template <int NM, int NK, int D>
__global__ __launch_bounds__(256) void simulate_kernel(DevProblem pb, const int8_t *__restrict__ x, int64_t n,
                                                       int8_t *__restrict__ traj) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t i = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (i >= n) return;
  const int8_t *xi = x + i * pb.P;
  auto xv = [xi](int p) -> int { return xi[p]; };
  SA_DECLARE_A(A, NM, NK);
  build_a(A, pb, lane, xv);
  lane_mismatch<NM, NK, D, true>(A, pb, lane, pb.obs_r, pb.obs_w, traj + (size_t)i * pb.C * (pb.T + 1) * pb.N);
}

// ---------------------------------------------------------------------------
// K2: Table 1's serial part on the device: global best over the chains
// (lowest chain id on ties), its vector copied for the next stage, and the
// stage's statistics summed.  One block of 256.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs ra) {
  __shared__ unsigned long long keys[256];
  __shared__ unsigned long long sums[4][256];
  const int tid = threadIdx.x;
  unsigned long long best = ~0ull;
  unsigned long long s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int64_t c = tid; c < ra.n_chains; c += 256) {
    const unsigned long long key = ((unsigned long long)(uint32_t)ra.cbest[c] << 32) | (unsigned long long)c;
    best = key < best ? key : best;
    s0 += ra.cstats[c * 4 + 0];
    s1 += ra.cstats[c * 4 + 1];
    s2 += ra.cstats[c * 4 + 2];
    s3 += ra.cstats[c * 4 + 3];
  }
  keys[tid] = best;
  sums[0][tid] = s0;
  sums[1][tid] = s1;
  sums[2][tid] = s2;
  sums[3][tid] = s3;
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if (tid < half) {
      const unsigned long long o = keys[tid + half];
      keys[tid] = o < keys[tid] ? o : keys[tid];
#pragma unroll
      for (int q = 0; q < 4; ++q) sums[q][tid] += sums[q][tid + half];
    }
    __syncthreads();
  }
  const int64_t winner = (int64_t)(keys[0] & 0xffffffffull);
  if (tid == 0) {
    ra.rec->best_cost = (int32_t)(keys[0] >> 32);
    ra.rec->winner = (int32_t)winner;
    ra.rec->accepted = sums[0][0];
    ra.rec->uphill = sums[1][0];
    ra.rec->neutral = sums[2][0];
    ra.rec->infeasible = sums[3][0];
  }
  const int8_t *from = ra.xbest + winner * ra.P;
  for (int i = tid; i < ra.P; i += 256) ra.xwin[i] = from[i];
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------


int launch_eval(const DevProblem &pb, const int8_t *x, int64_t n, int32_t *cost, void *stream) {
  hipStream_t s = (hipStream_t)stream;
#define SA_CASE(M, K)                                                                         \
  case M:                                                                                     \
    if (pb.d == 1)                                                                            \
      eval_kernel<M, K, 1><<<grid_for(n), 256, 0, s>>>(pb, x, n, cost);                       \
    else                                                                                      \
      eval_kernel<M, K, 2><<<grid_for(n), 256, 0, s>>>(pb, x, n, cost);                       \
    break;
  switch (pb.nm) {
    SA_FOR_TILES(SA_CASE)
    default:
      return (int)hipErrorInvalidValue;
  }
#undef SA_CASE
  return (int)hipGetLastError();
}

int launch_simulate(const DevProblem &pb, const int8_t *x, int64_t n, int8_t *traj, void *stream) {
  hipStream_t s = (hipStream_t)stream;
#define SA_CASE(M, K)                                                                         \
  case M:                                                                                     \
    if (pb.d == 1)                                                                            \
      simulate_kernel<M, K, 1><<<grid_for(n), 256, 0, s>>>(pb, x, n, traj);                   \
    else                                                                                      \
      simulate_kernel<M, K, 2><<<grid_for(n), 256, 0, s>>>(pb, x, n, traj);                   \
    break;
  switch (pb.nm) {
    SA_FOR_TILES(SA_CASE)
    default:
      return (int)hipErrorInvalidValue;
  }
#undef SA_CASE
  return (int)hipGetLastError();
}

int launch_reduce(const ReduceArgs &ra, void *stream) {
  reduce_kernel<<<1, 256, 0, (hipStream_t)stream>>>(ra);
  return (int)hipGetLastError();
}

}  // namespace sa
