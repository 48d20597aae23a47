// sa_k_batch.hip -- kernels over batches of vectors: cost (§2.3, §2.5.3) and
// trajectories (§2.2) of n parameter vectors, one wave per vector.
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


}  // namespace sa
