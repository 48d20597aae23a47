// sa_k_stage.hip -- one temperature stage of Table 1 for every chain of one
// network, in a register layout specialised to the network's tile counts.
// Method: Reimer et al., arXiv 2506.19866, Table 1 (one chain per wave).
#include "sa_chain.h"

namespace sa {

// LDS of a block: the observation tables shared by its chains, then one
// chain area per wave.
// HOLD: clamped nodes held by a select per dword; otherwise by accumulator
// offsets of the product (every clamp value 0 or 2, DevProblem::cofs).
template <int NM, int NK, int D, bool HOLD>
__global__ __launch_bounds__(256) void stage_kernel(DevProblem pb, StageArgs sa) {
  extern __shared__ uint32_t smem[];
  if (sa.stop && *sa.stop) return;  // the run was aborted at a stage boundary
  const int n_obs = obs_dwords(pb);
  uint32_t *lds_r = smem, *lds_w = smem + n_obs;
  for (int i = threadIdx.x; i < n_obs; i += blockDim.x) {
    lds_r[i] = pb.obs_r[i];
    lds_w[i] = pb.obs_w[i];
  }
  __syncthreads();

  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x >> 6;
  const int64_t chain = (int64_t)blockIdx.x * kWavesPerBlock + wv;
  if (chain >= sa.n_chains) return;
  ChainJob job;
  job.x_start = sa.x_start + (sa.group ? (chain / sa.group) * pb.P : chain * sa.x_start_stride);
  job.xbest = sa.xbest + chain * pb.P;
  job.cbest = sa.cbest + chain;
  job.stats = sa.cstats + chain * kStatWords;
  job.seed = sa.seed;
  job.chain = (uint64_t)chain;
  job.net = (uint64_t)sa.net;
  job.g0 = (uint64_t)sa.stage * (uint64_t)sa.L;
  job.L = sa.L;
  job.dcap = sa.dcap;
  job.tau = sa.tau;
  uint8_t *lds = reinterpret_cast<uint8_t *>(smem + 2 * n_obs) + (size_t)wv * chain_lds_bytes(pb);
  run_chain<NM, NK, D, false, NoHooks, HOLD>(pb, job, lane, lds, lds_r, lds_w);
}

size_t stage_smem_bytes(const DevProblem &pb, int waves_per_block) {
  return (size_t)2 * obs_dwords(pb) * 4 + (size_t)waves_per_block * chain_lds_bytes(pb);
}

int stage_waves_per_block(const DevProblem &) { return kWavesPerBlock; }

int launch_stage(const DevProblem &pb, const StageArgs &sa, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const size_t smem = stage_smem_bytes(pb, kWavesPerBlock);
#define SA_CASE(M, K)                                                                         \
  case M:                                                                                     \
    if (pb.hold_by_offset) {                                                                  \
      if (pb.d == 1)                                                                          \
        stage_kernel<M, K, 1, false><<<grid_for(sa.n_chains), 256, smem, s>>>(pb, sa);        \
      else                                                                                    \
        stage_kernel<M, K, 2, false><<<grid_for(sa.n_chains), 256, smem, s>>>(pb, sa);        \
    } else if (pb.d == 1) {                                                                   \
      stage_kernel<M, K, 1, true><<<grid_for(sa.n_chains), 256, smem, s>>>(pb, sa);           \
    } else {                                                                                  \
      stage_kernel<M, K, 2, true><<<grid_for(sa.n_chains), 256, smem, s>>>(pb, sa);           \
    }                                                                                         \
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
