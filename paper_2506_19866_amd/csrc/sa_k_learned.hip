// sa_k_learned.hip -- one temperature stage of Table 1 with the learned
// proposal (or with plain candidates and a trace of the steps with their
// features), for every chain of one network of up to 127 nodes.
// Method: Reimer et al., arXiv 2506.19866, Table 1; the proposal is an
// extension (sa_learned.h).
#include "sa_learned.h"

namespace sa {

// LDS of a block: the observation tables, the parameter descriptors, then
// one area per wave.
template <int NM, int NK, int D>
__global__ __launch_bounds__(256) void learned_stage_kernel(DevProblem pb, StageArgs sa, LearnedArgs la) {
  extern __shared__ uint32_t smem[];
  if (sa.stop && *sa.stop) return;  // the run was aborted at a stage boundary
  const int n_obs = obs_dwords(pb);
  uint32_t *lds_r = smem, *lds_w = smem + n_obs;
  uint32_t *cursor = smem + 2 * n_obs;
  const bool model = la.w1f != nullptr;
  // The network fragments (16.5 KB) stay in global memory, read through the
  // caches at refreshes only: kept out of LDS, a workgroup's LDS lets three
  // workgroups share a CU instead of two.
  uint32_t *s_pinfo = cursor;
  cursor += round4(pb.P);
  for (int i = threadIdx.x; i < n_obs; i += blockDim.x) {
    lds_r[i] = pb.obs_r[i];
    lds_w[i] = pb.obs_w[i];
  }
  for (int i = threadIdx.x; i < pb.P; i += blockDim.x) s_pinfo[i] = pb.param_info[i];
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
  uint8_t *lds = reinterpret_cast<uint8_t *>(cursor) + (size_t)wv * learned_wave_bytes(pb);

  LearnedHooks<NM, NK, D> hk;
  hk.pb = &pb;
  hk.la = la;
  hk.pinfo = s_pinfo;
  hk.w1f = static_cast<const uint4 *>(la.w1f);
  hk.w2f = static_cast<const uint4 *>(la.w2f);
  hk.xref = lds + chain_lds_bytes(pb);
  hk.tbl = reinterpret_cast<uint32_t *>(hk.xref + round4(pb.P));
  hk.msh = reinterpret_cast<float *>(hk.tbl + learned_tbl_words(pb));
  hk.eh = hk.msh + round4(pb.N);
  hk.ah = hk.eh + round4(pb.N);
  hk.fst = reinterpret_cast<uint4 *>(hk.ah + round4(pb.N));
  hk.b2 = model ? *la.b2 : 0.f;
  hk.mn = 0.f;
  hk.total = 0u;
  hk.trace = la.trace ? la.trace + chain * la.trace_cap : nullptr;
  run_chain<NM, NK, D, false>(pb, job, lane, lds, lds_r, lds_w, &hk);
}

size_t learned_smem_bytes(const DevProblem &pb, bool model) {
  (void)model;
  return (size_t)2 * obs_dwords(pb) * 4 +
         (size_t)4 * round4(pb.P) + (size_t)kWavesPerBlock * learned_wave_bytes(pb);
}

#define SA_LEARNED_TILES(X) X(1, 1) X(2, 1) X(3, 1) X(4, 1) X(5, 1) X(6, 1) X(7, 1) X(8, 1)

int learned_stage_prepare(const DevProblem &pb, size_t smem) {
  hipError_t e = hipErrorInvalidValue;
#define SA_CASE(M, K)                                                                                       \
  case M:                                                                                                   \
    e = pb.d == 1 ? hipFuncSetAttribute((const void *)learned_stage_kernel<M, K, 1>,                        \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem)              \
                  : hipFuncSetAttribute((const void *)learned_stage_kernel<M, K, 2>,                        \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);             \
    break;
  switch (pb.nm) {
    SA_LEARNED_TILES(SA_CASE)
    default:
      break;
  }
#undef SA_CASE
  return (int)e;
}

int launch_learned_stage(const DevProblem &pb, const StageArgs &sa, const LearnedArgs &la, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const size_t smem = learned_smem_bytes(pb, la.w1f != nullptr);
#define SA_CASE(M, K)                                                                          \
  case M:                                                                                      \
    if (pb.d == 1)                                                                             \
      learned_stage_kernel<M, K, 1><<<grid_for(sa.n_chains), 256, smem, s>>>(pb, sa, la);     \
    else                                                                                       \
      learned_stage_kernel<M, K, 2><<<grid_for(sa.n_chains), 256, smem, s>>>(pb, sa, la);     \
    break;
  switch (pb.nm) {
    SA_LEARNED_TILES(SA_CASE)
    default:
      return (int)hipErrorInvalidValue;
  }
#undef SA_CASE
  return (int)hipGetLastError();
}

}  // namespace sa
