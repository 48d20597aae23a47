// sa_k_persist.hip -- many networks of uneven size in persistent launches
// per temperature stage (Table 1 for every network), and the per-network
// stage reduction.  Networks are grouped into size classes; a class runs in
// its largest register layout with each network's own tile counts as runtime
// bounds, so small networks keep small register footprints (and high
// occupancy) while one kernel serves every size within a class.
#include "sa_chain.h"

namespace sa {

template <int MX, int KX, int D>
__global__ __launch_bounds__(512) void persistent_kernel(BatchArgs a) {
  extern __shared__ uint32_t smem[];
  __shared__ int s_item;
  if (a.stop && *a.stop) return;  // the run was aborted at a stage boundary
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) s_item = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    const int item = s_item;
    __syncthreads();  // every wave has read the item before the next fetch
    if (item >= a.n_items) break;
    const int net = a.item_net[item];
    const DevProblem pb = a.probs[net];  // every item of this launch has step size D
    const int n_obs = obs_dwords(pb);
    uint32_t *lds_r = smem, *lds_w = smem + n_obs;
    for (int i = threadIdx.x; i < n_obs; i += blockDim.x) {
      lds_r[i] = pb.obs_r[i];
      lds_w[i] = pb.obs_w[i];
    }
    __syncthreads();
    const int64_t chain = (int64_t)a.item_chain0[item] + wv;
    if (wv < a.waves && chain < a.n_chains) {
      const int64_t gc = (int64_t)net * a.n_chains + chain;
      ChainJob job;
      job.x_start = a.first ? a.x_start + a.x_off[net] + chain * pb.P
                            : a.x_start + a.w_off[net] + (a.group ? chain / a.group : 0) * pb.P;
      job.xbest = a.xbest + a.x_off[net] + chain * pb.P;
      job.cbest = a.cbest + gc;
      job.stats = a.cstats + gc * kStatWords;
      job.seed = a.seed;
      job.chain = (uint64_t)chain;
      job.net = (uint64_t)net;
      job.g0 = (uint64_t)a.stage * (uint64_t)a.L;
      job.L = a.L;
      job.dcap = a.dcap;
      job.tau = a.tau;
      uint8_t *lds = reinterpret_cast<uint8_t *>(smem + 2 * n_obs) + (size_t)wv * chain_lds_bytes(pb);
      run_chain<MX, KX, D, true>(pb, job, lane, lds, lds_r, lds_w);
    }
    __syncthreads();  // the block's LDS is reused by the next item
  }
}

__global__ __launch_bounds__(256) void batch_reduce_kernel(BatchReduceArgs ra) {
  __shared__ unsigned long long keys[256];
  __shared__ unsigned long long sums[kStatWords][256];
  if (ra.ctl && ra.ctl[0]) return;  // the run was aborted at a stage boundary
  const int tid = threadIdx.x;
  const int net = blockIdx.x;
  const int64_t base = (int64_t)net * ra.n_chains;
  unsigned long long best = ~0ull;
  unsigned long long acc[kStatWords] = {};
  for (int64_t c = tid; c < ra.n_chains; c += 256) {
    const unsigned long long key = ((unsigned long long)(uint32_t)ra.cbest[base + c] << 32) | (unsigned long long)c;
    best = key < best ? key : best;
    const uint32_t *st = ra.cstats + (base + c) * kStatWords;
#pragma unroll
    for (int q = 0; q < kStatWords; ++q) acc[q] += st[q];
  }
  keys[tid] = best;
#pragma unroll
  for (int q = 0; q < kStatWords; ++q) sums[q][tid] = acc[q];
  __syncthreads();
  for (int half = 128; half > 0; half >>= 1) {
    if (tid < half) {
      const unsigned long long o = keys[tid + half];
      keys[tid] = o < keys[tid] ? o : keys[tid];
#pragma unroll
      for (int q = 0; q < kStatWords; ++q) sums[q][tid] += sums[q][tid + half];
    }
    __syncthreads();
  }
  const int64_t winner = (int64_t)(keys[0] & 0xffffffffull);
  if (tid == 0) {
    StageRecord *r = ra.rec + net;
    r->best_cost = (int32_t)(keys[0] >> 32);
    r->winner = (int32_t)winner;
    r->accepted = sums[0][0];
    r->uphill = sums[1][0];
    r->neutral = sums[2][0];
    r->infeasible = sums[3][0];
    r->simulated = sums[4][0];
    if (net == 0 && ra.queue)  // one work counter per (size class, step size) launch
      for (int q = 0; q < kPersistentQueues; ++q) ra.queue[q] = 0u;
    if (net == 0 && ra.ctl) ra.ctl[1] = (uint32_t)(ra.st + 1);
  }
  if (ra.group) return;  // every restart group copies its own winner (group_restart_kernel)
  const int P = ra.probs[net].P;
  const int8_t *from = ra.xbest + ra.x_off[net] + winner * P;
  int8_t *to = ra.xwin + ra.w_off[net];
  for (int i = tid; i < P; i += 256) to[i] = from[i];
}

// Island restart: one wavefront per restart group of ra.group consecutive
// chains (the last group of a network may be shorter): the group's best
// chain (lowest chain id on ties) is copied to the group's winner slot, from
// which every chain of the group starts the next stage.
__global__ __launch_bounds__(256) void group_restart_kernel(BatchReduceArgs ra, int64_t groups_per_net) {
  if (ra.ctl && ra.ctl[0]) return;  // the run was aborted at a stage boundary
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t gid = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (gid >= (int64_t)ra.n_probs * groups_per_net) return;
  const int net = (int)(gid / groups_per_net);
  const int64_t g = gid % groups_per_net;
  const int64_t c0 = g * ra.group, c1 = min(c0 + ra.group, ra.n_chains);
  const int64_t base = (int64_t)net * ra.n_chains;
  unsigned long long best = ~0ull;
  for (int64_t c = c0 + lane; c < c1; c += kWave) {
    const unsigned long long key = ((unsigned long long)(uint32_t)ra.cbest[base + c] << 32) | (unsigned long long)c;
    best = key < best ? key : best;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(best, off, kWave);
    best = o < best ? o : best;
  }
  const int64_t winner = (int64_t)(best & 0xffffffffull);
  const int P = ra.probs[net].P;
  const int8_t *from = ra.xbest + ra.x_off[net] + winner * P;
  int8_t *to = ra.xwin + ra.w_off[net] + g * P;
  for (int i = lane; i < P; i += kWave) to[i] = from[i];
}

__global__ void abort_gate_kernel(const volatile int32_t *flag, uint32_t *ctl) {
  if (threadIdx.x != 0) return;
  const int32_t f = __hip_atomic_load(const_cast<const int32_t *>(flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  if (f != 0) ctl[0] = 1u;
}

size_t persistent_smem_bytes(const DevProblem &pb, int waves) {
  return (size_t)2 * obs_dwords(pb) * 4 + (size_t)waves * chain_lds_bytes(pb);
}

// size classes: (m-tiles, k-tiles) of the layout each class runs in
#define SA_PERSISTENT_CLASSES(X) X(0, 4, 1) X(1, 8, 1) X(2, 10, 2)

// The class of a network with nm m-tiles; every network of a class has the
// class's k-fragments, and its m-tile count lies between rt_min_tiles of the
// class layout and the layout's own, which the time-step variants cover.
int persistent_class(int nm) { return nm <= 4 ? 0 : nm <= 8 ? 1 : 2; }
static_assert(rt_min_tiles(4) == 1 && rt_min_tiles(8) == 5 && rt_min_tiles(10) == 9,
              "size classes and time-step variants agree");

int persistent_blocks_per_cu(int cls, int waves, size_t smem) {
  int blocks = 0;
  hipError_t e = hipErrorInvalidValue;
#define SA_CASE(C, M, K) \
  case C:                \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, persistent_kernel<M, K, 1>, 64 * waves, smem); \
    break;
  switch (cls) {
    SA_PERSISTENT_CLASSES(SA_CASE)
    default:
      break;
  }
#undef SA_CASE
  if (e != hipSuccess) return 1;
  return blocks > 0 ? blocks : 1;
}

int launch_persistent(const BatchArgs &a, int cls, int d, int grid, size_t smem, void *stream) {
  hipStream_t s = (hipStream_t)stream;
#define SA_CASE(C, M, K)                                                    \
  case C:                                                                   \
    if (d == 1)                                                             \
      persistent_kernel<M, K, 1><<<grid, 64 * a.waves, smem, s>>>(a);       \
    else                                                                    \
      persistent_kernel<M, K, 2><<<grid, 64 * a.waves, smem, s>>>(a);       \
    break;
  switch (cls) {
    SA_PERSISTENT_CLASSES(SA_CASE)
    default:
      return (int)hipErrorInvalidValue;
  }
#undef SA_CASE
  return (int)hipGetLastError();
}

int launch_abort_gate(const volatile int32_t *flag, uint32_t *ctl, void *stream) {
  abort_gate_kernel<<<1, 64, 0, (hipStream_t)stream>>>(flag, ctl);
  return (int)hipGetLastError();
}

int launch_batch_reduce(const BatchReduceArgs &ra, void *stream) {
  batch_reduce_kernel<<<ra.n_probs, 256, 0, (hipStream_t)stream>>>(ra);
  if (ra.group > 0) {
    const int64_t groups_per_net = (ra.n_chains + ra.group - 1) / ra.group;
    group_restart_kernel<<<grid_for((int64_t)ra.n_probs * groups_per_net), 256, 0, (hipStream_t)stream>>>(
        ra, groups_per_net);
  }
  return (int)hipGetLastError();
}

}  // namespace sa
