// sa_k_stage.hip -- one temperature stage of Table 1 for every chain: each
// wavefront runs steps_per_stage steps of GetCandidate -> Simulate -> score ->
// Metropolis for its chain, entirely on chip.  Method: Reimer et al., arXiv
// 2506.19866, Table 1; constraints enforced when the candidate is drawn
// (§2.5.3).
#include "sa_device.h"

namespace sa {

// LDS of a block: the observation tables (reference bytes, weights) shared by
// its chains, then per wave: x_current [P4], x_best [P4] bytes and the
// per-node counts of non-zero out-edges [N4] and +1 in-edges [N4].
static inline __host__ __device__ int obs_dwords(const DevProblem &pb) { return pb.CG * pb.K * pb.nd * kWave; }
static inline __host__ __device__ int wave_bytes(const DevProblem &pb) { return 2 * round4(pb.P) + 2 * round4(pb.N); }

template <int NM, int NK, int D>
__global__ __launch_bounds__(256) void stage_kernel(DevProblem pb, StageArgs sa) {
  extern __shared__ uint32_t smem[];
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
  const int P = pb.P, E = pb.E;
  const int P4 = round4(P), N4 = round4(pb.N);
  uint8_t *xcur = reinterpret_cast<uint8_t *>(smem + 2 * n_obs) + (size_t)wv * wave_bytes(pb);
  uint8_t *xbst = xcur + P4;
  uint8_t *outnz = xbst + P4;
  uint8_t *inplus = outnz + N4;

  const int8_t *xs = sa.x_start + chain * sa.x_start_stride;
  for (int i = lane; i < P; i += kWave) xcur[i] = xbst[i] = (uint8_t)xs[i];
  wave_sync();
  auto xv = [xcur](int p) -> int { return (int)(int8_t)xcur[p]; };
  int vcur = uniform(wave_sum(lane_violations(pb, lane, xv, outnz, inplus)));
  SA_DECLARE_A(A, NM, NK);
  build_a(A, pb, lane, xv);
  // Table 1: every stage starts by scoring the vector it restarts from
  int ccur = uniform(wave_sum(lane_mismatch<NM, NK, D, false>(A, pb, lane, lds_r, lds_w, nullptr))) +
             pb.lambda * vcur;
  int cbest = ccur;
  uint32_t n_acc = 0, n_up = 0, n_neu = 0, n_inf = 0;
  wave_sync();

  const uint64_t g0 = (uint64_t)sa.stage * (uint64_t)sa.L;
  for (int it0 = 0; it0 < sa.L; it0 += kWave) {
    // one Philox block per step: lane j draws the block of step it0 + j
    const Draw dr = philox_top_words(g0 + (uint64_t)(it0 + lane), (uint64_t)chain, (uint64_t)sa.net, 0ull,
                                     sa.seed, 0ull);
    const int nsteps = min(kWave, sa.L - it0);
    for (int j = 0; j < nsteps; ++j) {
      const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)dr.w0, j);
      const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)dr.w1, j);
      const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)dr.w2, j);
      // GetCandidate (Table 1): uniform index, one of the two other values
      const int p = (int)(((uint64_t)r0 * (uint64_t)P) >> 32);
      const int old = uniform((int)(int8_t)xcur[p]);
      const bool is_edge = p < E;
      const int code = is_edge ? old + 1 : old;
      const int ncode = (code + 1 + (int)(r1 >> 31)) % 3;
      const int nv = is_edge ? ncode - 1 : ncode;
      // structural constraints (§2.5.3) from the per-node counts
      int vc = vcur, src = 0, dst = 0, on_new = 0, ip_new = 0;
      if (is_edge) {
        src = pb.edge_src[p];
        dst = pb.edge_dst[p];
        const int on = uniform((int)outnz[src]), ip = uniform((int)inplus[dst]);
        on_new = on + (nv != 0) - (old != 0);
        ip_new = ip + (nv == 1) - (old == 1);
        vc += (on_new == 0) - (on == 0) + (ip_new == 0) - (ip == 0);
      }
      // The candidate is written into A, scored, and written back unless it
      // is accepted.  Both writes happen on every step (with a zero mask where
      // they do not apply) so that A is updated in straight-line code.
      const bool feasible = !(pb.hard && vc > 0);
      int reg;
      uint32_t mask, bits_new;
      param_patch_args(pb, lane, p, nv, reg, mask, bits_new);
      reg = uniform(reg);
      if (!feasible) mask = 0u;
      patch_a(A, reg, mask, bits_new);
      int ccand = 0;
      if (feasible)
        ccand = uniform(wave_sum(lane_mismatch<NM, NK, D, false>(A, pb, lane, lds_r, lds_w, nullptr))) +
                pb.lambda * vc;
      const int delta = ccand - ccur;
      // Metropolis in fixed point: accept iff delta <= 0 or u32 < tau[delta]
      const bool accept = feasible && (delta <= 0 || (delta <= sa.dcap && r2 < sa.tau[delta]));
      patch_a(A, reg, accept ? 0u : mask, ((uint32_t)(is_edge ? old : -old) & 0xffu) * kLowBits);
      if (!feasible) {
        ++n_inf;  // infeasible candidate (§2.5.3): a rejected step, no redraw
      } else if (accept) {
        ++n_acc;
        n_up += delta > 0;
        n_neu += delta == 0;
        xcur[p] = (uint8_t)nv;
        if (is_edge) {
          outnz[src] = (uint8_t)on_new;
          inplus[dst] = (uint8_t)ip_new;
        }
        vcur = vc;
        ccur = ccand;
        if (ccand < cbest) {  // strict improvement of the chain's best
          cbest = ccand;
          wave_sync();
          const uint32_t *from = reinterpret_cast<const uint32_t *>(xcur);
          uint32_t *to = reinterpret_cast<uint32_t *>(xbst);
          for (int i = lane; i < P4 / 4; i += kWave) to[i] = from[i];
        }
        wave_sync();
      }
    }
  }
  wave_sync();
  int8_t *xo = sa.xbest + chain * P;
  for (int i = lane; i < P; i += kWave) xo[i] = (int8_t)xbst[i];
  if (lane == 0) {
    sa.cbest[chain] = cbest;
    uint32_t *st = sa.cstats + chain * 4;
    st[0] = n_acc;
    st[1] = n_up;
    st[2] = n_neu;
    st[3] = n_inf;
  }
}

size_t stage_smem_bytes(const DevProblem &pb, int waves_per_block) {
  return (size_t)2 * obs_dwords(pb) * 4 + (size_t)waves_per_block * wave_bytes(pb);
}

int stage_waves_per_block(const DevProblem &) { return kWavesPerBlock; }

int launch_stage(const DevProblem &pb, const StageArgs &sa, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const size_t smem = stage_smem_bytes(pb, kWavesPerBlock);
#define SA_CASE(M, K)                                                                         \
  case M:                                                                                     \
    if (pb.d == 1)                                                                            \
      stage_kernel<M, K, 1><<<grid_for(sa.n_chains), 256, smem, s>>>(pb, sa);                 \
    else                                                                                      \
      stage_kernel<M, K, 2><<<grid_for(sa.n_chains), 256, smem, s>>>(pb, sa);                 \
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
