// sa_chain.h -- one chain's temperature stage (Table 1), run by one wavefront:
// steps_per_stage steps of GetCandidate -> Simulate -> score -> Metropolis,
// entirely on chip.  Shared by the single-network stage kernel and the
// persistent kernel over many networks.  Constraints are enforced when the
// candidate is drawn (§2.5.3).
#pragma once
#include "sa_device.h"

namespace sa {

// LDS of one chain: x_current [P4], x_best [P4] bytes and the per-node counts
// of non-zero out-edges [N4] and +1 in-edges [N4].
__host__ __device__ inline int chain_lds_bytes(const DevProblem &pb) { return 2 * round4(pb.P) + 2 * round4(pb.N); }
// Shared observation tables of a block (reference bytes, weights).
__host__ __device__ inline int obs_dwords(const DevProblem &pb) { return pb.CG * pb.K * pb.nd * kWave; }

struct ChainJob {
  const int8_t *x_start;  // start vector [P]
  int8_t *xbest;          // best vector out [P]
  int32_t *cbest;         // best cost out
  uint32_t *stats;        // out: kStatWords statistics
  uint64_t seed;
  uint64_t chain;         // Philox chain id (within its network)
  uint64_t net;           // Philox network id
  uint64_t g0;            // global index of the stage's first step: stage * L
  int32_t L;
  int32_t dcap;
  const uint32_t *tau;    // thresholds of this stage, [dcap + 1]
};

// Hooks of the learned proposal (see sa_learned.h).  The plain method passes
// NoHooks, whose calls compile away.
//   refresh(A, it, ...)   before step it: rebuild the proposal table
//   select(...)           pick the candidate from the table, or decline
//   record(...)           after the decision, before the chain moves
// Sources of a candidate: 0 plain draw, 1 table, 2 plain because the table's
// move repeats the current value, 3 plain because the table is empty.
struct NoHooks {
  static constexpr bool kEnabled = false;
};

template <int NM, int NK, int D, bool RT, class Hooks = NoHooks, bool HOLD = true>
__device__ __forceinline__ void run_chain(const DevProblem &pb, const ChainJob &job, int lane, uint8_t *lds,
                                          const uint32_t *lds_r, const uint32_t *lds_w, Hooks *hk = nullptr) {
  const int P = pb.P, E = pb.E;
  const int P4 = round4(P), N4 = round4(pb.N);
  uint8_t *xcur = lds;
  uint8_t *xbst = xcur + P4;
  uint8_t *outnz = xbst + P4;
  uint8_t *inplus = outnz + N4;

  for (int i = lane; i < P; i += kWave) xcur[i] = xbst[i] = (uint8_t)job.x_start[i];
  wave_sync();
  auto xv = [xcur](int p) -> int { return (int)(int8_t)xcur[p]; };
  int vcur = uniform(wave_sum(lane_violations(pb, lane, xv, outnz, inplus)));
  SA_DECLARE_A(A, NM, NK);
  build_a(A, pb, lane, xv);
  // Table 1: every stage starts by scoring the vector it restarts from
  int ccur = uniform(wave_sum(lane_mismatch<NM, NK, D, false, RT, HOLD>(A, pb, lane, lds_r, lds_w, nullptr))) +
             pb.lambda * vcur;
  int cbest = ccur;
  uint32_t n_acc = 0, n_up = 0, n_neu = 0, n_inf = 0;
  wave_sync();

  for (int it0 = 0; it0 < job.L; it0 += kWave) {
    // one Philox block per step: lane j draws the block of step it0 + j
    const Draw dr = philox_top_words(job.g0 + (uint64_t)(it0 + lane), job.chain, job.net, 0ull, job.seed, 0ull);
    const int nsteps = min(kWave, job.L - it0);
    for (int j = 0; j < nsteps; ++j) {
      const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)dr.w0, j);
      const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)dr.w1, j);
      const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)dr.w2, j);
      int p, nv, source = 0;
      bool chosen = false;
      if constexpr (Hooks::kEnabled) {
        hk->refresh(A, it0 + j, xcur, outnz, inplus, ccur, vcur, lane, lds_r, lds_w);
        const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)dr.w3, j);
        chosen = hk->select(r0, r3, xcur, p, nv, source, lane);
      }
      if (!chosen) {
        // GetCandidate (Table 1): uniform index, one of the two other values
        p = (int)(((uint64_t)r0 * (uint64_t)P) >> 32);
        const int cur = uniform((int)(int8_t)xcur[p]);
        const int ncode = ((p < E ? cur + 1 : cur) + 1 + (int)(r1 >> 31)) % 3;
        nv = p < E ? ncode - 1 : ncode;
      }
      const int old = uniform((int)(int8_t)xcur[p]);
      const bool is_edge = p < E;
      // structural constraints (§2.5.3) from the per-node counts
      int vc = vcur, src = 0, dst = 0, on_new = 0, ip_new = 0;
      if (is_edge) {
        src = load_uniform(pb.edge_src, p);
        dst = load_uniform(pb.edge_dst, p);
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
      param_patch_args<NK>(pb, lane, p, nv, reg, mask, bits_new);
      reg = uniform(reg);
      if (!feasible) mask = 0u;
      patch_a(A, reg, mask, bits_new);
      int ccand = 0;
      if (feasible)
        ccand = uniform(wave_sum(lane_mismatch<NM, NK, D, false, RT, HOLD>(A, pb, lane, lds_r, lds_w, nullptr))) +
                pb.lambda * vc;
      const int delta = ccand - ccur;
      // Metropolis in fixed point: accept iff delta <= 0 or u32 < tau[delta]
      const bool accept = feasible && (delta <= 0 || (delta <= job.dcap && r2 < load_uniform(job.tau, delta)));
      patch_a(A, reg, accept ? 0u : mask, param_bits(p, E, old));
      if constexpr (Hooks::kEnabled)
        hk->record(job.g0 + (uint64_t)(it0 + j), p, old, nv, feasible, delta, accept, source, outnz, inplus, lane);
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
  for (int i = lane; i < P; i += kWave) job.xbest[i] = (int8_t)xbst[i];
  if (lane == 0) {
    *job.cbest = cbest;
    job.stats[0] = n_acc;
    job.stats[1] = n_up;
    job.stats[2] = n_neu;
    job.stats[3] = n_inf;
    job.stats[4] = 1u + (uint32_t)job.L - n_inf;  // every feasible candidate is simulated
  }
}

}  // namespace sa
