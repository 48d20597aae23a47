// sa_k_priority.hip -- the paper's own model (priority update, P = 3E + 3N):
// cost and trajectories of a batch of vectors, and one temperature stage of
// Table 1 for every chain, 64 / LC chains per wavefront (see sa_priority.h).
// Method: Reimer et al., arXiv 2506.19866, §2.1-§2.3, §2.5.3, Table 1.
#include "sa_priority.h"

namespace sa {

namespace {

constexpr int kBlock = 256;

// Segment of this lane: (first lane, lane within the segment, index of the
// segment's chain or vector in the launch).
template <int LC>
struct SegPos {
  int base, li;
  int64_t index;
  __device__ SegPos() {
    const int lane = threadIdx.x & (kWave - 1);
    base = lane & ~(LC - 1);
    li = lane & (LC - 1);
    index = ((int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6)) * (kWave / LC) + lane / LC;
  }
};

template <int LC, int DMAX>
__global__ __launch_bounds__(kBlock) void pr_eval_kernel(DevProblem pb, const int8_t *__restrict__ x, int64_t n,
                                                         int32_t *__restrict__ cost) {
  const SegPos<LC> sp;
  // the whole wave takes part in every ballot and reduction; a segment past
  // the last vector evaluates vector n - 1 and writes nothing
  if (__builtin_amdgcn_readfirstlane((int)(sp.index - sp.index % (kWave / LC) >= n))) return;
  const bool valid = sp.index < n;
  const int8_t *xi = x + (valid ? sp.index : n - 1) * pb.P;
  auto xv = [xi](int k) -> int { return xi[k]; };
  PrNode<LC, DMAX> nd;
  PrAddr<DMAX> ad;
  pr_build<LC, DMAX>(pb, sp.li, sp.base, xv, nd, ad);
  const int mis = seg_sum<LC>(pr_mismatch<LC, DMAX, false>(pb, sp.li, sp.base, nd, ad, pb.pr_start, pb.pr_obs,
                                                           nullptr));
  const int v = pr_violations<LC, DMAX>(pb, sp.li, nd);
  if (valid && sp.li == 0) cost[sp.index] = mis + pb.lambda * v;
}

template <int LC, int DMAX>
__global__ __launch_bounds__(kBlock) void pr_simulate_kernel(DevProblem pb, const int8_t *__restrict__ x, int64_t n,
                                                             int8_t *__restrict__ traj) {
  const SegPos<LC> sp;
  if (__builtin_amdgcn_readfirstlane((int)(sp.index - sp.index % (kWave / LC) >= n))) return;
  const bool valid = sp.index < n;
  const int64_t i = valid ? sp.index : n - 1;
  const int8_t *xi = x + i * pb.P;
  auto xv = [xi](int k) -> int { return xi[k]; };
  PrNode<LC, DMAX> nd;
  PrAddr<DMAX> ad;
  pr_build<LC, DMAX>(pb, sp.li, sp.base, xv, nd, ad);
  // a segment past the last vector still takes part in the lane exchanges,
  // with its stores switched off
  pr_mismatch<LC, DMAX, true>(pb, sp.li, sp.base, nd, ad, pb.pr_start, pb.pr_obs,
                              valid ? traj + (size_t)i * pb.C * (pb.T + 1) * pb.N : nullptr);
}

// LDS of a chain: x_current and x_best, P rounded up to 4 bytes each.
__host__ __device__ inline int pr_chain_bytes(const DevProblem &pb) { return 2 * round4(pb.P); }
__host__ __device__ inline int pr_table_bytes(const DevProblem &pb) {
  return round4(pb.C * pb.lc) + 4 * pb.C * (pb.T + 1) * pb.lc;
}

// One temperature stage: per chain L steps of GetCandidate -> Simulate ->
// score -> Metropolis (Table 1), with the priority model's domains.
template <int LC, int DMAX>
__global__ __launch_bounds__(kBlock) void pr_stage_kernel(DevProblem pb, StageArgs sa) {
  extern __shared__ uint32_t smem[];
  if (sa.stop && *sa.stop) return;  // the run was aborted at a stage boundary
  const int tb = pr_table_bytes(pb);
  uint8_t *lstart = reinterpret_cast<uint8_t *>(smem);
  uint32_t *lobs = reinterpret_cast<uint32_t *>(lstart + round4(pb.C * LC));
  {
    const uint32_t *gs = reinterpret_cast<const uint32_t *>(pb.pr_start);
    uint32_t *ls = reinterpret_cast<uint32_t *>(lstart);
    for (int i = threadIdx.x; i < pb.C * LC / 4; i += kBlock) ls[i] = gs[i];
    for (int i = threadIdx.x; i < pb.C * (pb.T + 1) * LC; i += kBlock) lobs[i] = pb.pr_obs[i];
  }
  __syncthreads();

  const SegPos<LC> sp;
  const int base = sp.base, li = sp.li;
  const int64_t n = sa.n_chains;
  if (__builtin_amdgcn_readfirstlane((int)(sp.index - sp.index % (kWave / LC) >= n))) return;
  const bool valid = sp.index < n;
  const int64_t chain = valid ? sp.index : n - 1;
  const int P = pb.P, E = pb.E, N = pb.N, P4 = round4(P);
  const int seg_in_block = (threadIdx.x >> 6) * (kWave / LC) + (threadIdx.x & (kWave - 1)) / LC;
  uint8_t *xcur = reinterpret_cast<uint8_t *>(smem) + tb + (size_t)seg_in_block * pr_chain_bytes(pb);
  uint8_t *xbst = xcur + P4;

  const int8_t *xs = sa.x_start + (sa.group ? (chain / sa.group) * P : chain * sa.x_start_stride);
  for (int k = li; k < P; k += LC) xcur[k] = xbst[k] = (uint8_t)xs[k];
  wave_sync();
  auto xv = [xcur](int k) -> int { return (int)(int8_t)xcur[k]; };
  PrNode<LC, DMAX> nd;
  PrAddr<DMAX> ad;
  pr_build<LC, DMAX>(pb, li, base, xv, nd, ad);
  int vcur = pr_violations<LC, DMAX>(pb, li, nd);
  // What this lane's node did in the current trajectory (kPrTold, ...),
  // recorded only where a wave holds one chain: with several chains per wave
  // a simulation is skipped only when all of them can skip it, which rarely
  // pays for the bookkeeping in every time step.
  constexpr bool kTrackActs = LC == 64;
  uint32_t acur = kPrTold | kPrReady | kPrFar | kPrVisited;
  // The range of this lane's node's image over the current trajectory (one
  // chain per wave), widened by [lo, hi] when a candidate that moved it
  // within saturation is accepted without a simulation, and recomputed by
  // every simulation that is accepted.
  PrImageRange rcur;
  rcur.lo = -kPrNoImage;
  rcur.hi = kPrNoImage;
  // Table 1: every stage starts by scoring the vector it restarts from
  int mcur = seg_sum<LC>(pr_mismatch<LC, DMAX, false>(pb, li, base, nd, ad, lstart, lobs, nullptr,
                                                      kTrackActs ? &acur : nullptr, kTrackActs ? &rcur : nullptr));
  int ccur = mcur + pb.lambda * vcur;
  int cbest = ccur;
  uint32_t n_acc = 0, n_up = 0, n_neu = 0, n_inf = 0, n_sim = 1;

  for (int it0 = 0; it0 < sa.L; it0 += LC) {
    // one Philox block per step: lane i of the segment draws step it0 + i
    const Draw dr = philox_top_words((uint64_t)sa.stage * (uint64_t)sa.L + (uint64_t)(it0 + li), (uint64_t)chain,
                                     (uint64_t)sa.net, 0ull, sa.seed, 0ull);
    const int nsteps = min(LC, sa.L - it0);
    for (int j = 0; j < nsteps; ++j) {
      const uint32_t r0 = seg_bcast<LC>(dr.w0, base, j);
      const uint32_t r1 = seg_bcast<LC>(dr.w1, base, j);
      const uint32_t r2 = seg_bcast<LC>(dr.w2, base, j);
      // GetCandidate: uniform element, one of the other values of its domain
      const int p = (int)(((uint64_t)r0 * (uint64_t)P) >> 32);
      const int blk = pr_block(p, E, N);
      const int ksz = pr_domain_size(blk);
      const int old = (int)(int8_t)xcur[p];
      int nc = pr_code(blk, old) + 1 + (int)(((uint64_t)r1 * (uint64_t)(ksz - 1)) >> 32);
      if (nc >= ksz) nc -= ksz;
      const int nv = pr_value(blk, nc);
      // The candidate is applied to the lane of the changed node in place and
      // undone below unless it is accepted (xcur keeps the current values).
      const int e = blk < 3 ? p - blk * E : 0;
      const int target = blk < 3 ? pb.edge_dst[e] : p - 3 * E - (blk - 3) * N;
      const bool mine = li == target;
      int slot = 0, src = 0, w0 = 0, p0 = 0, t0 = 0;
      bool moves = false;  // this lane's node can behave differently under the candidate
      int dlo = 0, dhi = 0;  // change of the node's image where it changes within saturation
      if (blk < 3) {
        slot = e - pb.in_ptr[target];
        src = pb.edge_src[e];
        // states the source took in the current trajectory (one chain per
        // wave: src is the same in every lane)
        uint32_t seen = kPrVisited;
        if constexpr (kTrackActs) seen = (uint32_t)__builtin_amdgcn_readlane((int)acur, uniform(src));
        if (mine) {
          w0 = xv(e);
          p0 = xv(E + e);
          t0 = xv(2 * E + e);
          const int w = blk == 0 ? nv : w0, pol = blk == 1 ? nv : p0, t = blk == 2 ? nv : t0;
          pr_set_edge<LC, DMAX>(nd, slot, src, w, pol, t);
          // an edge whose contribution (s div t) * w * p stays the same for
          // every state its source takes (w or p zero before and after, or a
          // source that never leaves 0) leaves every image unchanged
          const uint32_t tn = pr_edge_table(w, pol, t), to = pr_edge_table(w0, p0, t0), diff = tn ^ to;
          const bool at1 = (diff & 0x0000ff00u) && (seen & 0x00000100u);
          const bool at2 = (diff & 0x00ff0000u) && (seen & 0x00010000u);
          moves = at1 || at2;
          if (kTrackActs && moves) {
            // the image changes by d1 where the source is 1 and d2 where it
            // is 2; if it stays saturated at every step where the node is
            // free, no goal changes
            const int d1 = at1 ? (int)(int8_t)(tn >> 8) - (int)(int8_t)(to >> 8) : 0;
            const int d2 = at2 ? (int)(int8_t)(tn >> 16) - (int)(int8_t)(to >> 16) : 0;
            const int lo = min(0, min(d1, d2)), hi = max(0, max(d1, d2));
            if (rcur.lo + lo >= 2 || rcur.hi + hi <= 0) {
              moves = false;
              dlo = lo;
              dhi = hi;
            }
          }
        }
      } else if (mine) {
        // a node never eligible ignores its speed, one never told its memory
        // (and speed and step size), one never two levels from a goal it
        // moved to its step size
        if (blk == 3) nd.u = nv;
        if (blk == 4) nd.mem = nv;
        if (blk == 5) nd.d = nv;
        moves = (acur & (blk == 3 ? kPrReady : blk == 4 ? kPrTold : kPrFar)) != 0;
      }
      // the trajectory, and so the mismatch, is the current one unless some
      // node of the segment can behave differently
      const bool same_traj = seg_ballot<LC>(moves, base) == 0;
      // V changes only with a weight or a polarity; the reduction runs in
      // wave-uniform control flow
      int vc = vcur;
      if (__builtin_amdgcn_ballot_w64(blk < 2) != 0) {
        const int vnew = pr_violations<LC, DMAX>(pb, li, nd);
        if (blk < 2) vc = vnew;
      }
      const bool feasible = !(pb.hard && vc > 0);
      int mcand = mcur;
      uint32_t acand = acur;
      PrImageRange rcand = rcur;
      if (same_traj) {
        rcand.lo += dlo;
        rcand.hi += dhi;
      }
      if (__builtin_amdgcn_ballot_w64(feasible && !same_traj) != 0) {
        uint32_t a = acur;
        PrImageRange r = rcur;
        const int m = seg_sum<LC>(pr_mismatch<LC, DMAX, false>(pb, li, base, nd, ad, lstart, lobs, nullptr,
                                                               kTrackActs ? &a : nullptr, kTrackActs ? &r : nullptr));
        if (!same_traj) {
          mcand = m;
          acand = a;
          rcand = r;
        }
      }
      n_sim += feasible && !same_traj;
      const int ccand = feasible ? mcand + pb.lambda * vc : 0;
      const int delta = ccand - ccur;
      // Metropolis in fixed point: accept iff delta <= 0 or u32 < tau[delta]
      const bool accept =
          feasible && (delta <= 0 || (delta <= sa.dcap && r2 < sa.tau[min(max(delta, 0), sa.dcap)]));
      if (!feasible) {
        ++n_inf;  // infeasible candidate (§2.5.3): a rejected step, no redraw
      } else if (accept) {
        ++n_acc;
        n_up += delta > 0;
        n_neu += delta == 0;
        vcur = vc;
        mcur = mcand;
        acur = acand;
        rcur = rcand;
        ccur = ccand;
      }
      if (!accept && mine) {  // back to the current parameters
        if (blk < 3)
          pr_set_edge<LC, DMAX>(nd, slot, src, w0, p0, t0);
        else if (blk == 3)
          nd.u = old;
        else if (blk == 4)
          nd.mem = old;
        else
          nd.d = old;
      }
      wave_sync();
      if (accept && li == 0) xcur[p] = (uint8_t)nv;
      wave_sync();
      const bool improved = accept && ccand < cbest;  // strict improvement of the chain's best
      if (improved) cbest = ccand;
      if (__builtin_amdgcn_ballot_w64(improved) != 0) {
        const uint32_t *from = reinterpret_cast<const uint32_t *>(xcur);
        uint32_t *to = reinterpret_cast<uint32_t *>(xbst);
        if (improved)
          for (int k = li; k < P4 / 4; k += LC) to[k] = from[k];
        wave_sync();
      }
    }
  }
  wave_sync();
  if (valid) {
    int8_t *xb = sa.xbest + chain * P;
    for (int k = li; k < P; k += LC) xb[k] = (int8_t)xbst[k];
    if (li == 0) {
      sa.cbest[chain] = cbest;
      uint32_t *st = sa.cstats + chain * kStatWords;
      st[0] = n_acc;
      st[1] = n_up;
      st[2] = n_neu;
      st[3] = n_inf;
      st[4] = n_sim;
    }
  }
}

inline dim3 pr_grid(int64_t n, int lc) {
  const int64_t per_block = (int64_t)(kBlock / kWave) * (kWave / lc);
  return dim3((unsigned)((n + per_block - 1) / per_block));
}

}  // namespace

size_t priority_stage_smem_bytes(const DevProblem &pb) {
  return (size_t)pr_table_bytes(pb) + (size_t)(kBlock / kWave) * (kWave / pb.lc) * pr_chain_bytes(pb);
}

// (lanes per chain, regulator slots) of every instantiated kernel
#define SA_PR_DISPATCH(KERNEL, GRID, SMEM, ...)                                               \
  switch (pb.lc * 100 + pb.dmax) {                                                           \
    case 1600: KERNEL<16, 0><<<GRID, kBlock, SMEM, s>>>(__VA_ARGS__); break;                 \
    case 3200: KERNEL<32, 0><<<GRID, kBlock, SMEM, s>>>(__VA_ARGS__); break;                 \
    case 6408: KERNEL<64, 8><<<GRID, kBlock, SMEM, s>>>(__VA_ARGS__); break;                 \
    case 6416: KERNEL<64, 16><<<GRID, kBlock, SMEM, s>>>(__VA_ARGS__); break;                \
    case 6400: KERNEL<64, 0><<<GRID, kBlock, SMEM, s>>>(__VA_ARGS__); break;                 \
    default: return (int)hipErrorInvalidValue;                                               \
  }

int launch_priority_eval(const DevProblem &pb, const int8_t *x, int64_t n, int32_t *cost, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  SA_PR_DISPATCH(pr_eval_kernel, pr_grid(n, pb.lc), 0, pb, x, n, cost)
  return (int)hipGetLastError();
}

int launch_priority_simulate(const DevProblem &pb, const int8_t *x, int64_t n, int8_t *traj, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  SA_PR_DISPATCH(pr_simulate_kernel, pr_grid(n, pb.lc), 0, pb, x, n, traj)
  return (int)hipGetLastError();
}

int launch_priority_stage(const DevProblem &pb, const StageArgs &sa, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  const size_t smem = priority_stage_smem_bytes(pb);
  SA_PR_DISPATCH(pr_stage_kernel, pr_grid(sa.n_chains, pb.lc), smem, pb, sa)
  return (int)hipGetLastError();
}

#undef SA_PR_DISPATCH

}  // namespace sa
