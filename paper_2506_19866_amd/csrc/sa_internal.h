// sa_internal.h -- device-side problem layout shared by the host part of the
// library (sa_api.hip) and its kernels (sa_k_batch.hip, sa_k_stage.hip).  Not a public header.
//
// Register-resident simulation on the 4-bit matrix cores of gfx950
// -----------------------------------------------------------------
// One wavefront owns one chain.  The synchronous update of all nodes under 16
// conditions at once is one product per time step,
//     X[row(i)][c] = sum_j A[row(i)][col(j)] * S[col(j)][c] = 2 (h_i - 1),
// where A holds the chain's edge values a_ji in {-1, 0, 1} (and -theta_i - 1
// in {-3, -2, -1} in the column of a constant "bias" input fixed at 1), and S
// the states, one column per condition, held as 2s (codes 0x0, 0x4, 0x6 of
// 0, 2.0, 4.0).  Both operands are exact fp4 (e2m1) codes and the product
// runs as unscaled v_mfma_f32_16x16x128_f8f6f4 tiles with float32 results
// that are exact small integers: A is the 16x128 A operand of m-tile mt and k-fragment kf,
// S the 128x16 B operand of k-fragment kf.  A state's code is a thermometer
// code: bit 2 is [s >= 1], bit 1 is [s >= 2].
//
// Lane l holds A rows l%16 and B/D columns l%16 (condition), and 32 nibbles
// of the k-range of lane group g = l/16 (A and B share that k mapping).  The
// D result of m-tile mt holds rows 4g + r (r = 0..3) in lane group g.  Each
// node gets one "slot" (g, q): its state leaves the product in lane group g,
// m-tile q/4, register r = q%4, and re-enters the next product as nibble q%32
// of k-fragment q/32 in the same lane group.  So the 4 results of m-tile mt
// pack into half a dword of the next B operand (k-fragment mt/8, dword
// (mt%8)/2, bytes 2(mt%2) and 2(mt%2)+1) and the whole trajectory stays in the
// lane's registers: no LDS, no cross-lane traffic.
#pragma once
#include <stdint.h>

namespace sa {

constexpr int kWave = 64;
constexpr int kMaxTilesM = 12;  // N <= 191: 12 m-tiles, 2 k-fragments of 128
constexpr int kMaxCondGroups = 4;

// fp4 code of the state s in {0, 1, 2} (the value 2s)
constexpr uint32_t state_code(int s) { return s == 0 ? 0u : (s == 1 ? 0x4u : 0x6u); }

struct DevProblem {
  int32_t N, E, P, C, T, K, O;
  int32_t CG;      // condition groups of 16
  int32_t nm, nk;  // m-tiles (16 rows) and k-fragments (128 columns)
  int32_t nd;      // dwords per lane (8 slots each) that hold observed slots
  int32_t d;       // step size
  int32_t hard;
  int32_t lambda;
  // [P]: lane | m-tile << 8 | k-fragment << 12 | dword << 14 | nibble << 16
  // of the A entry of parameter p (independent of the register layout)
  const uint32_t *param_pos;
  const int32_t *edge_src, *edge_dst;  // [E]
  const int32_t *in_ptr;               // [N+1]
  const int32_t *out_ptr, *out_eid;    // [N+1], [E]: out-edges of each node (edge ids)
  // [CG][4*nk dwords][64 lanes]: packed state codes at t = 0 (clamped nodes
  // at their clamp value) and the mask of nibbles that are held (clamped
  // nodes, the bias slot, empty slots and lanes beyond the last condition)
  const uint32_t *b0, *cmask;
  // Where every clamp value is 0 or 2 and every clamped node sits in the
  // first dword of every lane (hold_by_offset = 1), clamped nodes are held by
  // the product itself instead: [CG][2 m-tiles][64 lanes][4] accumulator
  // offsets of m-tiles 0 and 1, +2^14 for a row whose node is clamped to 2 in
  // the lane's condition and -2^14 for one clamped to 0 (0 elsewhere), far
  // beyond any |2(h - 1)| <= 4 in-degree + 6 (and exact in float32), so the
  // node's target is its clamp value and it stays there; the bias row
  // (all-zero A row: target 1), empty slots and unclamped nodes need no
  // hold, except in the unused half of a layout's last dword, which keeps its
  // state.
  const float *cofs;
  int32_t hold_by_offset;
  // [CG][K][nd dwords][64 lanes]: packed reference values and weights, a
  // nibble per slot (weight 0 where unobserved)
  const uint32_t *obs_r, *obs_w;
  const int32_t *obs_t;                // [K]
  const int16_t *slot_node;            // [4][32*nk]: node at (g, q), -1 bias/empty
  // learned proposal (networks up to 127 nodes)
  int32_t sum_w;                       // sum of all observation weights
  const int16_t *node_slot;            // [N]: g * 32*nk + q of the node's slot
  const int32_t *node_sw, *node_wr;    // [N]: sum of W and of W*R over the node's observations (0: unobserved)
  // [P]: target i | source j << 7 | in-degree(i) << 14 | out-degree(j) << 21 |
  // edge << 28 | observed(i) << 29 | observed(j) << 30 (j = 0 for a threshold)
  const uint32_t *param_info;
  // priority model (model 1, sa_priority.h): lc lanes per chain (16, 32 or 64
  // >= N), node i on lane i of its chain's lane segment
  int32_t model;
  int32_t lc;
  int32_t dmax;             // regulator slots per node (8 or 16, >= the largest in-degree), 0: masks
  const uint8_t *pr_start;  // [C][lc]: state at t = 0 | 4 if held (clamped, or a lane beyond N)
  const uint32_t *pr_obs;   // [C][T+1][lc]: byte s = W * |s - R| for s = 0, 1, 2 (0 where not observed)
};

// One temperature stage of one problem.
struct StageArgs {
  int64_t n_chains;
  uint64_t seed;
  int32_t net;
  int32_t stage;          // absolute stage index k
  int32_t L;              // steps per stage
  int32_t dcap;           // largest uphill move with a non-zero threshold
  const uint32_t *tau;    // [dcap+1] thresholds of this stage (entry 0 unused)
  const int8_t *x_start;  // first stage: [n_chains*P]; later: winner [P], or one per group [n_groups*P]
  int64_t x_start_stride; // P (first stage) or 0
  int64_t group;          // later stages: chains per restart group (chain c starts from winner c / group), 0: one winner
  int8_t *xbest;          // [n_chains*P] out
  int32_t *cbest;         // [n_chains] out
  uint32_t *cstats;       // [n_chains*kStatWords] out
  const uint32_t *stop;   // nullable: the run's stop word; non-zero: return at entry, writing nothing
};

// Per-chain statistics of a stage: accepted, uphill, neutral, infeasible
// candidates, and the simulations run (start vector and scored candidates).
constexpr int kStatWords = 5;

struct StageRecord {
  int32_t best_cost;
  int32_t winner;
  uint64_t accepted, uphill, neutral, infeasible, simulated;
};


// One temperature stage of many networks in one persistent launch (per step
// size d present): blocks take work items (a network and `waves` of its
// chains) from a queue in longest-first order until it is empty.
struct BatchArgs {
  const DevProblem *probs;    // [n_probs], device copy
  int32_t n_probs;
  int64_t n_chains;           // per network
  const int32_t *item_net;    // [n_items]
  const int32_t *item_chain0; // [n_items]
  int32_t n_items;
  int32_t waves;              // chains per work item = waves per block
  uint32_t *queue;            // next item; zero when the launch starts
  uint64_t seed;
  int32_t stage, L, dcap;
  const uint32_t *tau;        // [dcap+1]
  const int8_t *x_start;      // first stage: x0 at x_off; later: winners at w_off (one per restart group)
  int32_t first;
  int64_t group;              // chains per restart group, 0: one group
  const int64_t *x_off;       // [n_probs]: byte offset of the network's chain vectors
  const int64_t *w_off;       // [n_probs]: byte offset of the network's winner vector
  int8_t *xbest;              // at x_off
  int32_t *cbest;             // [n_probs * n_chains]
  uint32_t *cstats;           // [n_probs * n_chains * kStatWords]
  const uint32_t *stop;       // nullable: the run's stop word; non-zero: return at entry, writing nothing
};

// Table 1's serial part for every network of a run (one block per network):
// winner, its vector copied for the next stage, statistics summed; also resets
// the work queue of the persistent kernel.  With restart groups the winner is
// only recorded, and the group kernel copies every group's own winner.
struct BatchReduceArgs {
  int32_t n_probs;
  int64_t n_chains;
  int64_t group;              // chains per restart group, 0: one group
  const DevProblem *probs;
  const int64_t *x_off, *w_off;
  const int32_t *cbest;
  const int8_t *xbest;
  const uint32_t *cstats;
  int8_t *xwin;
  StageRecord *rec;           // [n_probs] of this stage
  uint32_t *queue;            // [kPersistentQueues] work counters to reset, or null
  uint32_t *ctl;              // nullable: run control {stop word, stages completed}; with a non-zero stop
                              // word the stage's reduction writes nothing, else it sets ctl[1] = st + 1
  int32_t st;                 // stage index within the run
};

// One traced annealing step (the C ABI's sa_trace_record).
struct TraceRecord {
  uint16_t features[32];  // bf16 features of the candidate (refresh-time aggregates, current vector)
  int32_t param, value, delta;
  uint32_t flags;         // bit 0 accepted, bit 1 feasible, bits 2-3 source
};

// The learned proposal's part of a stage (sa_k_learned.hip).
struct LearnedArgs {
  const void *w1f, *w2f;   // bf16 network fragments; null: plain candidates, refreshes only for the trace
  const float *b2;         // device scalar
  int32_t refresh;         // steps between table refreshes
  uint64_t eps_u;          // the plain candidate is taken when Philox word 3's top 32 bits are below this
  float lt;                // f32(ln(T_k) / 5) of the stage
  TraceRecord *trace;      // [n_chains][trace_cap] or null
  int64_t trace_cap;
  int64_t trace_every;
  int64_t trace_first;     // first traced global step of the run
};

// Launch wrappers (sa_k_batch.hip, sa_k_stage.hip, sa_k_persist.hip,
// sa_k_learned.hip).  All return a hipError_t as int.
int launch_eval(const DevProblem &pb, const int8_t *x, int64_t n, int32_t *cost, void *stream);
int launch_simulate(const DevProblem &pb, const int8_t *x, int64_t n, int8_t *traj, void *stream);
int launch_stage(const DevProblem &pb, const StageArgs &sa, void *stream);
size_t stage_smem_bytes(const DevProblem &pb, int waves_per_block);
int stage_waves_per_block(const DevProblem &pb);
// Persistent launch of size class cls (layout (4,1), (8,1) or (10,2)) and step size d.
int launch_persistent(const BatchArgs &a, int cls, int d, int grid, size_t smem, void *stream);
int persistent_class(int nm);
int launch_batch_reduce(const BatchReduceArgs &ra, void *stream);
// Stage boundary of a run with a host abort flag: reads the flag once
// (system scope, so the host's latest store is seen) and, if it is non-zero,
// sets the run's stop word ctl[0], which every later kernel of the run reads
// at entry.
// Instruction-throughput probes (sa_k_probe.hip): the launch, and the work
// one launch does (lane-ops, or flops for the matrix product).
int launch_probe(int kind, void *sink, int blocks, int threads, void *stream);
double probe_work(int kind, int blocks, int threads);
int launch_abort_gate(const volatile int32_t *flag, uint32_t *ctl, void *stream);
size_t persistent_smem_bytes(const DevProblem &pb, int waves);
// Workgroups of `waves` waves with `smem` bytes of LDS of class cls that fit on one CU.
int persistent_blocks_per_cu(int cls, int waves, size_t smem);
constexpr int kPersistentTilesM = 10, kPersistentTilesK = 2;  // networks up to 159 nodes
constexpr int kPersistentClasses = 3;
constexpr int kPersistentQueues = 2 * kPersistentClasses;     // one work counter per (class, step size)
int launch_learned_stage(const DevProblem &pb, const StageArgs &sa, const LearnedArgs &la, void *stream);
// Priority model (sa_k_priority.hip): cost, trajectories and one stage.
int launch_priority_eval(const DevProblem &pb, const int8_t *x, int64_t n, int32_t *cost, void *stream);
int launch_priority_simulate(const DevProblem &pb, const int8_t *x, int64_t n, int8_t *traj, void *stream);
int launch_priority_stage(const DevProblem &pb, const StageArgs &sa, void *stream);
size_t priority_stage_smem_bytes(const DevProblem &pb);
// LDS of a learned-stage workgroup; prepare sets the kernel's LDS limit to it.
size_t learned_smem_bytes(const DevProblem &pb, bool model);
int learned_stage_prepare(const DevProblem &pb, size_t smem);
constexpr int kLearnedMaxTilesM = 8;      // networks up to 127 nodes
constexpr int kLearnedMaxObsTimes = 42;   // byte accumulators of the refresh aggregates

}  // namespace sa
