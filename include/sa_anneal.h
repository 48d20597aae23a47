/*
 * sa_anneal.h -- C ABI of the MI355X (gfx950) library that fits the ternary
 * parameters of a discrete logic model of a regulatory network to sparse
 * time-course data by massively parallel simulated annealing.
 *
 * Method: Reimer et al., "GPU-accelerated modeling of biological regulatory
 * networks" (arXiv 2506.19866).
 *   - model: §2.1 (states s in {0,1,2}; image K_i = sum over regulators of the
 *     regulator terms) with the synchronous update named in §2.2; here the
 *     term of edge j->i is a_ji * s_j with a in {-1,0,+1} (polarity times a
 *     0/1 weight, threshold 1) and the node threshold theta_i in {0,1,2} is
 *     subtracted from the image (theta = 0 is the zero node bias of §2.5.3 b);
 *     a free node moves towards clamp(K_i, 0, 2) by at most d levels per step;
 *   - objective: §2.3, the Manhattan distance between simulated and reference
 *     data at the observed points, weighted by |G| + 1 where G is the
 *     difference between consecutive observed time points (0 at the first);
 *   - constraints: §2.5.3 (a) every node has a non-zero out-edge and (b) every
 *     node has an activating (+1) in-edge; cost = M + lambda * V where V counts
 *     the failing nodes of (a) plus those of (b);
 *   - search: Table 1 (parallel simulated annealing with a global restart from
 *     the best chain after every temperature stage);
 *   - the paper's own parameterisation with the priority update of §2.2 is
 *     selected per problem (SA_MODEL_PRIORITY below); objective, constraints
 *     and search are the same.
 *
 * Conventions of every entry point:
 *   - return 0 (SA_OK) on success, a negative SA_ERR_* code on failure; the
 *     message of the last failure of the calling thread is sa_last_error();
 *   - "host" pointers are read during the call only (the library copies what
 *     it keeps); "device" pointers are HIP device memory owned by the caller
 *     and must stay valid until the work queued on the given stream is done;
 *   - `stream` is a hipStream_t (NULL = the default stream); calls that take a
 *     stream only enqueue work on it, except where stated;
 *   - objects returned through `out` are owned by the library and released by
 *     the matching sa_destroy_* call; they may be used from one thread at a
 *     time.
 */
#ifndef SA_ANNEAL_H
#define SA_ANNEAL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SA_OK = 0,
  SA_ERR_ARG = -1,         /* null pointer, size or count out of range */
  SA_ERR_DOMAIN = -2,      /* a state, parameter or observation outside its domain */
  SA_ERR_TOPOLOGY = -3,    /* malformed graph, or (hard mode) a node without in- or out-edges */
  SA_ERR_INFEASIBLE = -4,  /* hard mode: a starting vector breaks a constraint */
  SA_ERR_DEVICE = -5,      /* a HIP call failed */
  SA_ERR_OOM = -6,         /* device allocation failed */
  SA_ERR_UNSUPPORTED = -7, /* size beyond what the kernels handle (see sa_create_problem) */
  SA_ERR_OVERFLOW = -8,    /* the largest possible cost does not fit in int32 */
  SA_ERR_ABORTED = -9      /* sa_run_launch: the run's abort flag is set, nothing was queued */
};

enum { SA_HARD = 0, SA_PENALTY = 1 };

/* The logic model of a problem.
 * SA_MODEL_SYNCHRONOUS: every node moves at every step (the synchronous scheme
 *   §2.2 names as the usual alternative); one ternary parameter per edge,
 *   a in {-1,0,1} (the product p * w with w in {0,1} and threshold 1), and one
 *   per node, theta in {0,1,2} subtracted from the image; P = E + N.
 * SA_MODEL_PRIORITY: the paper's own model.  Per edge a weight w in {0,1,2},
 *   a polarity p in {-1,0,1} and a threshold t in {1,2}; the image of node i
 *   is K_i = sum over in-edges (s_j div t) * w * p (§2.1).  Per node a speed
 *   u in {1..6, 10, 11, 12}, a memory m in {0,1,2} and a step size d in {1,2}
 *   drive the priority update of §2.2: a free node whose clamped image differs
 *   from its state at m + 1 consecutive steps is eligible, with priority u
 *   times the steps since it last moved; the eligible nodes of the highest
 *   priority move towards the image by at most d.  Constraints (§2.5.3):
 *   (a) an out-edge with w != 0, (b) an in-edge with p = +1 and w != 0.
 *   x = [w_e] ++ [p_e] ++ [t_e] (edges in in-CSR order) ++ [u_i] ++ [m_i] ++
 *   [d_i]; P = 3E + 3N.  Networks of at most 64 nodes. */
enum { SA_MODEL_SYNCHRONOUS = 0, SA_MODEL_PRIORITY = 1 };

typedef struct sa_problem sa_problem;
typedef struct sa_run sa_run;
typedef struct sa_mlp sa_mlp; /* proposal network, see the end of this header */

/* A network, its experimental conditions and the reference data (§2.3, §2.5).
 * All pointers are host pointers, copied by sa_create_problem. */
typedef struct {
  int32_t n_nodes;            /* N >= 1 */
  int32_t n_edges;            /* E >= 0 */
  const int32_t *in_row_ptr;  /* [N+1]: in-edges of node i are in_row_ptr[i] .. in_row_ptr[i+1]-1;
                                 this order is the canonical parameter order */
  const int32_t *in_src;      /* [E]: source node, strictly ascending within a row, never the target */
  int32_t n_conditions;       /* C >= 1 (initial states plus perturbations) */
  const int8_t *init_state;   /* [C*N]: state at t = 0, in {0,1,2} */
  const int8_t *clamp;        /* [C*N]: -1 = free, else the value the node is held at for all t */
  int32_t n_steps;            /* T_s >= 1 synchronous update steps */
  int32_t n_obs_times;        /* K >= 1 */
  const int32_t *obs_times;   /* [K]: strictly increasing, in [0, T_s] */
  int32_t n_obs_nodes;        /* O >= 1 */
  const int32_t *obs_nodes;   /* [O]: distinct nodes */
  const int8_t *observed;     /* [C*K*O]: reference data R, row-major (condition, time, node), in {0,1,2} */
  int32_t step_size;          /* d in {1,2} */
  int32_t constraint_mode;    /* SA_HARD: a proposal that breaks (a) or (b) is a rejected step (§2.5.3);
                                 SA_PENALTY: every proposal is scored with lambda * V */
  int32_t penalty;            /* lambda >= 0; 0 selects 1 + 2 * sum(W), larger than any mismatch */
  int32_t model;              /* SA_MODEL_SYNCHRONOUS or SA_MODEL_PRIORITY (step_size is then unused:
                                 each node carries its own d) */
} sa_problem_desc;

typedef struct {
  int32_t n_params;   /* P = E + N: x = [a_e in in-CSR order] ++ [theta_0 .. theta_{N-1}];
                         P = 3E + 3N for SA_MODEL_PRIORITY (layout above) */
  int32_t n_nodes, n_edges, n_conditions, n_steps, n_obs_times, n_obs_nodes;
  int32_t weight_sum; /* sum of W over all observations */
  int32_t penalty;    /* lambda in effect */
  int32_t max_cost;   /* 2 * weight_sum + lambda * 2N */
  int32_t clamps_by_offset; /* 1: the plain kernels hold clamped nodes through accumulator offsets of
                               the product (every clamp value 0 or 2 and at most 32 clamped nodes,
                               placed in the first state dword); 0: through a select per dword */
  int32_t obs_dwords;       /* synchronous model: packed state dwords per lane that the scoring reads
                               (with their reference and weight dwords) at every observed time; 0 for
                               the priority model */
} sa_problem_info;

/* Validates the description, precomputes the weights W and lambda and the
 * register layout of the kernels, and copies everything to the current HIP
 * device (synchronous).  Sizes handled: N <= 191, C <= 64 (synchronous
 * model); N <= 64 (priority model).
 * Errors: SA_ERR_ARG, SA_ERR_DOMAIN, SA_ERR_TOPOLOGY, SA_ERR_UNSUPPORTED,
 * SA_ERR_OVERFLOW, SA_ERR_DEVICE, SA_ERR_OOM. */
int sa_create_problem(const sa_problem_desc *desc, sa_problem **out);
int sa_destroy_problem(sa_problem *prob);
int sa_problem_get_info(const sa_problem *prob, sa_problem_info *info);

/* cost_dev[i] = M(x_i) + lambda * V(x_i) (§2.3, §2.5.3) for the n vectors
 * x_dev[i*P .. i*P+P-1] (device, int8, a in {-1,0,1}, theta in {0,1,2}; or
 * the priority model's layout and domains).
 * Values outside the domain are not checked (their cost is unspecified).
 * n = 0 is a no-op. */
int sa_eval_cost(const sa_problem *prob, const int8_t *x_dev, int64_t n, int32_t *cost_dev, void *stream);

/* traj_dev[((i*C + c)*(T_s+1) + t)*N + v] = state of node v at step t under
 * condition c for vector x_i (device, int8): the trajectories of §2.2 under
 * the problem's update scheme, clamped nodes held.  n = 0 is a no-op. */
int sa_simulate(const sa_problem *prob, const int8_t *x_dev, int64_t n, int8_t *traj_dev, void *stream);

/* Annealing schedule and chains (Table 1).  Stage k runs at
 * T_k = T0 * rho * rho * ... (k products, IEEE double) and accepts an uphill
 * move of size D iff the top 32 bits of Philox word 2 are below
 * floor(2^32 * exp(-D / T_k)) (clipped to 2^32 - 1).  Step `it` of stage k
 * of chain n of problem p draws Philox4x64-10 with counter
 * (k * steps_per_stage + it, n, p, 0) and key (seed, 0). */
typedef struct {
  int64_t n_chains;          /* chains per problem, >= 1 */
  uint64_t seed;
  double T0;                 /* > 0 */
  double rho;                /* > 0 */
  int32_t first_stage;       /* >= 0: stage index of the first stage (resume from a checkpoint) */
  int32_t n_stages;          /* >= 0: stages in the schedule of this run */
  int32_t steps_per_stage;   /* L >= 1 */
  int32_t record_times;      /* non-zero: time every stage kernel with a HIP event pair on the launch stream */
  int32_t kernel;            /* SA_KERNEL_AUTO: the register layout specialised to the network for one
                                problem, the many-network persistent kernel for several;
                                SA_KERNEL_PERSISTENT: the persistent kernel also for one problem */
  int32_t chains_per_block;  /* persistent kernel: chains per work item / workgroup, 1, 2, 4 or 8;
                                0 = autotune (times the first stage with each, keeps the fastest) */
  int32_t use_graph;         /* non-zero: every sa_run_launch call becomes one captured hipGraph launch;
                                excludes record_times */
  /* Learned proposal and step trace (an extension of Table 1's GetCandidate,
   * not in the paper).  Both need one problem, kernel SA_KERNEL_AUTO, at most
   * 127 nodes and at most 42 observed times.  Before steps it = 0, R, 2R, ...
   * of every stage a chain simulates its current vector once more and
   * refreshes per-node aggregates of its observed-time states; with a model
   * it also scores its 2P single-parameter moves from 32 features and builds
   * integer weights floor(exp(score - max) * 2^16) (0 for moves that break
   * a structural constraint in hard mode).  A learned step takes the first
   * move whose cumulative weight exceeds (top 32 bits of Philox word 0 *
   * total) >> 32, unless the top 32 bits of word 3 are below
   * floor(eps_plain * 2^32) (eps_plain = 1: always), the weights are all 0,
   * or the chain already holds that move's value: then it takes Table 1's
   * candidate.  Constraints, simulation, score, Metropolis and restarts are
   * those of the plain method. */
  int32_t proposal;          /* SA_PROPOSAL_PLAIN or SA_PROPOSAL_LEARNED */
  int32_t refresh_every;     /* R >= 1 (learned runs and traced runs) */
  const sa_mlp *model;       /* learned: the scoring network; alive and unchanged while the run's work is queued */
  double eps_plain;          /* learned: in [0, 1] */
  void *trace_dev;           /* device, nullable: sa_trace_record [n_chains][trace_capacity] */
  int64_t trace_capacity;    /* records per chain, >= 1 with trace_dev */
  int32_t trace_every;       /* >= 1 with trace_dev: the steps whose global index g = k * L + it is a
                                multiple of trace_every are recorded, in slot (g - g_first) / trace_every
                                where g_first is the run's first such g; slots beyond the capacity are
                                dropped.  Features use the aggregates of the chain's last refresh. */
  int64_t group_size;        /* >= 0.  Island restart (the reduction within groups of chains suggested
                                in §4): with 0 < group_size < n_chains, at every stage boundary each group
                                of group_size consecutive chains (the last one may be shorter) restarts
                                from its own best chain (lowest chain id on ties) instead of the global
                                best; 0 or >= n_chains is Table 1's global restart.  Stage statistics and
                                sa_best still report the global best.  Plain proposals only. */
  volatile int32_t *abort_flag_host;
                             /* nullable.  Stopping a queued run at a stage boundary of Table 1's stage
                                loop (the point where §2.4.1's loop reduces, restarts and cools; a
                                checkpoint there is the winner's vector and the stage index): pinned host
                                memory (hipHostMalloc, or a pinned torch tensor) that stays valid and
                                pinned until the run is destroyed; else SA_ERR_ARG at creation.  Before
                                every queued stage, graph-captured ones included, one small kernel reads the
                                flag once (system scope); if it is non-zero, that stage and every later
                                stage of the run return at their kernels' entry without writing anything,
                                so the run keeps the state of its last completed stage, and sa_run_launch
                                queues nothing while the flag reads non-zero (SA_ERR_ABORTED).  The flag is
                                the caller's to set, at any time, from any host thread; the library never
                                writes it.  sa_run_stages_done gives the stages that completed; resuming is
                                a new run with first_stage advanced by that count and every chain's
                                starting vector the winner's (sa_best; with island restarts each chain's
                                group winner, from sa_chain_best), bit-identical to the uninterrupted run. */
} sa_run_desc;

enum { SA_KERNEL_AUTO = 0, SA_KERNEL_PERSISTENT = 1 };
enum { SA_PROPOSAL_PLAIN = 0, SA_PROPOSAL_LEARNED = 1 };
/* source of a candidate (trace flags bits 2-3) */
enum { SA_SOURCE_PLAIN = 0, SA_SOURCE_LEARNED = 1, SA_SOURCE_STALE = 2, SA_SOURCE_EMPTY = 3 };

/* One traced step: the candidate's 32 features (bfloat16 bit patterns; the
 * feature definitions are those of the proposal network's inputs), the
 * candidate (parameter index and new value), the cost change (0 when
 * infeasible) and flags: bit 0 accepted, bit 1 feasible, bits 2-3 source. */
typedef struct {
  uint16_t features[32];
  int32_t param;
  int32_t value;
  int32_t delta;
  uint32_t flags;
} sa_trace_record;

typedef struct {
  int32_t n_probs;
  int32_t kernel;            /* SA_KERNEL_PERSISTENT when the many-network kernel runs */
  int32_t chains_per_block;  /* as chosen (by the autotuner when asked) */
  int32_t stages_launched;
  int32_t tiles_m;           /* register layout of problem 0: m-tiles of 16 rows */
  int32_t frags_k;           /* and k-fragments of 128 columns */
} sa_run_info;

/* Per temperature stage, per problem (before the global restart). */
typedef struct {
  int32_t best_cost;         /* lowest chain-best cost */
  int32_t winner;            /* its chain (lowest id on ties) */
  uint64_t accepted;         /* accepted proposals, all chains */
  uint64_t uphill;           /* accepted with D > 0 */
  uint64_t neutral;          /* accepted with D = 0 */
  uint64_t infeasible;       /* hard mode: proposals rejected for breaking (a) or (b) */
  uint64_t simulated;        /* trajectory simulations run: one per chain for its start vector and one per
                                feasible candidate, except (priority model) candidates that provably keep the
                                current trajectory (an edge whose (s div t) * w * p is unchanged for every s),
                                which are scored without one */
} sa_stage_stats;

/* Creates a run over n_probs independent problems (each with desc->n_chains
 * chains) and queues nothing.  x0_dev (device, int8) holds every chain's
 * starting vector, problems in order, [n_chains * P_p] each; it is copied.  In
 * hard mode every starting vector must satisfy (a) and (b) (else
 * SA_ERR_INFEASIBLE); checking that synchronises `stream`.  Several problems
 * (or desc->kernel = SA_KERNEL_PERSISTENT) run in one persistent launch per
 * stage and step size, networks up to 159 nodes; problem p draws its Philox
 * blocks with network id p.  Autotuning (chains_per_block = 0) runs the first
 * stage once per candidate before returning; results do not depend on it.
 * Problems of SA_MODEL_PRIORITY run on their own stage kernel, one launch
 * per problem and stage (problem p with network id p), with SA_KERNEL_AUTO
 * and plain proposals, and are not mixed with synchronous ones in a run (else
 * SA_ERR_UNSUPPORTED); island restarts, resume and graphs apply as above. */
int sa_run_create(sa_problem *const *probs, int32_t n_probs, const sa_run_desc *desc,
                  const int8_t *x0_dev, sa_run **out, void *stream);

/* Queues the next n_stages stages of the schedule (asynchronous).  The total
 * over all calls may not exceed desc->n_stages. */
int sa_run_launch(sa_run *run, int32_t n_stages, void *stream);

/* sa_run_create followed by sa_run_launch of the whole schedule. */
int sa_run_chains(sa_problem *const *probs, int32_t n_probs, const sa_run_desc *desc,
                  const int8_t *x0_dev, sa_run **out, void *stream);

/* Global best after the last completed stage: vector (host, [P]), its cost and
 * the chain it came from.  Synchronises the run's stream.  Any output may be NULL.
 * SA_ERR_ARG if no stage has completed (none launched, or aborted before the first). */
int sa_best(sa_run *run, int32_t prob, int8_t *x_host, int32_t *cost, int32_t *winner_chain);

/* Kernel choices of a run (no synchronisation). */
int sa_run_get_info(sa_run *run, sa_run_info *info);

/* Statistics of every launched stage (host, [stages launched]).  Synchronises.
 * Stages skipped by an abort read as all zero with best_cost = winner = -1. */
int sa_stats(sa_run *run, int32_t prob, sa_stage_stats *stats_host);

/* Stages of the run that have completed: the stages launched unless the abort
 * flag skipped the rest (abort_flag_host).  Synchronises the run's stream. */
int sa_run_stages_done(sa_run *run, int32_t *done);

/* Every chain's best cost (host, [n_chains]) and vector (host, [n_chains*P])
 * after the last launched stage, before the restart.  Synchronises.  Either
 * output may be NULL. */
int sa_chain_best(sa_run *run, int32_t prob, int32_t *cost_host, int8_t *x_host);

/* Duration in milliseconds of the stage kernel of every launched stage
 * (host, [stages launched]); needs desc->record_times.  Synchronises. */
int sa_stage_times(sa_run *run, int32_t prob, float *ms_host);

int sa_destroy_run(sa_run *run);

/* The whole schedule of one problem without any device allocation: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Same method, kernels
 * and results as sa_run_chains with that desc: bit for bit the same best
 * vector, cost, winner and stage statistics.  The run's state (chain bests,
 * costs, statistics, thresholds, stage records) lives in one fixed device
 * array of SA_NOALLOC_SCRATCH_BYTES per GPU, held from the library's load to
 * the end of the process, shared by every call on that GPU: calls that overlap
 * on one GPU (other streams, other host threads) race and give wrong results.
 * Nothing in it needs clearing: every stage writes all of its state before
 * reading it.  Supports the specialised kernel with plain proposals and the
 * global restart (kernel SA_KERNEL_AUTO, proposal SA_PROPOSAL_PLAIN,
 * group_size 0 or >= n_chains, no trace, record_times, use_graph or
 * abort_flag_host; else SA_ERR_UNSUPPORTED), n_stages >= 1, and runs needing
 * at most SA_NOALLOC_SCRATCH_BYTES: 256-byte aligned blocks of 48 bytes per
 * stage, n_chains * (P + 24) bytes, P bytes and the thresholds (4 bytes per
 * entry, at most 46 per stage for T <= 2); e.g. 16384 chains of a
 * 723-parameter problem need 12.3 MB.  Larger runs: SA_ERR_UNSUPPORTED, before
 * any device work.
 * x0_dev (device) [n_chains * P] starting vectors, read while the run is
 * queued; x_best_dev (device) [P] receives the global best vector,
 * best_dev (device) [2] its cost and chain, stats_dev (device, nullable)
 * [n_stages] the stage statistics (sa_stage_stats layout).  Checks the
 * starting vectors as sa_run_create does and synchronises `stream` for that;
 * the stages are then queued on `stream` and the call returns. */
#define SA_NOALLOC_SCRATCH_BYTES (16u << 20)
int sa_run_chains_noalloc(const sa_problem *prob, const sa_run_desc *desc, const int8_t *x0_dev,
                          int8_t *x_best_dev, int32_t *best_dev, sa_stage_stats *stats_dev, void *stream);

/* ---------------------------------------------------------------------------
 * Learned proposal network.  An extension of Table 1's GetCandidate (not in
 * the paper): a network scores every single-parameter move of a chain from 32
 * features, and the learned run draws its candidates from those scores.
 * Architecture: 32 inputs -> 256 ReLU units -> 1 score; bf16 weights and
 * activations, float32 accumulation on the matrix cores.  Training: binary
 * cross-entropy with logits, mean over the batch, Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8) on float32 master weights.
 * All calls on one model use its internal scratch: queue them on one stream.
 * ------------------------------------------------------------------------- */
#define SA_MLP_INPUTS 32
#define SA_MLP_HIDDEN 256
#define SA_MLP_N_PARAMS (SA_MLP_INPUTS * SA_MLP_HIDDEN + SA_MLP_HIDDEN + 1)

/* params (host, SA_MLP_N_PARAMS floats): W1[k][h] row-major (k < 32 inputs,
 * h < 256 hidden units; input 31 is the constant 1, so W1[31][.] is the
 * hidden bias), then w2[256], then b2.  Non-finite values give SA_ERR_DOMAIN.
 * The model lives on the current device; creation synchronises the device. */
int sa_mlp_create(const float *params, sa_mlp **out);
int sa_mlp_destroy(sa_mlp *model);

/* Copies the float32 master parameters to host (synchronises the device). */
int sa_mlp_get_params(const sa_mlp *model, float *params);

/* Replaces the parameters and resets the Adam state (synchronises the device). */
int sa_mlp_set_params(sa_mlp *model, const float *params);

/* Scores of n feature rows: x_dev [n][32] bfloat16 bit patterns (device),
 * logit_dev [n] float (device).  n = 0 is a no-op. */
int sa_mlp_forward(const sa_mlp *model, const uint16_t *x_dev, int64_t n, float *logit_dev, void *stream);

/* Gradient of the batch's mean binary cross-entropy, labels y_dev [n] in
 * [0, 1] (device): grad_dev [SA_MLP_N_PARAMS] floats in the layout of params
 * (device); loss_dev (device, nullable) receives the mean loss.  n >= 1. */
int sa_mlp_gradients(sa_mlp *model, const uint16_t *x_dev, const float *y_dev, int64_t n, float *grad_dev,
                     float *loss_dev, void *stream);

/* One Adam step with learning rate lr > 0 on the batch's gradient;
 * loss_dev (device, nullable) receives the batch's mean loss before the step. */
int sa_mlp_train_step(sa_mlp *model, const uint16_t *x_dev, const float *y_dev, int64_t n, float lr,
                      float *loss_dev, void *stream);

/* ---------------------------------------------------------------------------
 * Measured instruction peaks, the denominators of the benchmark's roofline
 * figures (not part of the method).  The annealing kernels are bound by
 * 32-bit integer VALU issue, a floating-point -> fp4 packing conversion and
 * fp4 matrix products; the chip's published figures cover floating-point
 * arithmetic only, so each rate is measured on the device: every lane of a
 * full-occupancy grid (8 waves per SIMD) runs 8 independent dependency
 * chains of one instruction.
 *   SA_PEAK_VALU_XOR, _ADD, _BITOP3: v_xor_b32, v_add_u32, v_bitop3_b32, in
 *     32-bit lane-ops per second (64 per wave instruction);
 *   SA_PEAK_CVT_FP4: v_cvt_scalef32_pk_fp4_f32 (2 floats to 2 fp4 codes per
 *     lane), in values converted per second;
 *   SA_PEAK_MFMA_FP4: the unscaled fp4 x fp4 16x16x128 matrix product, in
 *     flops per second (2 x 16 x 16 x 128 per instruction);
 *   SA_PEAK_CVT_FP6: v_cvt_scalef32_2xpk16_fp6_f32 (32 floats to 32 fp6
 *     codes per lane), in values converted per second;
 *   SA_PEAK_MFMA_FP4_FP6: the same product with the B operand read as fp6;
 *   SA_PEAK_LDS_READ: 16-byte LDS reads (ds_read_b128), every lane of a wave
 *     reading consecutive words (no bank conflict), in bytes per second.
 * (SA_PEAK_CVT_FP6 and SA_PEAK_MFMA_FP4_FP6 price an fp6 state encoding
 * against the fp4 one.)
 * rate (host) receives the rate; ms (host, nullable) the best of two timed
 * launches after a warm-up one.  Allocates a small buffer, synchronises
 * `stream`. */
enum { SA_PEAK_VALU_XOR = 0, SA_PEAK_VALU_ADD = 1, SA_PEAK_VALU_BITOP3 = 2, SA_PEAK_CVT_FP4 = 3,
       SA_PEAK_MFMA_FP4 = 4, SA_PEAK_CVT_FP6 = 5, SA_PEAK_MFMA_FP4_FP6 = 6, SA_PEAK_LDS_READ = 7 };
int sa_measure_peak(int32_t kind, double *rate, double *ms, void *stream);

/* Message of the last failure on the calling thread ("" if none). */
const char *sa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SA_ANNEAL_H */
