/*
 * sa_oracle.c -- plain serial CPU oracle for the synchronous ternary logic
 * model of a regulatory network and for the parallel simulated annealing that
 * fits its parameters to time-course data (Reimer et al., "GPU-accelerated
 * modeling of biological regulatory networks", arXiv 2506.19866).
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark load this library.  It
 * shares no code, header, table or constant generator with the GPU library:
 * every definition below is written out again from the paper.
 *
 * Readings of the paper taken here:
 *   - update scheme: synchronous, every node moves from the states of the
 *     previous time step (the alternative named in §2.2);
 *   - parameters: x = [a_e for every edge, in-CSR order] ++ [theta_i per node],
 *     a_e = p*w with w in {0,1} and t = 1 (§2.1), theta_i in {0,1,2} is
 *     subtracted from the image, so theta = 0 is the paper's zero node bias
 *     (§2.5.3 b);
 *   - the node moves towards clamp(K_i, 0, 2) by at most d levels (§2.1, §2.2);
 *   - objective: gradient-weighted Manhattan distance over observed entries
 *     (§2.3, objective equation) plus lambda * (#violated constraints, §2.5.3);
 *   - annealing: Table 1, with a counter-based Philox4x64-10 stream, fixed-point
 *     Metropolis thresholds, lowest-chain-id tie-break.
 *
 * A second model, selected by ora_problem.model = 1, is the paper's own
 * parameterisation with the priority update scheme (§2.1, §2.2), for which
 * the readings are:
 *   - parameters: x = [w_e] ++ [p_e] ++ [t_e] (every edge, in-CSR order) ++
 *     [u_i] ++ [m_i] ++ [d_i] (every node), P = 3E + 3N, with w in {0,1,2},
 *     p in {-1,0,1}, t in {1,2}, u in {1..6, 10, 11, 12}, m in {0,1,2},
 *     d in {1,2}; the image is K_i = sum_j (s_j div t_ji) * w_ji * p_ji with
 *     no node bias (§2.5.3 b);
 *   - a free node is "told to update" at step t when clamp(K_i, 0, 2), from
 *     the states of step t-1, differs from its state; it is eligible when it
 *     has been told at more than m_i consecutive steps (this one included);
 *     its priority is u_i times the steps since its last update (or since
 *     t = 0); the eligible nodes of the highest priority move towards
 *     clamp(K_i, 0, 2) by at most d_i levels, and their step and telling
 *     counts restart; every other node keeps its state;
 *   - constraints: (a) a node needs an out-edge with w != 0; (b) a node needs
 *     an in-edge with p = +1 and w != 0 (§2.5.3).
 *
 * Nothing here is blocked, fused or reordered: one candidate is one full
 * re-simulation, exactly as Table 1 states.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t n_nodes, n_edges;
  const int32_t *row_ptr; /* [N+1]: in-edges of node i are row_ptr[i]..row_ptr[i+1]-1 */
  const int32_t *src;     /* [E]:   source node of each in-edge */
  int32_t n_cond;
  const int8_t *init;     /* [C*N]: state at t = 0 per condition */
  const int8_t *clamp;    /* [C*N]: -1 = free, else the value the node is held at */
  int32_t n_steps;        /* T_s */
  int32_t n_obs_t;
  const int32_t *obs_t;   /* [K] observed time points */
  int32_t n_obs_n;
  const int32_t *obs_n;   /* [O] observed nodes */
  const int8_t *observed; /* [C*K*O] reference data R */
  int32_t step_size;      /* d in {1,2} */
  int32_t hard;           /* 1: a proposal that breaks a constraint is rejected */
  int64_t penalty;        /* lambda; <= 0 selects 1 + 2*sum(W) */
  int32_t model;          /* 0: synchronous ternary model; 1: the paper's priority update (step_size unused) */
} ora_problem;

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from the        */
/* published description: ten rounds; each round multiplies words 0 and 2 by */
/* the two Philox multipliers, and mixes the high halves with words 1, 3 and  */
/* the round key; the key is bumped by the two Weyl constants between rounds. */
/* ------------------------------------------------------------------------ */
static void mul64_full(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *lo = (uint64_t)p;
  *hi = (uint64_t)(p >> 64);
}

void ora_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t mult0 = 0xD2E7470EE14C6C93ull, mult1 = 0xCA5A826395121157ull;
  const uint64_t weyl0 = 0x9E3779B97F4A7C15ull, weyl1 = 0xBB67AE8584CAA73Bull;
  uint64_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += weyl0;
      k1 += weyl1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul64_full(mult0, c[0], &hi0, &lo0);
    mul64_full(mult1, c[2], &hi1, &lo1);
    uint64_t n0 = hi1 ^ c[1] ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c[3] ^ k1;
    uint64_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ------------------------------------------------------------------------ */
/* Model                                                                     */
/* ------------------------------------------------------------------------ */
int64_t ora_n_params(const ora_problem *p) {
  return p->model == 1 ? 3 * (int64_t)p->n_edges + 3 * (int64_t)p->n_nodes : (int64_t)p->n_edges + p->n_nodes;
}

/* Speed values of the priority model (§2.2): slow 1..6, fast 10..12. */
static const int kSpeeds[9] = {1, 2, 3, 4, 5, 6, 10, 11, 12};

/* One condition: trajectory s(t) for t = 0..T_s, written to traj[(T_s+1)*N].
 * §2.1: the image of node i is the sum over its regulators j of (a_ji * s_j),
 * here minus theta_i; §2.2 (synchronous reading): every free node computes its
 * image from s(t-1) and moves towards clamp(image, 0, 2) by at most d levels.
 * A clamped node keeps its clamp value at every t (its regulators are ignored). */
static void simulate_condition(const ora_problem *p, const int8_t *x, int c, int8_t *traj) {
  const int N = p->n_nodes, E = p->n_edges, T = p->n_steps;
  const int8_t *a = x;
  const int8_t *theta = x + E;
  const int8_t *clamp = p->clamp + (size_t)c * N;
  const int8_t *init = p->init + (size_t)c * N;
  for (int i = 0; i < N; ++i) traj[i] = clamp[i] >= 0 ? clamp[i] : init[i];
  for (int t = 1; t <= T; ++t) {
    const int8_t *prev = traj + (size_t)(t - 1) * N;
    int8_t *next = traj + (size_t)t * N;
    for (int i = 0; i < N; ++i) {
      if (clamp[i] >= 0) {
        next[i] = prev[i];
        continue;
      }
      int h = 0;
      for (int e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) h += a[e] * prev[p->src[e]];
      int image = h - theta[i];
      int target = image < 0 ? 0 : (image > 2 ? 2 : image);
      int s = prev[i];
      int moved;
      if (p->step_size == 1) {
        moved = s + (target > s) - (target < s);
      } else {
        /* d = 2 covers the whole {0,1,2} range in one step */
        moved = target;
      }
      next[i] = (int8_t)moved;
    }
  }
}

/* One condition under the priority update (§2.1 image with w, p, t; §2.2
 * priority scheme with u, m, d; readings in the header). */
static void simulate_condition_priority(const ora_problem *p, const int8_t *x, int c, int8_t *traj) {
  const int N = p->n_nodes, E = p->n_edges, T = p->n_steps;
  const int8_t *w = x, *pol = x + E, *thr = x + 2 * E;
  const int8_t *speed = x + 3 * E, *memory = x + 3 * E + N, *dstep = x + 3 * E + 2 * N;
  const int8_t *clamp = p->clamp + (size_t)c * N;
  const int8_t *init = p->init + (size_t)c * N;
  int *image = (int *)malloc(sizeof(int) * (size_t)N);
  int *since = (int *)calloc((size_t)N, sizeof(int));   /* steps since the last update */
  int *told = (int *)calloc((size_t)N, sizeof(int));    /* consecutive steps told to update */
  int *prio = (int *)malloc(sizeof(int) * (size_t)N);
  for (int i = 0; i < N; ++i) traj[i] = clamp[i] >= 0 ? clamp[i] : init[i];
  for (int t = 1; t <= T; ++t) {
    const int8_t *prev = traj + (size_t)(t - 1) * N;
    int8_t *next = traj + (size_t)t * N;
    for (int i = 0; i < N; ++i) {
      int k = 0;
      for (int e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e) k += (prev[p->src[e]] / thr[e]) * w[e] * pol[e];
      image[i] = k;
    }
    int best = 0;
    for (int i = 0; i < N; ++i) {
      prio[i] = 0;
      if (clamp[i] >= 0) continue;
      since[i] += 1;
      const int target = image[i] < 0 ? 0 : (image[i] > 2 ? 2 : image[i]);
      if (target != prev[i]) {
        told[i] += 1;
        if (told[i] > memory[i]) prio[i] = speed[i] * since[i];
      } else {
        told[i] = 0;
      }
      if (prio[i] > best) best = prio[i];
    }
    for (int i = 0; i < N; ++i) {
      next[i] = prev[i];
      if (best == 0 || prio[i] != best) continue;
      const int target = image[i] < 0 ? 0 : (image[i] > 2 ? 2 : image[i]);
      const int dist = target > prev[i] ? target - prev[i] : prev[i] - target;
      const int move = dist < dstep[i] ? dist : dstep[i];
      next[i] = (int8_t)(prev[i] + (target > prev[i] ? move : -move));
      since[i] = 0;
      told[i] = 0;
    }
  }
  free(image); free(since); free(told); free(prio);
}

static void simulate_one(const ora_problem *p, const int8_t *x, int c, int8_t *traj) {
  if (p->model == 1)
    simulate_condition_priority(p, x, c, traj);
  else
    simulate_condition(p, x, c, traj);
}

/* traj: [C][T_s+1][N] */
void ora_simulate(const ora_problem *p, const int8_t *x, int8_t *traj) {
  const size_t per = (size_t)(p->n_steps + 1) * p->n_nodes;
  for (int c = 0; c < p->n_cond; ++c) simulate_one(p, x, c, traj + per * c);
}

/* Gradient weight of observation (c, k, o), §2.3 (gradient matrix G): the first
 * observed time has G = 0; later rows are differences between consecutive
 * observed time points.  Weight = |G| + 1. */
static int weight_of(const ora_problem *p, int c, int k, int o) {
  const int K = p->n_obs_t, O = p->n_obs_n;
  if (k == 0) return 1;
  int r1 = p->observed[((size_t)c * K + k) * O + o];
  int r0 = p->observed[((size_t)c * K + (k - 1)) * O + o];
  return 1 + abs(r1 - r0);
}

int64_t ora_weight_sum(const ora_problem *p) {
  int64_t total = 0;
  for (int c = 0; c < p->n_cond; ++c)
    for (int k = 0; k < p->n_obs_t; ++k)
      for (int o = 0; o < p->n_obs_n; ++o) total += weight_of(p, c, k, o);
  return total;
}

int64_t ora_lambda(const ora_problem *p) {
  return p->penalty > 0 ? p->penalty : 1 + 2 * ora_weight_sum(p);
}

/* M(x): §2.3 objective, sum over observed entries of |S - R| * (|G| + 1). */
int64_t ora_mismatch(const ora_problem *p, const int8_t *x) {
  const int N = p->n_nodes, T = p->n_steps, K = p->n_obs_t, O = p->n_obs_n;
  int8_t *traj = (int8_t *)malloc((size_t)(T + 1) * N);
  int64_t m = 0;
  for (int c = 0; c < p->n_cond; ++c) {
    simulate_one(p, x, c, traj);
    for (int k = 0; k < K; ++k)
      for (int o = 0; o < O; ++o) {
        int s = traj[(size_t)p->obs_t[k] * N + p->obs_n[o]];
        int r = p->observed[((size_t)c * K + k) * O + o];
        m += (int64_t)weight_of(p, c, k, o) * abs(s - r);
      }
  }
  free(traj);
  return m;
}

/* V(x): §2.5.3 (a) every node needs an outgoing edge with non-zero weight;
 * (b) every node needs an incoming activating edge (a = +1).  Counts the
 * nodes that fail (a) plus the nodes that fail (b). */
int32_t ora_violations(const ora_problem *p, const int8_t *x) {
  const int N = p->n_nodes, E = p->n_edges;
  const int pri = p->model == 1;
  int32_t v = 0;
  for (int i = 0; i < N; ++i) {
    int has_out = 0, has_act_in = 0;
    for (int j = 0; j < N; ++j)
      for (int e = p->row_ptr[j]; e < p->row_ptr[j + 1]; ++e)
        if (p->src[e] == i && x[e] != 0) has_out = 1;   /* a_e != 0, or w_e != 0 */
    for (int e = p->row_ptr[i]; e < p->row_ptr[i + 1]; ++e)
      if (pri ? (x[E + e] == 1 && x[e] != 0) : x[e] == 1) has_act_in = 1;
    v += !has_out;
    v += !has_act_in;
  }
  return v;
}

/* Cost = M + lambda * V.  lambda = 1 + 2*sum(W) exceeds the largest possible M,
 * so every feasible vector costs less than every infeasible one. */
int64_t ora_cost(const ora_problem *p, const int8_t *x) {
  return ora_mismatch(p, x) + ora_lambda(p) * (int64_t)ora_violations(p, x);
}

void ora_cost_batch(const ora_problem *p, const int8_t *xs, int64_t n, int64_t *out) {
  const int64_t P = ora_n_params(p);
  for (int64_t i = 0; i < n; ++i) out[i] = ora_cost(p, xs + i * P);
}

/* ------------------------------------------------------------------------ */
/* Annealing schedule and fixed-point Metropolis threshold                   */
/* ------------------------------------------------------------------------ */
/* Table 1 cools by T <- rho*T once per stage; the temperature of stage k is
 * that product iterated k times in IEEE double. */
double ora_stage_temperature(double T0, double rho, int64_t k) {
  double T = T0;
  for (int64_t i = 0; i < k; ++i) T = T * rho;
  return T;
}

/* Number of stages of the paper's schedule: while T > T_min, run a stage and
 * cool (Table 1, constants of §2.4.1). */
int64_t ora_count_stages(double T0, double T_min, double rho) {
  int64_t n = 0;
  double T = T0;
  while (T > T_min) {
    ++n;
    T = T * rho;
  }
  return n;
}

/* Table 1 accepts with probability exp((delta_cur - delta_cand)/T).  In fixed
 * point: a 32-bit uniform u accepts an uphill move of size D iff
 * u < floor(2^32 * exp(-D/T)); the threshold is clipped to 2^32-1. */
uint32_t ora_threshold(double T, int64_t delta) {
  double v = ldexp(exp(-(double)delta / T), 32);
  if (v >= 4294967295.0) return 0xFFFFFFFFu;
  return (uint32_t)floor(v);
}

/* ------------------------------------------------------------------------ */
/* Proposal (GetCandidate, Table 1): one random element changes to one of its  */
/* two other values.  Draws come from the Philox block of (step g, chain n,     */
/* network net) under key (seed, 0).                                          */
/* ------------------------------------------------------------------------ */
void ora_draw(uint64_t seed, uint64_t g, uint64_t chain, uint64_t net, uint64_t out[4]) {
  const uint64_t ctr[4] = {g, chain, net, 0};
  const uint64_t key[2] = {seed, 0};
  ora_philox4x64_10(ctr, key, out);
}

/* Decodes the draw: returns the index; *new_value is the proposed value. */
int64_t ora_propose(const ora_problem *p, const int8_t *x, const uint64_t u[4], int8_t *new_value) {
  const int64_t P = ora_n_params(p);
  int64_t i = (int64_t)(((u[0] >> 32) * (uint64_t)P) >> 32);
  if (p->model == 1) {
    /* the element's domain, as codes 0..k-1; one of the k-1 other codes,
     * uniformly (for k = 3 the same rule as the ternary model) */
    const int64_t E = p->n_edges, N = p->n_nodes;
    int k, code;
    if (i < E) { k = 3; code = x[i]; }                       /* w in {0,1,2} */
    else if (i < 2 * E) { k = 3; code = x[i] + 1; }          /* p in {-1,0,1} */
    else if (i < 3 * E) { k = 2; code = x[i] - 1; }          /* t in {1,2} */
    else if (i < 3 * E + N) {                                /* u in {1..6,10,11,12} */
      k = 9;
      for (code = 0; code < 8 && kSpeeds[code] != x[i]; ++code) {
      }
    } else if (i < 3 * E + 2 * N) { k = 3; code = x[i]; }    /* m in {0,1,2} */
    else { k = 2; code = x[i] - 1; }                         /* d in {1,2} */
    const int step = 1 + (int)(((u[1] >> 32) * (uint64_t)(k - 1)) >> 32);
    const int nc = (code + step) % k;
    int v;
    if (i < E) v = nc;
    else if (i < 2 * E) v = nc - 1;
    else if (i < 3 * E) v = nc + 1;
    else if (i < 3 * E + N) v = kSpeeds[nc];
    else if (i < 3 * E + 2 * N) v = nc;
    else v = nc + 1;
    *new_value = (int8_t)v;
    return i;
  }
  int is_edge = i < p->n_edges;
  int code = is_edge ? x[i] + 1 : x[i];           /* a in {-1,0,1} -> {0,1,2} */
  int step = 1 + (int)(u[1] >> 63);               /* +1 or +2 (mod 3): never a no-op */
  int new_code = (code + step) % 3;
  *new_value = (int8_t)(is_edge ? new_code - 1 : new_code);
  return i;
}

/* ------------------------------------------------------------------------ */
/* Parallel simulated annealing (Table 1)                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t n_chains;
  uint64_t seed;
  int32_t net;          /* network id in the Philox counter */
  double T0, rho;
  int32_t first_stage;  /* stage index of the first stage run (resume) */
  int32_t n_stages;
  int32_t steps_per_stage;
  int32_t n_threads;
  int64_t first_chain;  /* Philox chain id of chain 0 (to recompute any subset of a larger run) */
  int64_t group_size;   /* island restart: 0 (or >= n_chains) restarts every chain from the global
                           best (Table 1); G restarts each group of G consecutive chains from the
                           best of that group (the grouped reduction suggested in §4) */
} ora_run_args;

typedef struct {
  const ora_problem *p;
  const ora_run_args *args;
  int64_t chain_lo, chain_hi;
  int64_t stage;
  double T;
  int8_t *x_cur, *x_best;  /* [n_chains*P] */
  int64_t *c_cur, *c_best; /* [n_chains] */
  uint64_t accepted, uphill, neutral, infeasible;
} ora_worker;

static void *run_chains_of_stage(void *arg) {
  ora_worker *w = (ora_worker *)arg;
  const ora_problem *p = w->p;
  const int64_t P = ora_n_params(p);
  const int64_t L = w->args->steps_per_stage;
  int8_t *cand = (int8_t *)malloc((size_t)P);
  for (int64_t n = w->chain_lo; n < w->chain_hi; ++n) {
    int8_t *xc = w->x_cur + n * P;
    int8_t *xb = w->x_best + n * P;
    for (int64_t it = 0; it < L; ++it) {
      uint64_t g = (uint64_t)(w->stage * L + it);
      uint64_t u[4];
      ora_draw(w->args->seed, g, (uint64_t)(w->args->first_chain + n), (uint64_t)w->args->net, u);
      int8_t nv;
      int64_t i = ora_propose(p, xc, u, &nv);
      memcpy(cand, xc, (size_t)P);
      cand[i] = nv;
      if (p->hard && ora_violations(p, cand) > 0) {
        /* §2.5.3: constraints are enforced when the candidate is drawn; a
         * candidate that breaks one is a rejected step (no redraw) */
        w->infeasible++;
        continue;
      }
      int64_t c_cand = ora_cost(p, cand);
      int64_t delta = c_cand - w->c_cur[n];
      uint32_t r = (uint32_t)(u[2] >> 32);
      int accept = delta <= 0 || r < ora_threshold(w->T, delta);
      if (!accept) continue;
      w->accepted++;
      if (delta > 0) w->uphill++;
      if (delta == 0) w->neutral++;
      memcpy(xc, cand, (size_t)P);
      w->c_cur[n] = c_cand;
      if (c_cand < w->c_best[n]) {
        memcpy(xb, cand, (size_t)P);
        w->c_best[n] = c_cand;
      }
    }
  }
  free(cand);
  return NULL;
}

/* Returns 0 on success, -1 if a starting vector breaks a constraint in hard
 * mode.  Outputs (any may be NULL):
 *   x_out[P], cost_out, winner_out: global best of the last stage (lowest
 *   chain id on ties), before the restart;
 *   stage_best[S], stage_winner[S], stage_accepted[S], stage_uphill[S],
 *   stage_neutral[S], stage_infeasible[S]: per stage, before the restart;
 *   chain_best[n_chains], chain_xbest[n_chains*P]: every chain's best after
 *   the last stage, before the restart. */
int ora_run(const ora_problem *p, const ora_run_args *args, const int8_t *x0,
            int8_t *x_out, int64_t *cost_out, int64_t *winner_out,
            int64_t *stage_best, int64_t *stage_winner, uint64_t *stage_accepted,
            uint64_t *stage_uphill, uint64_t *stage_neutral, uint64_t *stage_infeasible,
            int64_t *chain_best, int8_t *chain_xbest) {
  const int64_t P = ora_n_params(p);
  const int64_t n = args->n_chains;
  int8_t *x_cur = (int8_t *)malloc((size_t)(n * P));
  int8_t *x_best = (int8_t *)malloc((size_t)(n * P));
  int64_t *c_cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  int64_t *c_best = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  memcpy(x_cur, x0, (size_t)(n * P));
  memcpy(x_best, x0, (size_t)(n * P));
  int status = 0;
  for (int64_t c = 0; c < n; ++c) {
    if (p->hard && ora_violations(p, x0 + c * P) > 0) status = -1;
    c_cur[c] = c_best[c] = ora_cost(p, x0 + c * P);
  }
  int n_threads = args->n_threads > 0 ? args->n_threads : 1;
  if (n_threads > n) n_threads = (int)n;
  ora_worker *workers = (ora_worker *)calloc((size_t)n_threads, sizeof(ora_worker));
  pthread_t *tids = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  int64_t winner = 0;
  const int64_t G = args->group_size > 0 && args->group_size < n ? args->group_size : n;
  int8_t *xw = (int8_t *)malloc((size_t)P);
  int8_t *x_glob = (int8_t *)malloc((size_t)P);
  int64_t c_glob = 0;
  for (int32_t s = 0; s < args->n_stages && status == 0; ++s) {
    int64_t k = (int64_t)args->first_stage + s;
    double T = ora_stage_temperature(args->T0, args->rho, k);
    for (int t = 0; t < n_threads; ++t) {
      ora_worker *w = &workers[t];
      memset(w, 0, sizeof(*w));
      w->p = p; w->args = args; w->stage = k; w->T = T;
      w->chain_lo = n * t / n_threads;
      w->chain_hi = n * (t + 1) / n_threads;
      w->x_cur = x_cur; w->x_best = x_best; w->c_cur = c_cur; w->c_best = c_best;
      if (n_threads == 1)
        run_chains_of_stage(w);
      else
        pthread_create(&tids[t], NULL, run_chains_of_stage, w);
    }
    uint64_t acc = 0, up = 0, neu = 0, inf = 0;
    for (int t = 0; t < n_threads; ++t) {
      if (n_threads > 1) pthread_join(tids[t], NULL);
      acc += workers[t].accepted; up += workers[t].uphill;
      neu += workers[t].neutral; inf += workers[t].infeasible;
    }
    /* Table 1, serial part: global minimum over all chains (lowest chain id
     * on ties); it is the stage's result. */
    winner = 0;
    for (int64_t c = 1; c < n; ++c)
      if (c_best[c] < c_best[winner]) winner = c;
    if (stage_best) stage_best[s] = c_best[winner];
    if (stage_winner) stage_winner[s] = winner;
    if (stage_accepted) stage_accepted[s] = acc;
    if (stage_uphill) stage_uphill[s] = up;
    if (stage_neutral) stage_neutral[s] = neu;
    if (stage_infeasible) stage_infeasible[s] = inf;
    if (s == args->n_stages - 1) {
      if (chain_best) memcpy(chain_best, c_best, sizeof(int64_t) * (size_t)n);
      if (chain_xbest) memcpy(chain_xbest, x_best, (size_t)(n * P));
    }
    memcpy(x_glob, x_best + winner * P, (size_t)P);
    c_glob = c_best[winner];
    /* Restart: every chain from its group's best (lowest chain id on ties
     * within the group); one group of all chains is Table 1's global restart. */
    for (int64_t g0 = 0; g0 < n; g0 += G) {
      const int64_t g1 = g0 + G < n ? g0 + G : n;
      int64_t gw = g0;
      for (int64_t c = g0 + 1; c < g1; ++c)
        if (c_best[c] < c_best[gw]) gw = c;
      const int64_t cw = c_best[gw];
      memcpy(xw, x_best + gw * P, (size_t)P);
      for (int64_t c = g0; c < g1; ++c) {
        memcpy(x_cur + c * P, xw, (size_t)P);
        memcpy(x_best + c * P, xw, (size_t)P);
        c_cur[c] = c_best[c] = cw;
      }
    }
  }
  free(xw);
  if (status == 0) {
    if (x_out) memcpy(x_out, args->n_stages > 0 ? x_glob : x_best, (size_t)P);
    if (cost_out) *cost_out = args->n_stages > 0 ? c_glob : c_best[0];
    if (winner_out) *winner_out = winner;
  }
  free(x_glob);
  free(workers); free(tids);
  free(x_cur); free(x_best); free(c_cur); free(c_best);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive search over all 3^P vectors (tiny networks only).             */
/* Candidate m has parameter i equal to the base-3 digit i of m (least       */
/* significant first), read as a code: a = code - 1, theta = code.           */
/* Returns the minimum cost; writes the first minimiser and the number of    */
/* minimisers; costs[3^P] (optional) receives every cost.                    */
/* ------------------------------------------------------------------------ */
/* Ternary model only (model 0): returns -1 for any other model. */
int64_t ora_brute_force(const ora_problem *p, int8_t *argmin_x, int64_t *n_minima, int64_t *costs) {
  if (p->model != 0) return -1;
  const int64_t P = ora_n_params(p);
  int64_t total = 1;
  for (int64_t i = 0; i < P; ++i) total *= 3;
  int8_t *x = (int8_t *)malloc((size_t)P);
  int64_t best = INT64_MAX, count = 0;
  for (int64_t m = 0; m < total; ++m) {
    int64_t rest = m;
    for (int64_t i = 0; i < P; ++i) {
      int code = (int)(rest % 3);
      rest /= 3;
      x[i] = (int8_t)(i < p->n_edges ? code - 1 : code);
    }
    int64_t c = ora_cost(p, x);
    if (costs) costs[m] = c;
    if (c < best) {
      best = c;
      count = 1;
      if (argmin_x) memcpy(argmin_x, x, (size_t)P);
    } else if (c == best) {
      ++count;
    }
  }
  free(x);
  if (n_minima) *n_minima = count;
  return best;
}
