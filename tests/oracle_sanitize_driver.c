/*
 * Test driver for running the CPU oracle under the compilers' address,
 * undefined-behaviour and thread sanitizers (test infrastructure only).
 *
 * Reads one problem and a work list from a whitespace-separated text file
 * (written by tests/test_oracle_sanitizers.py), calls the oracle's entry
 * points and prints their results, one per line, for the test to compare with
 * the same calls made through the oracle's Python binding.
 *
 * Input, in order:
 *   N E C T K O step_size hard penalty model
 *   row_ptr[N+1] src[E] init[C*N] clamp[C*N] obs_t[K] obs_n[O] observed[C*K*O]
 *   n_vec, then n_vec parameter vectors of P values
 *   n_chains seed T0 rho n_stages steps_per_stage n_threads group_size
 *   x0[n_chains*P]
 *   brute (0 or 1: run the exhaustive search as well)
 * Output lines:
 *   vec <cost> <mismatch> <violations> <trajectory checksum>
 *   run <status> <cost> <winner>
 *   stage <best> <winner> <accepted> <uphill> <neutral> <infeasible>
 *   chain <best>
 *   xbest <P values of the run's best vector>
 *   brute <min cost> <number of minima>
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
  int32_t n_nodes, n_edges;
  const int32_t *row_ptr;
  const int32_t *src;
  int32_t n_cond;
  const int8_t *init;
  const int8_t *clamp;
  int32_t n_steps;
  int32_t n_obs_t;
  const int32_t *obs_t;
  int32_t n_obs_n;
  const int32_t *obs_n;
  const int8_t *observed;
  int32_t step_size;
  int32_t hard;
  int64_t penalty;
  int32_t model;
} ora_problem;

typedef struct {
  int64_t n_chains;
  uint64_t seed;
  int32_t net;
  double T0, rho;
  int32_t first_stage, n_stages, steps_per_stage, n_threads;
  int64_t first_chain;
  int64_t group_size;
} ora_run_args;

int64_t ora_n_params(const ora_problem *p);
void ora_simulate(const ora_problem *p, const int8_t *x, int8_t *traj);
int64_t ora_mismatch(const ora_problem *p, const int8_t *x);
int32_t ora_violations(const ora_problem *p, const int8_t *x);
int64_t ora_cost(const ora_problem *p, const int8_t *x);
int ora_run(const ora_problem *p, const ora_run_args *args, const int8_t *x0, int8_t *x_out, int64_t *cost_out,
            int64_t *winner_out, int64_t *stage_best, int64_t *stage_winner, uint64_t *stage_accepted,
            uint64_t *stage_uphill, uint64_t *stage_neutral, uint64_t *stage_infeasible, int64_t *chain_best,
            int8_t *chain_xbest);
int64_t ora_brute_force(const ora_problem *p, int8_t *argmin_x, int64_t *n_minima, int64_t *costs);

static FILE *in;

static int64_t next_int(void) {
  long long v;
  if (fscanf(in, "%lld", &v) != 1) {
    fprintf(stderr, "input ended early\n");
    exit(2);
  }
  return (int64_t)v;
}

static double next_double(void) {
  double v;
  if (fscanf(in, "%lf", &v) != 1) {
    fprintf(stderr, "input ended early\n");
    exit(2);
  }
  return v;
}

static int32_t *read_i32(int64_t n) {
  int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) a[i] = (int32_t)next_int();
  return a;
}

static int8_t *read_i8(int64_t n) {
  int8_t *a = (int8_t *)malloc((size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; ++i) a[i] = (int8_t)next_int();
  return a;
}

int main(int argc, char **argv) {
  if (argc != 2 || !(in = fopen(argv[1], "r"))) {
    fprintf(stderr, "usage: %s <input file>\n", argv[0]);
    return 2;
  }
  ora_problem p;
  p.n_nodes = (int32_t)next_int();
  p.n_edges = (int32_t)next_int();
  p.n_cond = (int32_t)next_int();
  p.n_steps = (int32_t)next_int();
  p.n_obs_t = (int32_t)next_int();
  p.n_obs_n = (int32_t)next_int();
  p.step_size = (int32_t)next_int();
  p.hard = (int32_t)next_int();
  p.penalty = next_int();
  p.model = (int32_t)next_int();
  const int64_t N = p.n_nodes, E = p.n_edges, C = p.n_cond, K = p.n_obs_t, O = p.n_obs_n;
  int32_t *row_ptr = read_i32(N + 1), *src = read_i32(E);
  int8_t *init = read_i8(C * N), *clamp = read_i8(C * N);
  int32_t *obs_t = read_i32(K), *obs_n = read_i32(O);
  int8_t *observed = read_i8(C * K * O);
  p.row_ptr = row_ptr;
  p.src = src;
  p.init = init;
  p.clamp = clamp;
  p.obs_t = obs_t;
  p.obs_n = obs_n;
  p.observed = observed;
  const int64_t P = ora_n_params(&p);

  const int64_t n_vec = next_int();
  int8_t *vecs = read_i8(n_vec * P);
  int8_t *traj = (int8_t *)malloc((size_t)(C * (p.n_steps + 1) * N));
  for (int64_t v = 0; v < n_vec; ++v) {
    const int8_t *x = vecs + v * P;
    ora_simulate(&p, x, traj);
    int64_t sum = 0;
    for (int64_t i = 0; i < C * (p.n_steps + 1) * N; ++i) sum += (i % 9973 + 1) * (int64_t)traj[i];
    printf("vec %lld %lld %d %lld\n", (long long)ora_cost(&p, x), (long long)ora_mismatch(&p, x),
           (int)ora_violations(&p, x), (long long)sum);
  }

  ora_run_args a;
  a.n_chains = next_int();
  a.seed = (uint64_t)next_int();
  a.T0 = next_double();
  a.rho = next_double();
  a.n_stages = (int32_t)next_int();
  a.steps_per_stage = (int32_t)next_int();
  a.n_threads = (int32_t)next_int();
  a.group_size = next_int();
  a.net = 0;
  a.first_stage = 0;
  a.first_chain = 0;
  int8_t *x0 = read_i8(a.n_chains * P);
  const int64_t S = a.n_stages;
  int8_t *x_out = (int8_t *)malloc((size_t)P);
  int64_t cost = 0, winner = 0;
  int64_t *stage_best = (int64_t *)malloc(sizeof(int64_t) * (size_t)S);
  int64_t *stage_winner = (int64_t *)malloc(sizeof(int64_t) * (size_t)S);
  uint64_t *acc = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)S), *up = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)S);
  uint64_t *neu = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)S), *inf = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)S);
  int64_t *chain_best = (int64_t *)malloc(sizeof(int64_t) * (size_t)a.n_chains);
  int8_t *chain_xbest = (int8_t *)malloc((size_t)(a.n_chains * P));
  const int status = ora_run(&p, &a, x0, x_out, &cost, &winner, stage_best, stage_winner, acc, up, neu, inf,
                             chain_best, chain_xbest);
  printf("run %d %lld %lld\n", status, (long long)cost, (long long)winner);
  for (int64_t s = 0; s < S; ++s)
    printf("stage %lld %lld %llu %llu %llu %llu\n", (long long)stage_best[s], (long long)stage_winner[s],
           (unsigned long long)acc[s], (unsigned long long)up[s], (unsigned long long)neu[s],
           (unsigned long long)inf[s]);
  for (int64_t c = 0; c < a.n_chains; ++c) printf("chain %lld\n", (long long)chain_best[c]);
  printf("xbest");
  for (int64_t i = 0; i < P; ++i) printf(" %d", (int)x_out[i]);
  printf("\n");

  if (next_int()) {
    int8_t *argmin = (int8_t *)malloc((size_t)P);
    int64_t n_min = 0;
    const int64_t best = ora_brute_force(&p, argmin, &n_min, NULL);
    printf("brute %lld %lld\n", (long long)best, (long long)n_min);
    free(argmin);
  }

  free(row_ptr);
  free(src);
  free(init);
  free(clamp);
  free(obs_t);
  free(obs_n);
  free(observed);
  free(vecs);
  free(traj);
  free(x0);
  free(x_out);
  free(stage_best);
  free(stage_winner);
  free(acc);
  free(up);
  free(neu);
  free(inf);
  free(chain_best);
  free(chain_xbest);
  fclose(in);
  return 0;
}
