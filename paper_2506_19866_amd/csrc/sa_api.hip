// sa_api.hip -- host part of the C ABI declared in include/sa_anneal.h:
// validation, problem staging (weights, lambda, register layout of the
// kernels), fixed-point Metropolis tables and stage orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sa_anneal.h"
#include "sa_internal.h"
#include "sa_mlp.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? SA_ERR_OOM : SA_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SA_HIP(call, what)                    \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Bump allocator over one device buffer (each array 256-byte aligned).
struct Layout {
  size_t bytes = 0;
  size_t take(size_t n) {
    size_t at = bytes;
    bytes += (n + 255) & ~size_t(255);
    return at;
  }
};

}  // namespace

struct sa_problem {
  int device = 0;
  sa_problem_info info{};
  sa::DevProblem dev{};
  void *dmem = nullptr;
};

struct sa_run {
  std::vector<sa_problem *> probs;
  sa_run_desc desc{};
  int device = 0;
  int64_t n = 0;                 // chains per problem
  bool persistent = false;       // many-network kernel (else the specialised one)
  int waves = 4;                 // chains per work item (persistent kernel)
  int cus = 256;
  std::vector<int> blocks_per_cu;  // per launch group
  std::vector<int64_t> x_off, w_off;
  // launch groups of the persistent kernel: (size class, step size)
  std::vector<int> item_class_begin, item_class_count, item_class_d, item_class_cls;
  std::vector<size_t> class_smem;
  int8_t *x0 = nullptr, *xbest = nullptr, *xwin = nullptr;
  int32_t *cbest = nullptr;
  uint32_t *cstats = nullptr, *tau = nullptr, *queue = nullptr;
  sa::StageRecord *rec = nullptr;  // [n_stages][n_probs]
  sa::DevProblem *probs_dev = nullptr;
  int64_t *x_off_dev = nullptr, *w_off_dev = nullptr;
  int32_t *item_net = nullptr, *item_chain0 = nullptr;
  std::vector<size_t> tau_off;
  std::vector<int32_t> dcap;
  int32_t launched = 0;
  int64_t group = 0;               // chains per restart group (0: Table 1's global restart)
  hipStream_t stream = nullptr;
  std::vector<hipEvent_t> ev_start, ev_stop;  // per stage, when record_times is set
  std::vector<hipGraphExec_t> graphs;
  hipStream_t capture_stream = nullptr;  // private stream the stages are captured on
  // persistent kernel with several launch groups: the groups of a stage run
  // concurrently, group k > 0 on side[k - 1], forked from and joined to the
  // launch stream with events (so one group's drain tail overlaps the others)
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  bool learned = false;                  // learned proposal or trace: the learned-stage kernel
  sa::LearnedArgs la{};                  // its stage-independent part
  std::vector<float> lt;                 // per stage: f32(ln(T_k) / 5)
  uint32_t *ctl = nullptr;               // device {stop word, stages completed}
  const volatile int32_t *abort_host = nullptr;  // the caller's pinned flag, and its device address
  const volatile int32_t *abort_dev = nullptr;
};

struct sa_mlp {
  int device = 0;
  float *master = nullptr, *m = nullptr, *v = nullptr;  // [kMlpParams] each
  uint4 *w1f = nullptr, *w2f = nullptr;                 // bf16 fragments
  float *partial = nullptr, *loss_partial = nullptr;    // [kMlpMaxWaves][kMlpParams], [kMlpMaxWaves]
  int64_t steps = 0;                                    // Adam steps taken
  void *dmem = nullptr;
};

static_assert(sizeof(sa_trace_record) == sizeof(sa::TraceRecord) && sizeof(sa_trace_record) == 80,
              "trace record layout");

extern "C" const char *sa_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// problem staging
// ---------------------------------------------------------------------------
static int validate(const sa_problem_desc *d) {
  if (!d) return fail(SA_ERR_ARG, "desc is NULL");
  const int N = d->n_nodes, E = d->n_edges, C = d->n_conditions, T = d->n_steps;
  const int K = d->n_obs_times, O = d->n_obs_nodes;
  if (N < 1 || E < 0 || C < 1 || T < 1 || K < 1 || O < 1)
    return fail(SA_ERR_ARG, "sizes out of range (N=%d E=%d C=%d T=%d K=%d O=%d)", N, E, C, T, K, O);
  if (!d->in_row_ptr || (E > 0 && !d->in_src) || !d->init_state || !d->clamp || !d->obs_times ||
      !d->obs_nodes || !d->observed)
    return fail(SA_ERR_ARG, "a required array is NULL");
  if (d->model != SA_MODEL_SYNCHRONOUS && d->model != SA_MODEL_PRIORITY)
    return fail(SA_ERR_ARG, "unknown model %d", d->model);
  if (d->model == SA_MODEL_SYNCHRONOUS && d->step_size != 1 && d->step_size != 2)
    return fail(SA_ERR_DOMAIN, "step_size must be 1 or 2");
  if (d->model == SA_MODEL_PRIORITY && N > 64)
    return fail(SA_ERR_UNSUPPORTED, "priority model: n_nodes %d > 64", N);
  if (d->constraint_mode != SA_HARD && d->constraint_mode != SA_PENALTY)
    return fail(SA_ERR_ARG, "unknown constraint_mode %d", d->constraint_mode);
  if (d->penalty < 0) return fail(SA_ERR_DOMAIN, "penalty must be >= 0");
  if (d->in_row_ptr[0] != 0 || d->in_row_ptr[N] != E)
    return fail(SA_ERR_TOPOLOGY, "in_row_ptr must start at 0 and end at n_edges");
  for (int i = 0; i < N; ++i) {
    if (d->in_row_ptr[i + 1] < d->in_row_ptr[i]) return fail(SA_ERR_TOPOLOGY, "in_row_ptr not monotone at %d", i);
    for (int e = d->in_row_ptr[i]; e < d->in_row_ptr[i + 1]; ++e) {
      const int j = d->in_src[e];
      if (j < 0 || j >= N) return fail(SA_ERR_TOPOLOGY, "edge %d: source %d out of range", e, j);
      if (j == i) return fail(SA_ERR_TOPOLOGY, "edge %d: self-loop on node %d", e, i);
      if (e > d->in_row_ptr[i] && d->in_src[e - 1] >= j)
        return fail(SA_ERR_TOPOLOGY, "edge %d: sources of node %d not strictly ascending", e, i);
    }
  }
  for (int i = 0; i < C * N; ++i) {
    if (d->init_state[i] < 0 || d->init_state[i] > 2) return fail(SA_ERR_DOMAIN, "init_state[%d] = %d", i, d->init_state[i]);
    if (d->clamp[i] < -1 || d->clamp[i] > 2) return fail(SA_ERR_DOMAIN, "clamp[%d] = %d", i, d->clamp[i]);
  }
  for (int k = 0; k < K; ++k) {
    if (d->obs_times[k] < 0 || d->obs_times[k] > T) return fail(SA_ERR_DOMAIN, "obs_times[%d] out of [0, T]", k);
    if (k > 0 && d->obs_times[k] <= d->obs_times[k - 1]) return fail(SA_ERR_DOMAIN, "obs_times not increasing");
  }
  std::vector<char> seen(N, 0);
  for (int o = 0; o < O; ++o) {
    const int v = d->obs_nodes[o];
    if (v < 0 || v >= N) return fail(SA_ERR_DOMAIN, "obs_nodes[%d] = %d out of range", o, v);
    if (seen[v]) return fail(SA_ERR_DOMAIN, "obs_nodes repeats node %d", v);
    seen[v] = 1;
  }
  for (long i = 0; i < (long)C * K * O; ++i)
    if (d->observed[i] < 0 || d->observed[i] > 2) return fail(SA_ERR_DOMAIN, "observed[%ld] = %d", i, d->observed[i]);
  if (d->constraint_mode == SA_HARD) {
    std::vector<int> outdeg(N, 0);
    for (int e = 0; e < E; ++e) outdeg[d->in_src[e]]++;
    for (int i = 0; i < N; ++i)
      if (d->in_row_ptr[i + 1] == d->in_row_ptr[i] || outdeg[i] == 0)
        return fail(SA_ERR_TOPOLOGY, "node %d lacks an in- or out-edge: constraints (a)/(b) cannot hold", i);
  }
  return SA_OK;
}

// The priority model's tables (sa_priority.h): per condition the start state
// of every lane of a chain's segment, per (condition, step) the reference byte.
static int create_priority(const sa_problem_desc *d, const std::vector<int> &W, long long wsum, long long lambda,
                           long long max_cost, sa_problem **out) {
  const int N = d->n_nodes, E = d->n_edges, C = d->n_conditions, T = d->n_steps;
  const int K = d->n_obs_times, O = d->n_obs_nodes, P = 3 * E + 3 * N;
  const int lc = N <= 16 ? 16 : N <= 32 ? 32 : 64;
  int max_in = 0;
  for (int i = 0; i < N; ++i) max_in = std::max(max_in, d->in_row_ptr[i + 1] - d->in_row_ptr[i]);
  // 16- and 32-lane segments (several chains per wave) gather regulator
  // states by ballots, which keep lane permutes off the time step's critical
  // path; one chain per wave takes the per-slot tables unless a node has more
  // than 16 in-edges
  const int dmax = lc <= 32 ? 0 : max_in <= 8 ? 8 : max_in <= 16 ? 16 : 0;
  std::vector<uint8_t> start((size_t)C * lc);
  std::vector<uint32_t> obs((size_t)C * (T + 1) * lc, 0);
  for (int c = 0; c < C; ++c)
    for (int v = 0; v < lc; ++v) {
      int val = 0, held = 1;
      if (v < N) {
        const int cl = d->clamp[(size_t)c * N + v];
        held = cl >= 0;
        val = held ? cl : d->init_state[(size_t)c * N + v];
      }
      start[(size_t)c * lc + v] = (uint8_t)(val | held << 2);
    }
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < K; ++k)
      for (int o = 0; o < O; ++o) {
        const size_t at = ((size_t)c * K + k) * O + o;
        uint32_t cost = 0;
        for (int v = 0; v < 3; ++v) cost |= (uint32_t)(W[at] * std::abs(v - d->observed[at])) << (8 * v);
        obs[((size_t)c * (T + 1) + d->obs_times[k]) * lc + d->obs_nodes[o]] = cost;
      }
  std::vector<int32_t> esrc(E), edst(E);
  for (int i = 0; i < N; ++i)
    for (int e = d->in_row_ptr[i]; e < d->in_row_ptr[i + 1]; ++e) {
      esrc[e] = d->in_src[e];
      edst[e] = i;
    }

  auto *pr = new sa_problem();
  hipGetDevice(&pr->device);
  Layout lay;
  const size_t o_esrc = lay.take((size_t)E * 4), o_edst = lay.take((size_t)E * 4);
  const size_t o_inptr = lay.take((size_t)(N + 1) * 4);
  const size_t o_start = lay.take(start.size()), o_obs = lay.take(obs.size() * 4);
  hipError_t e = hipMalloc(&pr->dmem, lay.bytes);
  if (e != hipSuccess) {
    delete pr;
    return hip_fail(e, "hipMalloc(problem)");
  }
  std::vector<char> host(lay.bytes, 0);
  auto put = [&](size_t off, const void *src, size_t n) {
    if (n) memcpy(host.data() + off, src, n);
  };
  put(o_esrc, esrc.data(), (size_t)E * 4);
  put(o_edst, edst.data(), (size_t)E * 4);
  put(o_inptr, d->in_row_ptr, (size_t)(N + 1) * 4);
  put(o_start, start.data(), start.size());
  put(o_obs, obs.data(), obs.size() * 4);
  e = hipMemcpy(pr->dmem, host.data(), lay.bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(pr->dmem);
    delete pr;
    return hip_fail(e, "hipMemcpy(problem)");
  }
  const char *base = (const char *)pr->dmem;
  sa::DevProblem &dp = pr->dev;
  dp.N = N; dp.E = E; dp.P = P; dp.C = C; dp.T = T; dp.K = K; dp.O = O;
  dp.hard = d->constraint_mode == SA_HARD;
  dp.lambda = (int32_t)lambda;
  dp.sum_w = (int32_t)wsum;
  dp.edge_src = (const int32_t *)(base + o_esrc);
  dp.edge_dst = (const int32_t *)(base + o_edst);
  dp.in_ptr = (const int32_t *)(base + o_inptr);
  dp.model = SA_MODEL_PRIORITY;
  dp.lc = lc;
  dp.dmax = dmax;
  dp.pr_start = (const uint8_t *)(base + o_start);
  dp.pr_obs = (const uint32_t *)(base + o_obs);

  sa_problem_info &in = pr->info;
  in.n_params = P; in.n_nodes = N; in.n_edges = E; in.n_conditions = C; in.n_steps = T;
  in.n_obs_times = K; in.n_obs_nodes = O;
  in.weight_sum = (int32_t)wsum;
  in.penalty = (int32_t)lambda;
  in.max_cost = (int32_t)max_cost;
  in.clamps_by_offset = 0;
  in.obs_dwords = 0;
  *out = pr;
  return SA_OK;
}

extern "C" int sa_create_problem(const sa_problem_desc *d, sa_problem **out) {
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  *out = nullptr;
  int rc = validate(d);
  if (rc != SA_OK) return rc;
  const int N = d->n_nodes, E = d->n_edges, C = d->n_conditions, T = d->n_steps;
  const int K = d->n_obs_times, O = d->n_obs_nodes, P = N + E;

  // gradient weights (§2.3): 1 at the first observed time, else 1 + |R_k - R_{k-1}|
  std::vector<int> W((size_t)C * K * O);
  long long wsum = 0;
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < K; ++k)
      for (int o = 0; o < O; ++o) {
        const size_t at = ((size_t)c * K + k) * O + o;
        const int w = k == 0 ? 1 : 1 + std::abs(d->observed[at] - d->observed[at - O]);
        W[at] = w;
        wsum += w;
      }
  const long long lambda = d->penalty > 0 ? d->penalty : 1 + 2 * wsum;
  const long long max_cost = 2 * wsum + lambda * 2 * (long long)N;
  if (max_cost >= (1ll << 31) - 1) return fail(SA_ERR_OVERFLOW, "largest cost %lld does not fit int32", max_cost);
  if (d->model == SA_MODEL_PRIORITY) return create_priority(d, W, wsum, lambda, max_cost, out);

  // tiles: nm m-tiles of 16 rows hold the nodes, nk k-fragments of 128
  // columns (32 slots per lane group) hold nodes + bias; layouts with two
  // fragments start at 9 m-tiles
  const int nk = N / 128 + 1;
  int nm = (N + 15) / 16;
  if (nk == 2 && nm < 9) nm = 9;
  if (N > 191 || nm > sa::kMaxTilesM) return fail(SA_ERR_UNSUPPORTED, "n_nodes %d > 191", N);
  const int CG = (C + 15) / 16;
  if (CG > sa::kMaxCondGroups) return fail(SA_ERR_UNSUPPORTED, "n_conditions %d > 64", C);

  // slots: observed nodes first (their states then sit in the first dwords of
  // every lane), round-robin over the four lane groups; bias after the nodes.
  // Clamped nodes go before them when that puts every clamped node in the
  // first dword of every lane without lengthening the observed dwords and
  // every clamp value is 0 or 2: the plain kernels (specialised and
  // many-network) then hold them by accumulator offsets of the first two
  // m-tiles (DevProblem::cofs) and need no per-dword select.
  std::vector<int> order, obs_index(N, -1);
  for (int o = 0; o < O; ++o) obs_index[d->obs_nodes[o]] = o;
  std::vector<char> clamped(N, 0);
  bool values_02 = true;
  for (int c = 0; c < C; ++c)
    for (int v = 0; v < N; ++v) {
      const int cl = d->clamp[(size_t)c * N + v];
      clamped[v] |= cl >= 0;
      values_02 = values_02 && cl != 1;
    }
  int n_clamped = 0, n_clamped_unobs = 0;
  for (int v = 0; v < N; ++v) {
    n_clamped += clamped[v];
    n_clamped_unobs += clamped[v] && obs_index[v] < 0;
  }
  const bool hold_by_offset = values_02 && n_clamped <= 32 &&
                              (n_clamped_unobs + O + 31) / 32 <= std::max(1, (O + 31) / 32);
  if (hold_by_offset) {
    // unobserved clamped, observed clamped, observed, the rest
    for (int v = 0; v < N; ++v)
      if (clamped[v] && obs_index[v] < 0) order.push_back(v);
    for (int o = 0; o < O; ++o)
      if (clamped[d->obs_nodes[o]]) order.push_back(d->obs_nodes[o]);
    for (int o = 0; o < O; ++o)
      if (!clamped[d->obs_nodes[o]]) order.push_back(d->obs_nodes[o]);
    for (int v = 0; v < N; ++v)
      if (!clamped[v] && obs_index[v] < 0) order.push_back(v);
  } else {
    for (int o = 0; o < O; ++o) order.push_back(d->obs_nodes[o]);
    for (int v = 0; v < N; ++v)
      if (obs_index[v] < 0) order.push_back(v);
  }
  std::vector<int> sg(N), sq(N);
  const int slots = 32 * nk;
  std::vector<int16_t> slot_node((size_t)4 * slots, -1);
  for (int k = 0; k < N; ++k) {
    const int v = order[k];
    sg[v] = k % 4;
    sq[v] = k / 4;
    slot_node[(size_t)sg[v] * slots + sq[v]] = (int16_t)v;
  }
  const int gb = N % 4, qb = N / 4;
  int nd = 1;
  for (int o = 0; o < O; ++o) nd = std::max(nd, sq[d->obs_nodes[o]] / 8 + 1);

  // A entry of parameter p: row of its target node i, column of its source
  // node j (edge) or of the bias (theta_i)
  std::vector<uint32_t> param_pos(P);
  std::vector<int32_t> edst(E), esrc(E);
  auto place = [&](int p, int i, int colg, int colq) {
    const int lane = (4 * sg[i] + sq[i] % 4) + 16 * colg;
    const int mt = sq[i] / 4, kf = colq / 32, dw = (colq % 32) / 8, n = colq % 8;
    param_pos[p] = (uint32_t)lane | ((uint32_t)mt << 8) | ((uint32_t)kf << 12) | ((uint32_t)dw << 14) |
                   ((uint32_t)n << 16);
  };
  for (int i = 0; i < N; ++i)
    for (int e = d->in_row_ptr[i]; e < d->in_row_ptr[i + 1]; ++e) {
      const int j = d->in_src[e];
      edst[e] = i;
      esrc[e] = j;
      place(e, i, sg[j], sq[j]);
    }
  for (int i = 0; i < N; ++i) place(E + i, i, gb, qb);

  std::vector<int32_t> out_ptr(N + 1, 0), out_eid(E);
  for (int e = 0; e < E; ++e) out_ptr[esrc[e] + 1]++;
  for (int i = 0; i < N; ++i) out_ptr[i + 1] += out_ptr[i];
  {
    std::vector<int32_t> fill(out_ptr.begin(), out_ptr.end() - 1);
    for (int e = 0; e < E; ++e) out_eid[fill[esrc[e]]++] = e;
  }

  // accumulator offsets of m-tiles 0 and 1: [CG][2][64 lanes][4] (row 4g + r
  // of m-tile mt in lane group g is slot q = 4 mt + r)
  std::vector<float> cofs((size_t)CG * 2 * 64 * 4, 0.f);
  for (int cg = 0; cg < CG && hold_by_offset; ++cg)
    for (int mt = 0; mt < std::min(nm, 2); ++mt)
      for (int lane = 0; lane < 64; ++lane) {
        const int c = cg * 16 + lane % 16, g = lane / 16;
        for (int r = 0; r < 4; ++r) {
          const int v = slot_node[(size_t)g * slots + 4 * mt + r];
          if (c >= C || v < 0) continue;
          const int cl = d->clamp[(size_t)c * N + v];
          cofs[(((size_t)cg * 2 + mt) * 64 + lane) * 4 + r] = cl == 2 ? 16384.f : cl == 0 ? -16384.f : 0.f;
        }
      }

  // per (condition group, dword, lane): initial states and the held-byte mask
  const int Q4 = 4 * nk;
  std::vector<uint32_t> b0((size_t)CG * Q4 * 64), cm((size_t)CG * Q4 * 64);
  std::vector<uint32_t> orr((size_t)CG * K * nd * 64, 0), ow((size_t)CG * K * nd * 64, 0);
  for (int cg = 0; cg < CG; ++cg)
    for (int lane = 0; lane < 64; ++lane) {
      const int c = cg * 16 + lane % 16, g = lane / 16;
      for (int q4 = 0; q4 < Q4; ++q4) {
        uint32_t vb = 0, vm = 0;
        for (int b = 0; b < 8; ++b) {
          const int q = q4 * 8 + b;
          const int v = slot_node[(size_t)g * slots + q];
          int val = 0, held = 1;
          if (c < C && g == gb && q == qb) {
            val = 1;  // constant bias input
          } else if (c < C && v >= 0) {
            const int cl = d->clamp[(size_t)c * N + v];
            if (cl >= 0) {
              val = cl;
            } else {
              val = d->init_state[(size_t)c * N + v];
              held = 0;
            }
          }
          vb |= sa::state_code(val) << (4 * b);
          vm |= (held ? 0xfu : 0u) << (4 * b);
        }
        const size_t at = ((size_t)cg * Q4 + q4) * 64 + lane;
        b0[at] = vb;
        cm[at] = vm;
      }
      if (c >= C) continue;
      for (int k = 0; k < K; ++k)
        for (int q4 = 0; q4 < nd; ++q4) {
          uint32_t vr = 0, vw = 0;
          for (int b = 0; b < 8; ++b) {
            const int v = slot_node[(size_t)g * slots + q4 * 8 + b];
            if (v < 0 || obs_index[v] < 0) continue;
            const size_t at = ((size_t)c * K + k) * O + obs_index[v];
            vr |= sa::state_code(d->observed[at]) << (4 * b);
            vw |= (uint32_t)W[at] << (4 * b);
          }
          const size_t at = (((size_t)cg * K + k) * nd + q4) * 64 + lane;
          orr[at] = vr;
          ow[at] = vw;
        }
    }

  // learned proposal: per-node slot and observation sums, per-parameter descriptor
  std::vector<int16_t> node_slot(N);
  std::vector<int32_t> node_sw(N, 0), node_wr(N, 0), indeg(N), outdeg(N);
  for (int v = 0; v < N; ++v) {
    node_slot[v] = (int16_t)(sg[v] * slots + sq[v]);
    indeg[v] = d->in_row_ptr[v + 1] - d->in_row_ptr[v];
    outdeg[v] = out_ptr[v + 1] - out_ptr[v];
  }
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < K; ++k)
      for (int o = 0; o < O; ++o) {
        const size_t at = ((size_t)c * K + k) * O + o;
        node_sw[d->obs_nodes[o]] += W[at];
        node_wr[d->obs_nodes[o]] += W[at] * d->observed[at];
      }
  std::vector<uint32_t> param_info(P);
  for (int p = 0; p < P; ++p) {
    const bool edge = p < E;
    const int i = edge ? edst[p] : p - E, j = edge ? esrc[p] : 0;
    param_info[p] = (uint32_t)(i & 127) | (uint32_t)(j & 127) << 7 | (uint32_t)(std::min(indeg[i], 127)) << 14 |
                    (uint32_t)(edge ? std::min(outdeg[j], 127) : 0) << 21 | (uint32_t)edge << 28 |
                    (uint32_t)(obs_index[i] >= 0) << 29 | (uint32_t)(edge && obs_index[j] >= 0) << 30;
  }

  auto *pr = new sa_problem();
  hipGetDevice(&pr->device);
  Layout lay;
  const size_t o_pos = lay.take(param_pos.size() * 4);
  const size_t o_esrc = lay.take((size_t)E * 4), o_edst = lay.take((size_t)E * 4);
  const size_t o_inptr = lay.take((size_t)(N + 1) * 4), o_outptr = lay.take((size_t)(N + 1) * 4);
  const size_t o_outeid = lay.take((size_t)E * 4);
  const size_t o_b0 = lay.take(b0.size() * 4), o_cm = lay.take(cm.size() * 4), o_cofs = lay.take(cofs.size() * 4);
  const size_t o_or = lay.take(orr.size() * 4), o_ow = lay.take(ow.size() * 4);
  const size_t o_obst = lay.take((size_t)K * 4), o_slot = lay.take(slot_node.size() * 2);
  const size_t o_nslot = lay.take((size_t)N * 2), o_nsw = lay.take((size_t)N * 4), o_nwr = lay.take((size_t)N * 4);
  const size_t o_pinfo = lay.take((size_t)P * 4);
  hipError_t e = hipMalloc(&pr->dmem, lay.bytes);
  if (e != hipSuccess) {
    delete pr;
    return hip_fail(e, "hipMalloc(problem)");
  }
  char *base = (char *)pr->dmem;
  std::vector<char> host(lay.bytes, 0);
  auto put = [&](size_t off, const void *src, size_t n) {
    if (n) memcpy(host.data() + off, src, n);
  };
  put(o_pos, param_pos.data(), param_pos.size() * 4);
  put(o_esrc, esrc.data(), (size_t)E * 4);
  put(o_edst, edst.data(), (size_t)E * 4);
  put(o_inptr, d->in_row_ptr, (size_t)(N + 1) * 4);
  put(o_outptr, out_ptr.data(), (size_t)(N + 1) * 4);
  put(o_outeid, out_eid.data(), (size_t)E * 4);
  put(o_b0, b0.data(), b0.size() * 4);
  put(o_cm, cm.data(), cm.size() * 4);
  put(o_cofs, cofs.data(), cofs.size() * 4);
  put(o_or, orr.data(), orr.size() * 4);
  put(o_ow, ow.data(), ow.size() * 4);
  put(o_obst, d->obs_times, (size_t)K * 4);
  put(o_slot, slot_node.data(), slot_node.size() * 2);
  put(o_nslot, node_slot.data(), (size_t)N * 2);
  put(o_nsw, node_sw.data(), (size_t)N * 4);
  put(o_nwr, node_wr.data(), (size_t)N * 4);
  put(o_pinfo, param_info.data(), (size_t)P * 4);
  e = hipMemcpy(pr->dmem, host.data(), lay.bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(pr->dmem);
    delete pr;
    return hip_fail(e, "hipMemcpy(problem)");
  }

  sa::DevProblem &dp = pr->dev;
  dp.N = N; dp.E = E; dp.P = P; dp.C = C; dp.T = T; dp.K = K; dp.O = O;
  dp.CG = CG; dp.nm = nm; dp.nk = nk; dp.nd = nd;
  dp.d = d->step_size;
  dp.hard = d->constraint_mode == SA_HARD;
  dp.lambda = (int32_t)lambda;
  dp.param_pos = (const uint32_t *)(base + o_pos);
  dp.edge_src = (const int32_t *)(base + o_esrc);
  dp.edge_dst = (const int32_t *)(base + o_edst);
  dp.in_ptr = (const int32_t *)(base + o_inptr);
  dp.out_ptr = (const int32_t *)(base + o_outptr);
  dp.out_eid = (const int32_t *)(base + o_outeid);
  dp.b0 = (const uint32_t *)(base + o_b0);
  dp.cmask = (const uint32_t *)(base + o_cm);
  dp.cofs = (const float *)(base + o_cofs);
  dp.hold_by_offset = hold_by_offset ? 1 : 0;
  dp.obs_r = (const uint32_t *)(base + o_or);
  dp.obs_w = (const uint32_t *)(base + o_ow);
  dp.obs_t = (const int32_t *)(base + o_obst);
  dp.slot_node = (const int16_t *)(base + o_slot);
  dp.sum_w = (int32_t)wsum;
  dp.node_slot = (const int16_t *)(base + o_nslot);
  dp.node_sw = (const int32_t *)(base + o_nsw);
  dp.node_wr = (const int32_t *)(base + o_nwr);
  dp.param_info = (const uint32_t *)(base + o_pinfo);

  sa_problem_info &in = pr->info;
  in.n_params = P; in.n_nodes = N; in.n_edges = E; in.n_conditions = C; in.n_steps = T;
  in.n_obs_times = K; in.n_obs_nodes = O;
  in.weight_sum = (int32_t)wsum;
  in.penalty = (int32_t)lambda;
  in.max_cost = (int32_t)max_cost;
  in.clamps_by_offset = hold_by_offset ? 1 : 0;
  in.obs_dwords = nd;
  *out = pr;
  return SA_OK;
}

extern "C" int sa_destroy_problem(sa_problem *p) {
  if (!p) return SA_OK;
  hipFree(p->dmem);
  delete p;
  return SA_OK;
}

extern "C" int sa_problem_get_info(const sa_problem *p, sa_problem_info *info) {
  if (!p || !info) return fail(SA_ERR_ARG, "NULL argument");
  *info = p->info;
  return SA_OK;
}

extern "C" int sa_eval_cost(const sa_problem *p, const int8_t *x, int64_t n, int32_t *cost, void *stream) {
  if (!p) return fail(SA_ERR_ARG, "problem is NULL");
  if (n < 0) return fail(SA_ERR_ARG, "n < 0");
  if (n == 0) return SA_OK;
  if (!x || !cost) return fail(SA_ERR_ARG, "NULL device pointer");
  SA_HIP(hipSetDevice(p->device), "hipSetDevice");
  if (p->dev.model == SA_MODEL_PRIORITY)
    SA_HIP((hipError_t)sa::launch_priority_eval(p->dev, x, n, cost, stream), "eval launch");
  else
    SA_HIP((hipError_t)sa::launch_eval(p->dev, x, n, cost, stream), "eval launch");
  return SA_OK;
}

extern "C" int sa_simulate(const sa_problem *p, const int8_t *x, int64_t n, int8_t *traj, void *stream) {
  if (!p) return fail(SA_ERR_ARG, "problem is NULL");
  if (n < 0) return fail(SA_ERR_ARG, "n < 0");
  if (n == 0) return SA_OK;
  if (!x || !traj) return fail(SA_ERR_ARG, "NULL device pointer");
  SA_HIP(hipSetDevice(p->device), "hipSetDevice");
  if (p->dev.model == SA_MODEL_PRIORITY)
    SA_HIP((hipError_t)sa::launch_priority_simulate(p->dev, x, n, traj, stream), "simulate launch");
  else
    SA_HIP((hipError_t)sa::launch_simulate(p->dev, x, n, traj, stream), "simulate launch");
  return SA_OK;
}

// ---------------------------------------------------------------------------
// runs
// ---------------------------------------------------------------------------
static int launch_cost(const sa::DevProblem &dp, const int8_t *x, int64_t n, int32_t *cost, hipStream_t s) {
  return dp.model == SA_MODEL_PRIORITY ? sa::launch_priority_eval(dp, x, n, cost, s) : sa::launch_eval(dp, x, n, cost, s);
}

// Domain of element k of a parameter vector (§2.1, §2.2).
static bool in_domain(const sa::DevProblem &dp, int k, int v) {
  const int E = dp.E, N = dp.N;
  if (dp.model != SA_MODEL_PRIORITY) return k < E ? (v >= -1 && v <= 1) : (v >= 0 && v <= 2);
  if (k < E) return v >= 0 && v <= 2;                                        // w
  if (k < 2 * E) return v >= -1 && v <= 1;                                   // p
  if (k < 3 * E) return v == 1 || v == 2;                                    // t
  if (k < 3 * E + N) return (v >= 1 && v <= 6) || (v >= 10 && v <= 12);      // u
  if (k < 3 * E + 2 * N) return v >= 0 && v <= 2;                            // m
  return v == 1 || v == 2;                                                   // d
}
// Metropolis threshold of Table 1 in fixed point: floor(2^32 exp(-D/T)),
// clipped to 2^32 - 1; tabulated for D = 1 .. dcap (the last non-zero).
static void tau_table(double T, int32_t max_delta, std::vector<uint32_t> &tab, int32_t &dcap) {
  tab.assign(1, 0u);
  dcap = 0;
  for (int32_t D = 1; D <= max_delta; ++D) {
    const double v = std::ldexp(std::exp(-(double)D / T), 32);
    const uint32_t t = v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)std::floor(v);
    if (t == 0) break;
    tab.push_back(t);
    dcap = D;
  }
}

static void free_run(sa_run *r) {
  for (hipEvent_t e : r->ev_start) hipEventDestroy(e);
  for (hipEvent_t e : r->ev_stop) hipEventDestroy(e);
  for (hipGraphExec_t g : r->graphs) hipGraphExecDestroy(g);
  if (r->capture_stream) hipStreamDestroy(r->capture_stream);
  for (hipStream_t x : r->side) hipStreamDestroy(x);
  if (r->fork) hipEventDestroy(r->fork);
  for (hipEvent_t x : r->join) hipEventDestroy(x);
  hipFree(r->x0);
  hipFree(r->xbest);
  hipFree(r->xwin);
  hipFree(r->cbest);
  hipFree(r->cstats);
  hipFree(r->tau);
  hipFree(r->queue);
  hipFree(r->rec);
  hipFree(r->probs_dev);
  hipFree(r->x_off_dev);
  hipFree(r->w_off_dev);
  hipFree(r->item_net);
  hipFree(r->item_chain0);
  hipFree(r->ctl);
  delete r;
}

// Work items of the persistent kernel: (network, first chain) with `waves`
// chains each, in launch groups of one size class and one step size (largest
// class first), longest networks first within a group (per-step work
// ~ C * T_s * m-tiles * k-tiles).  Returns the item count.
static int build_items(sa_run *r, int waves, std::vector<int32_t> &net, std::vector<int32_t> &chain0) {
  net.clear();
  chain0.clear();
  r->item_class_begin.clear();
  r->item_class_count.clear();
  r->item_class_d.clear();
  r->item_class_cls.clear();
  r->class_smem.clear();
  const int np = (int)r->probs.size();
  for (int cls = sa::kPersistentClasses - 1; cls >= 0; --cls)
    for (int d = 1; d <= 2; ++d) {
      std::vector<int> order;
      size_t smem = 0;
      for (int i = 0; i < np; ++i) {
        const sa::DevProblem &p = r->probs[i]->dev;
        if (p.d == d && sa::persistent_class(p.nm) == cls) {
          order.push_back(i);
          smem = std::max(smem, sa::persistent_smem_bytes(p, waves));
        }
      }
      if (order.empty()) continue;
      auto work = [&](int i) {
        const sa::DevProblem &p = r->probs[i]->dev;
        return (long long)p.C * p.T * p.nm * p.nk;
      };
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
      r->item_class_begin.push_back((int)net.size());
      r->item_class_d.push_back(d);
      r->item_class_cls.push_back(cls);
      r->class_smem.push_back(smem);
      for (int i : order)
        for (int64_t c = 0; c < r->n; c += waves) {
          net.push_back(i);
          chain0.push_back((int32_t)c);
        }
      r->item_class_count.push_back((int)net.size() - r->item_class_begin.back());
    }
  return (int)net.size();
}

static int upload_items(sa_run *r, int waves) {
  std::vector<int32_t> net, chain0;
  build_items(r, waves, net, chain0);
  SA_HIP(hipMemcpy(r->item_net, net.data(), net.size() * 4, hipMemcpyHostToDevice), "copy items");
  SA_HIP(hipMemcpy(r->item_chain0, chain0.data(), chain0.size() * 4, hipMemcpyHostToDevice), "copy items");
  r->waves = waves;
  r->blocks_per_cu.clear();
  for (size_t k = 0; k < r->item_class_cls.size(); ++k)
    r->blocks_per_cu.push_back(sa::persistent_blocks_per_cu(r->item_class_cls[k], waves, r->class_smem[k]));
  return SA_OK;
}

// Queues stage `st` (index within the run) on `stream`.  `control`: the
// stage takes part in the run's abort handling and stage count (not so for
// the autotuner's trial stages).
static int enqueue_stage(sa_run *r, int32_t st, hipStream_t stream, bool control = true) {
  const int np = (int)r->probs.size();
  const bool first = st == 0;
  const bool timed = !r->ev_start.empty();
  const uint32_t *stop = control && r->abort_dev ? r->ctl : nullptr;
  if (stop) SA_HIP((hipError_t)sa::launch_abort_gate(r->abort_dev, r->ctl, stream), "abort gate launch");
  if (timed) SA_HIP(hipEventRecord(r->ev_start[st], stream), "event record");
  if (!r->persistent) {
    // one launch per problem (several only for the priority model); problem
    // p draws its Philox blocks with network id p
    for (int p = 0; p < np; ++p) {
      const sa::DevProblem &pb = r->probs[p]->dev;
      sa::StageArgs a{};
      a.n_chains = r->n;
      a.seed = r->desc.seed;
      a.net = p;
      a.stage = r->desc.first_stage + st;
      a.L = r->desc.steps_per_stage;
      a.dcap = r->dcap[st];
      a.tau = r->tau + r->tau_off[st];
      a.x_start = first ? r->x0 + r->x_off[p] : r->xwin + r->w_off[p];
      a.x_start_stride = first ? pb.P : 0;
      a.group = first ? 0 : r->group;
      a.xbest = r->xbest + r->x_off[p];
      a.cbest = r->cbest + (size_t)p * r->n;
      a.cstats = r->cstats + (size_t)p * r->n * sa::kStatWords;
      a.stop = stop;
      if (r->learned) {
        sa::LearnedArgs la = r->la;
        la.lt = r->lt[st];
        SA_HIP((hipError_t)sa::launch_learned_stage(pb, a, la, stream), "learned stage launch");
      } else if (pb.model == SA_MODEL_PRIORITY) {
        SA_HIP((hipError_t)sa::launch_priority_stage(pb, a, stream), "priority stage launch");
      } else {
        SA_HIP((hipError_t)sa::launch_stage(pb, a, stream), "stage launch");
      }
    }
  } else {
    const size_t groups = r->item_class_d.size();
    const bool fork = groups > 1 && r->side.size() + 1 >= groups;
    if (fork) {
      SA_HIP(hipEventRecord(r->fork, stream), "fork event");
      for (size_t k = 1; k < groups; ++k) SA_HIP(hipStreamWaitEvent(r->side[k - 1], r->fork, 0), "fork wait");
    }
    for (size_t k = 0; k < groups; ++k) {
      hipStream_t gs = fork && k > 0 ? r->side[k - 1] : stream;
      sa::BatchArgs a{};
      a.probs = r->probs_dev;
      a.n_probs = np;
      a.n_chains = r->n;
      a.item_net = r->item_net + r->item_class_begin[k];
      a.item_chain0 = r->item_chain0 + r->item_class_begin[k];
      a.n_items = r->item_class_count[k];
      a.waves = r->waves;
      a.queue = r->queue + k;
      a.seed = r->desc.seed;
      a.stage = r->desc.first_stage + st;
      a.L = r->desc.steps_per_stage;
      a.dcap = r->dcap[st];
      a.tau = r->tau + r->tau_off[st];
      a.x_start = first ? r->x0 : r->xwin;
      a.first = first;
      a.group = r->group;
      a.x_off = r->x_off_dev;
      a.w_off = r->w_off_dev;
      a.xbest = r->xbest;
      a.cbest = r->cbest;
      a.cstats = r->cstats;
      a.stop = stop;
      const int grid = std::max(1, std::min(a.n_items, r->cus * r->blocks_per_cu[k]));
      SA_HIP((hipError_t)sa::launch_persistent(a, r->item_class_cls[k], r->item_class_d[k], grid, r->class_smem[k],
                                               gs),
             "persistent launch");
    }
    if (fork)
      for (size_t k = 1; k < groups; ++k) {
        SA_HIP(hipEventRecord(r->join[k - 1], r->side[k - 1]), "join event");
        SA_HIP(hipStreamWaitEvent(stream, r->join[k - 1], 0), "join wait");
      }
  }
  if (timed) SA_HIP(hipEventRecord(r->ev_stop[st], stream), "event record");
  sa::BatchReduceArgs ra{};
  ra.n_probs = np;
  ra.n_chains = r->n;
  ra.group = r->group;
  ra.probs = r->probs_dev;
  ra.x_off = r->x_off_dev;
  ra.w_off = r->w_off_dev;
  ra.cbest = r->cbest;
  ra.xbest = r->xbest;
  ra.cstats = r->cstats;
  ra.xwin = r->xwin;
  ra.rec = r->rec + (size_t)st * np;
  ra.queue = r->persistent ? r->queue : nullptr;
  ra.ctl = control ? r->ctl : nullptr;
  ra.st = st;
  SA_HIP((hipError_t)sa::launch_batch_reduce(ra, stream), "reduce launch");
  return SA_OK;
}

// Chains per work item for the persistent kernel: the candidate that runs the
// first stage fastest.  Re-running that stage only rewrites its outputs.
static int autotune_waves(sa_run *r, hipStream_t s) {
  const int candidates[] = {1, 2, 4, 8};
  float best_ms = 0.f;
  int best = 4;
  hipEvent_t e0, e1;
  SA_HIP(hipEventCreate(&e0), "event");
  SA_HIP(hipEventCreate(&e1), "event");
  int rc = SA_OK;
  for (int w : candidates) {
    if ((rc = upload_items(r, w)) != SA_OK) break;
    hipError_t e = hipMemsetAsync(r->queue, 0, sa::kPersistentQueues * sizeof(uint32_t), s);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e != hipSuccess) {
      rc = hip_fail(e, "autotune");
      break;
    }
    if ((rc = enqueue_stage(r, 0, s, false)) != SA_OK) break;
    float ms = 0.f;
    e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      rc = hip_fail(e, "autotune");
      break;
    }
    if (best_ms == 0.f || ms < best_ms) {
      best_ms = ms;
      best = w;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != SA_OK) return rc;
  rc = upload_items(r, best);
  if (rc != SA_OK) return rc;
  SA_HIP(hipMemsetAsync(r->queue, 0, sa::kPersistentQueues * sizeof(uint32_t), s), "queue reset");
  return SA_OK;
}

extern "C" int sa_run_create(sa_problem *const *probs, int32_t n_probs, const sa_run_desc *desc,
                             const int8_t *x0_dev, sa_run **out, void *stream) {
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!probs || !desc || !x0_dev) return fail(SA_ERR_ARG, "NULL argument");
  if (n_probs < 1) return fail(SA_ERR_ARG, "n_probs must be >= 1");
  for (int i = 0; i < n_probs; ++i)
    if (!probs[i]) return fail(SA_ERR_ARG, "problem %d is NULL", i);
  if (desc->n_chains < 1 || desc->n_chains > (1ll << 31) - 1) return fail(SA_ERR_ARG, "n_chains out of range");
  if (!(desc->T0 > 0) || !(desc->rho > 0)) return fail(SA_ERR_ARG, "T0 and rho must be > 0");
  if (desc->first_stage < 0 || desc->n_stages < 0 || desc->steps_per_stage < 1)
    return fail(SA_ERR_ARG, "stage counts out of range");
  if (desc->kernel != SA_KERNEL_AUTO && desc->kernel != SA_KERNEL_PERSISTENT)
    return fail(SA_ERR_ARG, "unknown kernel %d", desc->kernel);
  if (desc->chains_per_block != 0 && desc->chains_per_block != 1 && desc->chains_per_block != 2 &&
      desc->chains_per_block != 4 && desc->chains_per_block != 8)
    return fail(SA_ERR_ARG, "chains_per_block must be 0 (autotune), 1, 2, 4 or 8");
  if (desc->record_times && desc->use_graph) return fail(SA_ERR_ARG, "record_times and use_graph exclude each other");
  if (desc->group_size < 0) return fail(SA_ERR_ARG, "group_size must be >= 0");
  void *abort_dev = nullptr;
  if (desc->abort_flag_host) {
    hipError_t ae = hipHostGetDevicePointer(&abort_dev, const_cast<int32_t *>(desc->abort_flag_host), 0);
    if (ae != hipSuccess || !abort_dev) {
      (void)hipGetLastError();  // clear the sticky error the lookup leaves
      return fail(SA_ERR_ARG, "abort_flag_host is not pinned host memory (hipHostMalloc)");
    }
  }
  const bool learned = desc->proposal == SA_PROPOSAL_LEARNED, traced = desc->trace_dev != nullptr;
  if (desc->proposal != SA_PROPOSAL_PLAIN && !learned) return fail(SA_ERR_ARG, "unknown proposal %d", desc->proposal);
  if (learned && !desc->model) return fail(SA_ERR_ARG, "the learned proposal needs a model");
  if ((learned || traced) && desc->refresh_every < 1) return fail(SA_ERR_ARG, "refresh_every must be >= 1");
  if (learned && !(desc->eps_plain >= 0.0 && desc->eps_plain <= 1.0))
    return fail(SA_ERR_ARG, "eps_plain must be in [0, 1]");
  if (traced && (desc->trace_every < 1 || desc->trace_capacity < 1))
    return fail(SA_ERR_ARG, "trace_every and trace_capacity must be >= 1");
  if (learned || traced) {
    if (n_probs != 1 || desc->kernel != SA_KERNEL_AUTO)
      return fail(SA_ERR_UNSUPPORTED, "the learned proposal and the trace run one problem on the specialised kernel");
    if (desc->group_size > 0 && desc->group_size < desc->n_chains)
      return fail(SA_ERR_UNSUPPORTED, "the learned proposal and the trace restart every chain from the global best");
    const sa::DevProblem &dp = probs[0]->dev;
    if (dp.nm > sa::kLearnedMaxTilesM)
      return fail(SA_ERR_UNSUPPORTED, "learned proposal / trace: %d nodes (at most 127)", dp.N);
    if (dp.K > sa::kLearnedMaxObsTimes)
      return fail(SA_ERR_UNSUPPORTED, "learned proposal / trace: %d observed times (at most 42)", dp.K);
    if (learned && desc->model->device != probs[0]->device) return fail(SA_ERR_ARG, "model on another device");
  }
  const bool priority = probs[0]->dev.model == SA_MODEL_PRIORITY;
  for (int i = 0; i < n_probs; ++i)
    if ((probs[i]->dev.model == SA_MODEL_PRIORITY) != priority)
      return fail(SA_ERR_UNSUPPORTED, "problems of both models in one run");
  if (priority && (desc->kernel != SA_KERNEL_AUTO || learned || traced))
    return fail(SA_ERR_UNSUPPORTED, "the priority model runs on its own stage kernel with plain proposals");
  const int device = probs[0]->device;
  for (int i = 1; i < n_probs; ++i)
    if (probs[i]->device != device) return fail(SA_ERR_ARG, "problems on different devices");
  SA_HIP(hipSetDevice(device), "hipSetDevice");
  // several priority-model problems take one stage-kernel launch each
  const bool persistent = !priority && (n_probs > 1 || desc->kernel == SA_KERNEL_PERSISTENT);
  if (persistent)
    for (int i = 0; i < n_probs; ++i)
      if (probs[i]->dev.nm > sa::kPersistentTilesM)
        return fail(SA_ERR_UNSUPPORTED, "problem %d: %d nodes exceed the many-network kernel (159)", i,
                    probs[i]->dev.N);
  const int64_t n = desc->n_chains;
  hipStream_t s = (hipStream_t)stream;

  auto *r = new sa_run();
  r->probs.assign(probs, probs + n_probs);
  r->desc = *desc;
  r->device = device;
  r->n = n;
  r->persistent = persistent;
  r->stream = s;
  r->abort_host = desc->abort_flag_host;
  r->abort_dev = static_cast<const volatile int32_t *>(abort_dev);
  r->group = desc->group_size > 0 && desc->group_size < n ? desc->group_size : 0;
  const int64_t n_groups = r->group ? (n + r->group - 1) / r->group : 1;
  int64_t xo = 0, wo = 0;
  int32_t max_cost = 0;
  for (int i = 0; i < n_probs; ++i) {
    r->x_off.push_back(xo);
    r->w_off.push_back(wo);
    xo += n * probs[i]->dev.P;
    wo += n_groups * probs[i]->dev.P;
    max_cost = std::max(max_cost, probs[i]->info.max_cost);
  }
  if (learned || traced) {
    r->learned = true;
    const size_t smem = sa::learned_smem_bytes(probs[0]->dev, learned);
    if (smem > 160 * 1024) {
      free_run(r);
      return fail(SA_ERR_UNSUPPORTED, "learned stage kernel needs %zu bytes of LDS", smem);
    }
    hipError_t pe = (hipError_t)sa::learned_stage_prepare(probs[0]->dev, smem);
    if (pe != hipSuccess) {
      free_run(r);
      return hip_fail(pe, "learned stage LDS limit");
    }
    sa::LearnedArgs &la = r->la;
    la.refresh = desc->refresh_every;
    if (learned) {
      la.w1f = desc->model->w1f;
      la.w2f = desc->model->w2f;
      la.b2 = desc->model->master + sa::kMlpParams - 1;
      la.eps_u = desc->eps_plain >= 1.0 ? (1ull << 32)
                                        : std::min<uint64_t>((uint64_t)std::floor(desc->eps_plain * 4294967296.0),
                                                             0xFFFFFFFFull);
    }
    if (traced) {
      la.trace = static_cast<sa::TraceRecord *>(desc->trace_dev);
      la.trace_cap = desc->trace_capacity;
      la.trace_every = desc->trace_every;
      const int64_t g0 = (int64_t)desc->first_stage * desc->steps_per_stage;
      la.trace_first = (g0 + desc->trace_every - 1) / desc->trace_every * desc->trace_every;
    }
  } else if (priority) {
    for (int i = 0; i < n_probs; ++i) {
      const size_t smem = sa::priority_stage_smem_bytes(probs[i]->dev);
      if (smem > 64 * 1024) {
        free_run(r);
        return fail(SA_ERR_UNSUPPORTED, "problem %d: priority stage kernel needs %zu bytes of LDS (> 64 KiB)", i,
                    smem);
      }
    }
  } else if (!persistent) {
    const size_t smem = sa::stage_smem_bytes(probs[0]->dev, sa::stage_waves_per_block(probs[0]->dev));
    if (smem > 64 * 1024) {
      free_run(r);
      return fail(SA_ERR_UNSUPPORTED, "stage kernel needs %zu bytes of LDS (> 64 KiB)", smem);
    }
  }

  // starting vectors: domain on the host, constraints (hard mode) on the device
  std::vector<int8_t> hx((size_t)xo);
  hipError_t e = hipMemcpyAsync(hx.data(), x0_dev, hx.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_run(r);
    return hip_fail(e, "copy x0");
  }
  for (int i = 0; i < n_probs; ++i) {
    const int P = probs[i]->dev.P;
    for (int64_t c = 0; c < n; ++c)
      for (int k = 0; k < P; ++k) {
        const int v = hx[(size_t)(r->x_off[i] + c * P + k)];
        if (!in_domain(probs[i]->dev, k, v)) {
          free_run(r);
          return fail(SA_ERR_DOMAIN, "x0 problem %d chain %lld parameter %d = %d", i, (long long)c, k, v);
        }
      }
  }

  const int S = desc->n_stages;
  std::vector<uint32_t> all_tau, tab;
  double T = desc->T0;
  for (int k = 0; k < desc->first_stage; ++k) T = T * desc->rho;
  for (int st = 0; st < S; ++st) {
    int32_t cap;
    tau_table(T, max_cost, tab, cap);
    r->tau_off.push_back(all_tau.size());
    r->dcap.push_back(cap);
    r->lt.push_back((float)(std::log(T) / 5.0));
    all_tau.insert(all_tau.end(), tab.begin(), tab.end());
    T = T * desc->rho;
  }
  auto alloc = [&](void **ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes ? bytes : 1);
  };
  alloc((void **)&r->x0, (size_t)xo);
  alloc((void **)&r->xbest, (size_t)xo);
  alloc((void **)&r->xwin, (size_t)wo);
  alloc((void **)&r->cbest, (size_t)(n * n_probs) * 4);
  alloc((void **)&r->cstats, (size_t)(n * n_probs) * 4 * sa::kStatWords);
  alloc((void **)&r->tau, all_tau.size() * 4);
  alloc((void **)&r->queue, sa::kPersistentQueues * sizeof(uint32_t));
  alloc((void **)&r->rec, (size_t)std::max(S, 1) * n_probs * sizeof(sa::StageRecord));
  alloc((void **)&r->probs_dev, (size_t)n_probs * sizeof(sa::DevProblem));
  alloc((void **)&r->x_off_dev, (size_t)n_probs * 8);
  alloc((void **)&r->w_off_dev, (size_t)n_probs * 8);
  alloc((void **)&r->item_net, (size_t)(n * n_probs) * 4);
  alloc((void **)&r->item_chain0, (size_t)(n * n_probs) * 4);
  alloc((void **)&r->ctl, 2 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemsetAsync(r->ctl, 0, 2 * sizeof(uint32_t), s);
  for (int st = 0; st < S && desc->record_times && e == hipSuccess; ++st) {
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    r->ev_start.push_back(a);
    r->ev_stop.push_back(b);
  }
  std::vector<sa::DevProblem> dps;
  for (sa_problem *p : r->probs) dps.push_back(p->dev);
  if (e == hipSuccess) e = hipMemcpyAsync(r->x0, x0_dev, (size_t)xo, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && !all_tau.empty())
    e = hipMemcpyAsync(r->tau, all_tau.data(), all_tau.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(r->probs_dev, dps.data(), dps.size() * sizeof(sa::DevProblem), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(r->x_off_dev, r->x_off.data(), (size_t)n_probs * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(r->w_off_dev, r->w_off.data(), (size_t)n_probs * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(r->queue, 0, sa::kPersistentQueues * sizeof(uint32_t), s);
  // lambda >= 1, so V(x0) = 0 exactly when the cost with lambda equals the
  // cost with lambda = 0 (the mismatch alone)
  for (int i = 0; i < n_probs && e == hipSuccess; ++i) {
    const sa::DevProblem &dp = probs[i]->dev;
    if (!dp.hard) continue;
    int32_t *c1 = r->cbest, *c0 = (int32_t *)r->cstats;
    e = (hipError_t)launch_cost(dp, r->x0 + r->x_off[i], n, c1, s);
    sa::DevProblem m = dp;
    m.lambda = 0;
    if (e == hipSuccess) e = (hipError_t)launch_cost(m, r->x0 + r->x_off[i], n, c0, s);
    std::vector<int32_t> h1((size_t)n), h0((size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(h1.data(), c1, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h0.data(), c0, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
      for (int64_t c = 0; c < n; ++c)
        if (h1[(size_t)c] != h0[(size_t)c]) {
          free_run(r);
          return fail(SA_ERR_INFEASIBLE, "x0 of problem %d chain %lld breaks a structural constraint", i,
                      (long long)c);
        }
  }
  if (e != hipSuccess) {
    free_run(r);
    return hip_fail(e, "run setup");
  }
  if (persistent) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
      r->cus = cus;
    int rc = SA_OK;
    {
      // side streams and events for the concurrent launch groups (default priority)
      std::vector<int32_t> net, chain0;
      build_items(r, 4, net, chain0);
      const size_t groups = r->item_class_d.size();
      hipError_t ce = hipSuccess;
      if (groups > 1) ce = hipEventCreateWithFlags(&r->fork, hipEventDisableTiming);
      for (size_t k = 1; k < groups && ce == hipSuccess; ++k) {
        hipStream_t x = nullptr;
        hipEvent_t j = nullptr;
        ce = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
        if (ce == hipSuccess) r->side.push_back(x);
        if (ce == hipSuccess) ce = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (ce == hipSuccess) r->join.push_back(j);
      }
      if (ce != hipSuccess) rc = hip_fail(ce, "side streams");
    }
    if (rc == SA_OK)
      rc = desc->chains_per_block == 0 && S > 0 ? autotune_waves(r, s)
                                                : upload_items(r, desc->chains_per_block ? desc->chains_per_block : 4);
    if (rc == SA_OK) {
      const size_t lds_max = 160 * 1024;
      for (size_t smem : r->class_smem)
        if (smem > lds_max) rc = fail(SA_ERR_UNSUPPORTED, "many-network kernel needs %zu bytes of LDS", smem);
    }
    if (rc != SA_OK) {
      free_run(r);
      return rc;
    }
  }
  *out = r;
  return SA_OK;
}

extern "C" int sa_run_launch(sa_run *r, int32_t n_stages, void *stream) {
  if (!r) return fail(SA_ERR_ARG, "run is NULL");
  if (n_stages < 0 || r->launched + n_stages > r->desc.n_stages)
    return fail(SA_ERR_ARG, "stages beyond the schedule (%d launched of %d, asked %d)", r->launched,
                r->desc.n_stages, n_stages);
  SA_HIP(hipSetDevice(r->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  if (n_stages == 0) return SA_OK;
  if (r->abort_host && *r->abort_host != 0) return fail(SA_ERR_ABORTED, "the run's abort flag is set; nothing queued");
  if (r->desc.use_graph) {
    // The stages of this call become one graph (no memset nodes inside),
    // captured on the run's own stream (the caller's may be the null stream,
    // which cannot be captured) and launched on the caller's stream.
    if (!r->capture_stream) SA_HIP(hipStreamCreateWithFlags(&r->capture_stream, hipStreamNonBlocking), "stream create");
    hipStream_t cs = r->capture_stream;
    SA_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    int rc = SA_OK;
    for (int32_t i = 0; i < n_stages && rc == SA_OK; ++i) rc = enqueue_stage(r, r->launched + i, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc != SA_OK) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    r->graphs.push_back(x);
    SA_HIP(hipGraphLaunch(x, s), "graph launch");
  } else {
    for (int32_t i = 0; i < n_stages; ++i) {
      int rc = enqueue_stage(r, r->launched + i, s);
      if (rc != SA_OK) return rc;
    }
  }
  r->launched += n_stages;
  r->stream = s;
  return SA_OK;
}

extern "C" int sa_run_chains(sa_problem *const *probs, int32_t n_probs, const sa_run_desc *desc,
                             const int8_t *x0_dev, sa_run **out, void *stream) {
  int rc = sa_run_create(probs, n_probs, desc, x0_dev, out, stream);
  if (rc != SA_OK) return rc;
  rc = sa_run_launch(*out, desc->n_stages, stream);
  if (rc != SA_OK) {
    sa_destroy_run(*out);
    *out = nullptr;
  }
  return rc;
}

static int sync_run(sa_run *r, int32_t prob) {
  if (!r) return fail(SA_ERR_ARG, "run is NULL");
  if (prob < 0 || prob >= (int32_t)r->probs.size()) return fail(SA_ERR_ARG, "problem index %d out of range", prob);
  SA_HIP(hipSetDevice(r->device), "hipSetDevice");
  SA_HIP(hipStreamSynchronize(r->stream), "stream sync");
  return SA_OK;
}

// Stages of the run that have completed (after synchronising its stream):
// the stages launched, unless an abort skipped the rest.
static int stages_done(sa_run *r, int32_t &done) {
  uint32_t ctl[2] = {0, 0};
  SA_HIP(hipMemcpy(ctl, r->ctl, sizeof(ctl), hipMemcpyDeviceToHost), "copy run control");
  done = (int32_t)std::min<uint32_t>(ctl[1], (uint32_t)r->launched);
  return SA_OK;
}

extern "C" int sa_run_stages_done(sa_run *r, int32_t *done) {
  if (!done) return fail(SA_ERR_ARG, "done is NULL");
  int rc = sync_run(r, 0);
  if (rc != SA_OK) return rc;
  return stages_done(r, *done);
}

extern "C" int sa_best(sa_run *r, int32_t prob, int8_t *x_host, int32_t *cost, int32_t *winner) {
  int rc = sync_run(r, prob);
  if (rc != SA_OK) return rc;
  if (r->launched == 0) return fail(SA_ERR_ARG, "no stage launched");
  int32_t done = 0;
  if ((rc = stages_done(r, done)) != SA_OK) return rc;
  if (done == 0) return fail(SA_ERR_ARG, "no stage completed (aborted before the first)");
  const size_t np = r->probs.size();
  sa::StageRecord rec;
  SA_HIP(hipMemcpy(&rec, r->rec + (size_t)(done - 1) * np + prob, sizeof(rec), hipMemcpyDeviceToHost),
         "copy record");
  // the global winner is also the winner of its restart group
  const int64_t P = r->probs[prob]->dev.P;
  const int64_t slot = r->group ? rec.winner / r->group : 0;
  if (x_host)
    SA_HIP(hipMemcpy(x_host, r->xwin + r->w_off[prob] + slot * P, (size_t)P, hipMemcpyDeviceToHost), "copy best");
  if (cost) *cost = rec.best_cost;
  if (winner) *winner = rec.winner;
  return SA_OK;
}

extern "C" int sa_stats(sa_run *r, int32_t prob, sa_stage_stats *out) {
  int rc = sync_run(r, prob);
  if (rc != SA_OK) return rc;
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  const size_t np = r->probs.size();
  int32_t done = 0;
  if ((rc = stages_done(r, done)) != SA_OK) return rc;
  std::vector<sa::StageRecord> rec((size_t)r->launched * np);
  if (done)
    SA_HIP(hipMemcpy(rec.data(), r->rec, (size_t)done * np * sizeof(sa::StageRecord), hipMemcpyDeviceToHost),
           "copy records");
  for (int32_t i = 0; i < r->launched; ++i) {
    if (i >= done) {  // skipped by an abort
      out[i] = sa_stage_stats{};
      out[i].best_cost = -1;
      out[i].winner = -1;
      continue;
    }
    const sa::StageRecord &x = rec[(size_t)i * np + prob];
    out[i].best_cost = x.best_cost;
    out[i].winner = x.winner;
    out[i].accepted = x.accepted;
    out[i].uphill = x.uphill;
    out[i].neutral = x.neutral;
    out[i].infeasible = x.infeasible;
    out[i].simulated = x.simulated;
  }
  return SA_OK;
}

extern "C" int sa_chain_best(sa_run *r, int32_t prob, int32_t *cost, int8_t *x_host) {
  int rc = sync_run(r, prob);
  if (rc != SA_OK) return rc;
  const int64_t n = r->n;
  if (cost)
    SA_HIP(hipMemcpy(cost, r->cbest + (size_t)prob * n, (size_t)n * 4, hipMemcpyDeviceToHost), "copy chain costs");
  if (x_host)
    SA_HIP(hipMemcpy(x_host, r->xbest + r->x_off[prob], (size_t)(n * r->probs[prob]->dev.P), hipMemcpyDeviceToHost),
           "copy chain bests");
  return SA_OK;
}

extern "C" int sa_run_get_info(sa_run *r, sa_run_info *info) {
  if (!r || !info) return fail(SA_ERR_ARG, "NULL argument");
  info->n_probs = (int32_t)r->probs.size();
  info->kernel = r->persistent ? SA_KERNEL_PERSISTENT : SA_KERNEL_AUTO;
  const sa::DevProblem &dp0 = r->probs[0]->dev;
  info->chains_per_block = r->persistent                      ? r->waves
                           : dp0.model == SA_MODEL_PRIORITY ? 4 * (64 / dp0.lc)
                                                            : sa::stage_waves_per_block(dp0);
  info->stages_launched = r->launched;
  info->tiles_m = r->probs[0]->dev.nm;
  info->frags_k = r->probs[0]->dev.nk;
  return SA_OK;
}

extern "C" int sa_stage_times(sa_run *r, int32_t prob, float *ms) {
  int rc = sync_run(r, prob);
  if (rc != SA_OK) return rc;
  if (!ms) return fail(SA_ERR_ARG, "out is NULL");
  if (r->ev_start.empty()) return fail(SA_ERR_ARG, "run was created without record_times");
  for (int32_t i = 0; i < r->launched; ++i)
    SA_HIP(hipEventElapsedTime(&ms[i], r->ev_start[i], r->ev_stop[i]), "event elapsed");
  return SA_OK;
}

extern "C" int sa_destroy_run(sa_run *r) {
  if (!r) return SA_OK;
  hipSetDevice(r->device);
  hipStreamSynchronize(r->stream);
  free_run(r);
  return SA_OK;
}

// ---------------------------------------------------------------------------
// the run without allocations (sa_run_chains_noalloc)
// ---------------------------------------------------------------------------
// The run state lives in this fixed device array instead of hipMalloc'ed
// memory.  Host code never uses the array's name as an address: each device's
// copy is looked up once with hipGetSymbolAddress (with that device current)
// and that pointer is what the kernels get.
static constexpr size_t kNoAllocScratchBytes = (size_t)SA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

static constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];
static std::once_flag g_scratch_once[kMaxDevices];

static int scratch_for_device(int device, uint8_t *&ptr) {
  if (device < 0 || device >= kMaxDevices) return fail(SA_ERR_UNSUPPORTED, "device %d beyond %d", device, kMaxDevices);
  std::call_once(g_scratch_once[device], [device] {
    g_scratch_err[device] = hipGetSymbolAddress(&g_scratch_ptr[device], HIP_SYMBOL(scratch));
  });
  if (g_scratch_err[device] != hipSuccess) return hip_fail(g_scratch_err[device], "hipGetSymbolAddress(scratch)");
  if (!g_scratch_ptr[device]) return fail(SA_ERR_DEVICE, "no scratch address on device %d", device);
  ptr = static_cast<uint8_t *>(g_scratch_ptr[device]);
  return SA_OK;
}

static_assert(sizeof(sa_stage_stats) == sizeof(sa::StageRecord) && offsetof(sa_stage_stats, accepted) ==
                  offsetof(sa::StageRecord, accepted) && offsetof(sa_stage_stats, simulated) ==
                  offsetof(sa::StageRecord, simulated),
              "stage statistics layout");

extern "C" int sa_run_chains_noalloc(const sa_problem *prob, const sa_run_desc *desc, const int8_t *x0_dev,
                                     int8_t *x_best_dev, int32_t *best_dev, sa_stage_stats *stats_dev,
                                     void *stream) {
  if (!prob || !desc || !x0_dev || !x_best_dev || !best_dev) return fail(SA_ERR_ARG, "NULL argument");
  if (desc->n_chains < 1 || desc->n_chains > (1ll << 31) - 1) return fail(SA_ERR_ARG, "n_chains out of range");
  if (!(desc->T0 > 0) || !(desc->rho > 0)) return fail(SA_ERR_ARG, "T0 and rho must be > 0");
  if (desc->first_stage < 0 || desc->n_stages < 1 || desc->steps_per_stage < 1)
    return fail(SA_ERR_ARG, "stage counts out of range (at least one stage)");
  if (desc->kernel != SA_KERNEL_AUTO || desc->proposal != SA_PROPOSAL_PLAIN || desc->trace_dev ||
      desc->record_times || desc->use_graph || desc->abort_flag_host || desc->group_size < 0 ||
      (desc->group_size > 0 && desc->group_size < desc->n_chains))
    return fail(SA_ERR_UNSUPPORTED, "the allocation-free run takes plain proposals, the global restart and the "
                                    "specialised kernel, without trace, timing, graph or abort flag");
  const sa::DevProblem &dp = prob->dev;
  const int64_t n = desc->n_chains, P = dp.P;
  const int S = desc->n_stages;
  hipStream_t s = (hipStream_t)stream;
  SA_HIP(hipSetDevice(prob->device), "hipSetDevice");
  if (dp.model == SA_MODEL_PRIORITY) {
    if (sa::priority_stage_smem_bytes(dp) > 64 * 1024)
      return fail(SA_ERR_UNSUPPORTED, "priority stage kernel needs more than 64 KiB of LDS");
  } else if (sa::stage_smem_bytes(dp, sa::stage_waves_per_block(dp)) > 64 * 1024) {
    return fail(SA_ERR_UNSUPPORTED, "stage kernel needs more than 64 KiB of LDS");
  }

  // thresholds of every stage (host), as sa_run_create
  std::vector<uint32_t> all_tau, tab;
  std::vector<size_t> tau_off;
  std::vector<int32_t> dcap;
  double T = desc->T0;
  for (int k = 0; k < desc->first_stage; ++k) T = T * desc->rho;
  for (int st = 0; st < S; ++st) {
    int32_t cap;
    tau_table(T, prob->info.max_cost, tab, cap);
    tau_off.push_back(all_tau.size());
    dcap.push_back(cap);
    all_tau.insert(all_tau.end(), tab.begin(), tab.end());
    T = T * desc->rho;
  }
  // scratch layout: problem descriptor, offsets, thresholds, stage records,
  // chain bests, winner, chain costs and statistics (256-byte aligned)
  Layout lay;
  const size_t o_dp = lay.take(sizeof(sa::DevProblem)), o_xoff = lay.take(8), o_woff = lay.take(8),
               o_tau = lay.take(all_tau.size() * 4), o_rec = lay.take((size_t)S * sizeof(sa::StageRecord)),
               o_xbest = lay.take((size_t)(n * P)), o_xwin = lay.take((size_t)P), o_cbest = lay.take((size_t)n * 4),
               o_cstats = lay.take((size_t)n * 4 * sa::kStatWords);
  if (lay.bytes > kNoAllocScratchBytes)
    return fail(SA_ERR_UNSUPPORTED, "the run needs %zu bytes of scratch, more than the %zu the allocation-free "
                                    "entry point has", lay.bytes, kNoAllocScratchBytes);
  uint8_t *base = nullptr;
  if (int rc = scratch_for_device(prob->device, base)) return rc;

  // starting vectors: domain on the host
  std::vector<int8_t> hx((size_t)(n * P));
  SA_HIP(hipMemcpyAsync(hx.data(), x0_dev, hx.size(), hipMemcpyDeviceToHost, s), "copy x0");
  SA_HIP(hipStreamSynchronize(s), "stream sync");
  for (int64_t c = 0; c < n; ++c)
    for (int k = 0; k < P; ++k)
      if (!in_domain(dp, k, hx[(size_t)(c * P + k)]))
        return fail(SA_ERR_DOMAIN, "x0 chain %lld parameter %d = %d", (long long)c, k, hx[(size_t)(c * P + k)]);
  // the small tables, staged in one host block and copied in one call; the
  // stream is synchronised below, before the block goes out of scope
  std::vector<uint8_t> head(o_tau + all_tau.size() * 4);
  const int64_t zero = 0;
  std::memcpy(head.data() + o_dp, &dp, sizeof(dp));
  std::memcpy(head.data() + o_xoff, &zero, 8);
  std::memcpy(head.data() + o_woff, &zero, 8);
  if (!all_tau.empty()) std::memcpy(head.data() + o_tau, all_tau.data(), all_tau.size() * 4);
  SA_HIP(hipMemcpyAsync(base, head.data(), head.size(), hipMemcpyHostToDevice, s), "copy run tables");
  int32_t *cbest = reinterpret_cast<int32_t *>(base + o_cbest);
  uint32_t *cstats = reinterpret_cast<uint32_t *>(base + o_cstats);
  if (dp.hard) {
    // hard mode: every start satisfies (a) and (b) iff its cost equals its mismatch (lambda = 0)
    sa::DevProblem m = dp;
    m.lambda = 0;
    SA_HIP((hipError_t)launch_cost(dp, x0_dev, n, cbest, s), "start costs");
    SA_HIP((hipError_t)launch_cost(m, x0_dev, n, reinterpret_cast<int32_t *>(cstats), s), "start costs");
    std::vector<int32_t> h1((size_t)n), h0((size_t)n);
    SA_HIP(hipMemcpyAsync(h1.data(), cbest, (size_t)n * 4, hipMemcpyDeviceToHost, s), "copy costs");
    SA_HIP(hipMemcpyAsync(h0.data(), cstats, (size_t)n * 4, hipMemcpyDeviceToHost, s), "copy costs");
    SA_HIP(hipStreamSynchronize(s), "stream sync");
    for (int64_t c = 0; c < n; ++c)
      if (h1[(size_t)c] != h0[(size_t)c])
        return fail(SA_ERR_INFEASIBLE, "x0 chain %lld breaks a structural constraint", (long long)c);
  } else {
    SA_HIP(hipStreamSynchronize(s), "stream sync");
  }

  // a run whose device state points into the scratch array; enqueue_stage
  // queues exactly the kernels of sa_run_launch's eager path
  sa_run r;
  r.probs.assign(1, const_cast<sa_problem *>(prob));
  r.desc = *desc;
  r.device = prob->device;
  r.n = n;
  r.stream = s;
  r.x0 = const_cast<int8_t *>(x0_dev);
  r.xbest = reinterpret_cast<int8_t *>(base + o_xbest);
  r.xwin = reinterpret_cast<int8_t *>(base + o_xwin);
  r.cbest = cbest;
  r.cstats = cstats;
  r.tau = reinterpret_cast<uint32_t *>(base + o_tau);
  r.rec = reinterpret_cast<sa::StageRecord *>(base + o_rec);
  r.probs_dev = reinterpret_cast<sa::DevProblem *>(base + o_dp);
  r.x_off_dev = reinterpret_cast<int64_t *>(base + o_xoff);
  r.w_off_dev = reinterpret_cast<int64_t *>(base + o_woff);
  r.x_off.assign(1, 0);
  r.w_off.assign(1, 0);
  r.tau_off = tau_off;
  r.dcap = dcap;
  for (int st = 0; st < S; ++st)
    if (int rc = enqueue_stage(&r, st, s)) return rc;
  SA_HIP(hipMemcpyAsync(x_best_dev, r.xwin, (size_t)P, hipMemcpyDeviceToDevice, s), "copy best vector");
  SA_HIP(hipMemcpyAsync(best_dev, r.rec + (S - 1), 2 * sizeof(int32_t), hipMemcpyDeviceToDevice, s),
         "copy best cost");
  if (stats_dev)
    SA_HIP(hipMemcpyAsync(stats_dev, r.rec, (size_t)S * sizeof(sa::StageRecord), hipMemcpyDeviceToDevice, s),
           "copy stage statistics");
  return SA_OK;
}

// ---------------------------------------------------------------------------
// measured instruction peaks
// ---------------------------------------------------------------------------
extern "C" int sa_measure_peak(int32_t kind, double *rate, double *ms_out, void *stream) {
  if (!rate) return fail(SA_ERR_ARG, "rate is NULL");
  if (kind < SA_PEAK_VALU_XOR || kind > SA_PEAK_LDS_READ) return fail(SA_ERR_ARG, "unknown peak kind %d", kind);
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, cus = 0;
  SA_HIP(hipGetDevice(&dev), "hipGetDevice");
  SA_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "device attribute");
  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
  const int blocks = std::max(cus, 1) * 8, threads = 256;
  void *sink = nullptr;
  SA_HIP(hipMalloc(&sink, (size_t)blocks * threads * 4), "hipMalloc(probe)");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = 0.f;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // the first launch warms up clocks and code
    e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = (hipError_t)sa::launch_probe(kind, sink, blocks, threads, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess && rep > 0 && (best == 0.f || t < best)) best = t;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(sink);
  if (e != hipSuccess) return hip_fail(e, "peak probe");
  if (!(best > 0.f)) return fail(SA_ERR_DEVICE, "peak probe: no time measured");
  *rate = sa::probe_work(kind, blocks, threads) / (best * 1e-3);
  if (ms_out) *ms_out = best;
  return SA_OK;
}

// ---------------------------------------------------------------------------
// proposal network
// ---------------------------------------------------------------------------

static int mlp_check_params(const float *params) {
  if (!params) return fail(SA_ERR_ARG, "params is NULL");
  for (int i = 0; i < sa::kMlpParams; ++i)
    if (!std::isfinite(params[i])) return fail(SA_ERR_DOMAIN, "params[%d] is not finite", i);
  return SA_OK;
}

static int mlp_upload(sa_mlp *m, const float *params) {
  SA_HIP(hipSetDevice(m->device), "hipSetDevice");
  SA_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  SA_HIP(hipMemcpy(m->master, params, sizeof(float) * sa::kMlpParams, hipMemcpyHostToDevice), "copy params");
  SA_HIP(hipMemset(m->m, 0, sizeof(float) * sa::kMlpParams), "clear Adam state");
  SA_HIP(hipMemset(m->v, 0, sizeof(float) * sa::kMlpParams), "clear Adam state");
  m->steps = 0;
  sa::MlpUpdateArgs u{};
  u.master = m->master;
  u.w1f = m->w1f;
  u.w2f = m->w2f;
  SA_HIP(sa::launch_mlp_update(u, nullptr), "pack fragments");
  SA_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  return SA_OK;
}

extern "C" int sa_mlp_create(const float *params, sa_mlp **out) {
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (int rc = mlp_check_params(params)) return rc;
  auto *m = new sa_mlp();
  hipGetDevice(&m->device);
  Layout lay;
  const size_t o_master = lay.take(sizeof(float) * sa::kMlpParams), o_m = lay.take(sizeof(float) * sa::kMlpParams),
               o_v = lay.take(sizeof(float) * sa::kMlpParams), o_w1f = lay.take(sizeof(uint4) * sa::kW1FragU4),
               o_w2f = lay.take(sizeof(uint4) * sa::kW2FragU4),
               o_part = lay.take(sizeof(float) * sa::kMlpParams * (size_t)sa::kMlpMaxWaves),
               o_loss = lay.take(sizeof(float) * sa::kMlpMaxWaves);
  hipError_t e = hipMalloc(&m->dmem, lay.bytes);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "hipMalloc(model)");
  }
  char *base = static_cast<char *>(m->dmem);
  m->master = reinterpret_cast<float *>(base + o_master);
  m->m = reinterpret_cast<float *>(base + o_m);
  m->v = reinterpret_cast<float *>(base + o_v);
  m->w1f = reinterpret_cast<uint4 *>(base + o_w1f);
  m->w2f = reinterpret_cast<uint4 *>(base + o_w2f);
  m->partial = reinterpret_cast<float *>(base + o_part);
  m->loss_partial = reinterpret_cast<float *>(base + o_loss);
  if (int rc = mlp_upload(m, params)) {
    hipFree(m->dmem);
    delete m;
    return rc;
  }
  *out = m;
  return SA_OK;
}

extern "C" int sa_mlp_destroy(sa_mlp *m) {
  if (!m) return SA_OK;
  hipSetDevice(m->device);
  hipDeviceSynchronize();
  hipFree(m->dmem);
  delete m;
  return SA_OK;
}

extern "C" int sa_mlp_get_params(const sa_mlp *m, float *params) {
  if (!m || !params) return fail(SA_ERR_ARG, "NULL model or params");
  SA_HIP(hipSetDevice(m->device), "hipSetDevice");
  SA_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize");
  SA_HIP(hipMemcpy(params, m->master, sizeof(float) * sa::kMlpParams, hipMemcpyDeviceToHost), "copy params");
  return SA_OK;
}

extern "C" int sa_mlp_set_params(sa_mlp *m, const float *params) {
  if (!m) return fail(SA_ERR_ARG, "model is NULL");
  if (int rc = mlp_check_params(params)) return rc;
  return mlp_upload(m, params);
}

extern "C" int sa_mlp_forward(const sa_mlp *m, const uint16_t *x, int64_t n, float *logit, void *stream) {
  if (!m || n < 0) return fail(SA_ERR_ARG, "NULL model or negative n");
  if (n == 0) return SA_OK;
  if (!x || !logit) return fail(SA_ERR_ARG, "NULL x or logit");
  SA_HIP(sa::launch_mlp_forward(reinterpret_cast<const uint4 *>(x), n, logit, m->w1f, m->w2f, m->master,
                                (hipStream_t)stream),
         "mlp forward");
  return SA_OK;
}

static int mlp_backward(sa_mlp *m, const uint16_t *x, const float *y, int64_t n, hipStream_t s, int &waves) {
  const int64_t tiles = (n + 31) / 32;
  int64_t w = std::min<int64_t>(tiles, sa::kMlpMaxWaves);
  const int64_t tpw = (tiles + w - 1) / w;
  w = (tiles + tpw - 1) / tpw;
  if (tpw > INT32_MAX) return fail(SA_ERR_ARG, "batch too large");
  sa::MlpTrainArgs a{};
  a.x = reinterpret_cast<const uint4 *>(x);
  a.y = y;
  a.n = n;
  a.tiles_per_wave = (int)tpw;
  a.waves = (int)w;
  a.master = m->master;
  a.w1f = m->w1f;
  a.partial = m->partial;
  a.loss_partial = m->loss_partial;
  SA_HIP(sa::launch_mlp_train(a, s), "mlp forward/backward");
  waves = (int)w;
  return SA_OK;
}

extern "C" int sa_mlp_gradients(sa_mlp *m, const uint16_t *x, const float *y, int64_t n, float *grad,
                                float *loss, void *stream) {
  if (!m || !x || !y || !grad || n < 1) return fail(SA_ERR_ARG, "NULL argument or n < 1");
  int waves = 0;
  if (int rc = mlp_backward(m, x, y, n, (hipStream_t)stream, waves)) return rc;
  sa::MlpUpdateArgs u{};
  u.partial = m->partial;
  u.loss_partial = m->loss_partial;
  u.waves = waves;
  u.grad_out = grad;
  u.loss_out = loss;
  u.master = m->master;
  u.w1f = m->w1f;
  u.w2f = m->w2f;
  SA_HIP(sa::launch_mlp_update(u, (hipStream_t)stream), "mlp gradient reduction");
  return SA_OK;
}

extern "C" int sa_mlp_train_step(sa_mlp *m, const uint16_t *x, const float *y, int64_t n, float lr, float *loss,
                                 void *stream) {
  if (!m || !x || !y || n < 1) return fail(SA_ERR_ARG, "NULL argument or n < 1");
  if (!(lr > 0.f) || !std::isfinite(lr)) return fail(SA_ERR_ARG, "lr must be positive");
  int waves = 0;
  if (int rc = mlp_backward(m, x, y, n, (hipStream_t)stream, waves)) return rc;
  m->steps += 1;
  sa::MlpUpdateArgs u{};
  u.partial = m->partial;
  u.loss_partial = m->loss_partial;
  u.waves = waves;
  u.loss_out = loss;
  u.adam = 1;
  u.lr = lr;
  const double beta1 = 0.9, beta2 = 0.999;
  u.beta1 = (float)beta1;
  u.beta2 = (float)beta2;
  u.omb1 = (float)(1.0 - beta1);
  u.omb2 = (float)(1.0 - beta2);
  u.eps = 1e-8f;
  u.bc1 = (float)(1.0 - std::pow(beta1, (double)m->steps));
  u.bc2 = (float)(1.0 - std::pow(beta2, (double)m->steps));
  u.master = m->master;
  u.m = m->m;
  u.v = m->v;
  u.w1f = m->w1f;
  u.w2f = m->w2f;
  SA_HIP(sa::launch_mlp_update(u, (hipStream_t)stream), "mlp Adam step");
  return SA_OK;
}
