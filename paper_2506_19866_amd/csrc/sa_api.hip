// sa_api.hip -- host part of the C ABI declared in include/sa_anneal.h:
// validation, problem staging (weights, lambda, register layout of the
// kernels), fixed-point Metropolis tables and stage orchestration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sa_anneal.h"
#include "sa_internal.h"

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
  sa_problem *prob = nullptr;
  sa_run_desc desc{};
  int device = 0;
  int8_t *x0 = nullptr, *xbest = nullptr, *xwin = nullptr;
  int32_t *cbest = nullptr;
  uint32_t *cstats = nullptr, *tau = nullptr;
  sa::StageRecord *rec = nullptr;
  std::vector<size_t> tau_off;
  std::vector<int32_t> dcap;
  int32_t launched = 0;
  hipStream_t stream = nullptr;
  std::vector<hipEvent_t> ev_start, ev_stop;  // per stage, when record_times is set
};

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
  if (d->step_size != 1 && d->step_size != 2) return fail(SA_ERR_DOMAIN, "step_size must be 1 or 2");
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

  // tiles: nm m-tiles of 16 rows hold the nodes, nk k-tiles of 64 columns hold nodes + bias
  int nm = (N + 15) / 16;
  if (N + 1 > 64 * ((nm + 3) / 4)) ++nm;
  const int nk = (nm + 3) / 4;
  if (nm > sa::kMaxTilesM) return fail(SA_ERR_UNSUPPORTED, "n_nodes %d > 191", N);
  const int CG = (C + 15) / 16;
  if (CG > sa::kMaxCondGroups) return fail(SA_ERR_UNSUPPORTED, "n_conditions %d > 64", C);

  // slots: observed nodes first (their states then sit in the first dwords of
  // every lane), round-robin over the four lane groups; bias after the nodes
  std::vector<int> order, obs_index(N, -1);
  for (int o = 0; o < O; ++o) {
    order.push_back(d->obs_nodes[o]);
    obs_index[d->obs_nodes[o]] = o;
  }
  for (int v = 0; v < N; ++v)
    if (obs_index[v] < 0) order.push_back(v);
  std::vector<int> sg(N), sq(N);
  const int slots = 16 * nk;
  std::vector<int16_t> slot_node((size_t)4 * slots, -1);
  for (int k = 0; k < N; ++k) {
    const int v = order[k];
    sg[v] = k % 4;
    sq[v] = k / 4;
    slot_node[(size_t)sg[v] * slots + sq[v]] = (int16_t)v;
  }
  const int gb = N % 4, qb = N / 4;
  int nd = 1;
  for (int o = 0; o < O; ++o) nd = std::max(nd, sq[d->obs_nodes[o]] / 4 + 1);

  // A entry of parameter p: row of its target node i, column of its source
  // node j (edge) or of the bias (theta_i)
  std::vector<uint32_t> param_pos(P);
  std::vector<int32_t> edst(E), esrc(E);
  auto place = [&](int p, int i, int colg, int colq) {
    const int lane = (4 * sg[i] + sq[i] % 4) + 16 * colg;
    const int mt = sq[i] / 4, kt = colq / 16, dw = (colq % 16) / 4, b = colq % 4;
    const int reg = (mt * nk + kt) * 4 + dw;
    param_pos[p] = (uint32_t)lane | ((uint32_t)reg << 8) | ((uint32_t)b << 16);
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

  // per (condition group, dword, lane): initial states and the held-byte mask
  const int Q4 = 4 * nk;
  std::vector<uint32_t> b0((size_t)CG * Q4 * 64), cm((size_t)CG * Q4 * 64);
  std::vector<uint32_t> orr((size_t)CG * K * nd * 64, 0), ow((size_t)CG * K * nd * 64, 0);
  for (int cg = 0; cg < CG; ++cg)
    for (int lane = 0; lane < 64; ++lane) {
      const int c = cg * 16 + lane % 16, g = lane / 16;
      for (int q4 = 0; q4 < Q4; ++q4) {
        uint32_t vb = 0, vm = 0;
        for (int b = 0; b < 4; ++b) {
          const int q = q4 * 4 + b;
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
          vb |= (uint32_t)val << (8 * b);
          vm |= (held ? 0xffu : 0u) << (8 * b);
        }
        const size_t at = ((size_t)cg * Q4 + q4) * 64 + lane;
        b0[at] = vb;
        cm[at] = vm;
      }
      if (c >= C) continue;
      for (int k = 0; k < K; ++k)
        for (int q4 = 0; q4 < nd; ++q4) {
          uint32_t vr = 0, vw = 0;
          for (int b = 0; b < 4; ++b) {
            const int v = slot_node[(size_t)g * slots + q4 * 4 + b];
            if (v < 0 || obs_index[v] < 0) continue;
            const size_t at = ((size_t)c * K + k) * O + obs_index[v];
            vr |= (uint32_t)d->observed[at] << (8 * b);
            vw |= (uint32_t)W[at] << (8 * b);
          }
          const size_t at = (((size_t)cg * K + k) * nd + q4) * 64 + lane;
          orr[at] = vr;
          ow[at] = vw;
        }
    }

  auto *pr = new sa_problem();
  hipGetDevice(&pr->device);
  Layout lay;
  const size_t o_pos = lay.take(param_pos.size() * 4);
  const size_t o_esrc = lay.take((size_t)E * 4), o_edst = lay.take((size_t)E * 4);
  const size_t o_inptr = lay.take((size_t)(N + 1) * 4), o_outptr = lay.take((size_t)(N + 1) * 4);
  const size_t o_outeid = lay.take((size_t)E * 4);
  const size_t o_b0 = lay.take(b0.size() * 4), o_cm = lay.take(cm.size() * 4);
  const size_t o_or = lay.take(orr.size() * 4), o_ow = lay.take(ow.size() * 4);
  const size_t o_obst = lay.take((size_t)K * 4), o_slot = lay.take(slot_node.size() * 2);
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
  put(o_or, orr.data(), orr.size() * 4);
  put(o_ow, ow.data(), ow.size() * 4);
  put(o_obst, d->obs_times, (size_t)K * 4);
  put(o_slot, slot_node.data(), slot_node.size() * 2);
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
  dp.obs_r = (const uint32_t *)(base + o_or);
  dp.obs_w = (const uint32_t *)(base + o_ow);
  dp.obs_t = (const int32_t *)(base + o_obst);
  dp.slot_node = (const int16_t *)(base + o_slot);

  sa_problem_info &in = pr->info;
  in.n_params = P; in.n_nodes = N; in.n_edges = E; in.n_conditions = C; in.n_steps = T;
  in.n_obs_times = K; in.n_obs_nodes = O;
  in.weight_sum = (int32_t)wsum;
  in.penalty = (int32_t)lambda;
  in.max_cost = (int32_t)max_cost;
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
  SA_HIP((hipError_t)sa::launch_eval(p->dev, x, n, cost, stream), "eval launch");
  return SA_OK;
}

extern "C" int sa_simulate(const sa_problem *p, const int8_t *x, int64_t n, int8_t *traj, void *stream) {
  if (!p) return fail(SA_ERR_ARG, "problem is NULL");
  if (n < 0) return fail(SA_ERR_ARG, "n < 0");
  if (n == 0) return SA_OK;
  if (!x || !traj) return fail(SA_ERR_ARG, "NULL device pointer");
  SA_HIP(hipSetDevice(p->device), "hipSetDevice");
  SA_HIP((hipError_t)sa::launch_simulate(p->dev, x, n, traj, stream), "simulate launch");
  return SA_OK;
}

// ---------------------------------------------------------------------------
// runs
// ---------------------------------------------------------------------------
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
  hipFree(r->x0);
  hipFree(r->xbest);
  hipFree(r->xwin);
  hipFree(r->cbest);
  hipFree(r->cstats);
  hipFree(r->tau);
  hipFree(r->rec);
  delete r;
}

extern "C" int sa_run_create(sa_problem *const *probs, int32_t n_probs, const sa_run_desc *desc,
                             const int8_t *x0_dev, sa_run **out, void *stream) {
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!probs || !desc || !x0_dev) return fail(SA_ERR_ARG, "NULL argument");
  if (n_probs != 1) return fail(SA_ERR_UNSUPPORTED, "n_probs must be 1 in this version");
  sa_problem *p = probs[0];
  if (!p) return fail(SA_ERR_ARG, "problem is NULL");
  if (desc->n_chains < 1 || desc->n_chains > (1ll << 31) - 1) return fail(SA_ERR_ARG, "n_chains out of range");
  if (!(desc->T0 > 0) || !(desc->rho > 0)) return fail(SA_ERR_ARG, "T0 and rho must be > 0");
  if (desc->first_stage < 0 || desc->n_stages < 0 || desc->steps_per_stage < 1)
    return fail(SA_ERR_ARG, "stage counts out of range");
  SA_HIP(hipSetDevice(p->device), "hipSetDevice");
  const size_t smem = sa::stage_smem_bytes(p->dev, sa::stage_waves_per_block(p->dev));
  if (smem > 64 * 1024) return fail(SA_ERR_UNSUPPORTED, "stage kernel needs %zu bytes of LDS (> 64 KiB)", smem);
  const int64_t n = desc->n_chains;
  const int P = p->info.n_params, E = p->info.n_edges;
  hipStream_t s = (hipStream_t)stream;

  // starting vectors: domain on the host, constraints (hard mode) on the device
  std::vector<int8_t> hx((size_t)(n * P));
  SA_HIP(hipMemcpyAsync(hx.data(), x0_dev, hx.size(), hipMemcpyDeviceToHost, s), "copy x0");
  SA_HIP(hipStreamSynchronize(s), "sync");
  for (int64_t c = 0; c < n; ++c)
    for (int i = 0; i < P; ++i) {
      const int v = hx[(size_t)c * P + i];
      if (i < E ? (v < -1 || v > 1) : (v < 0 || v > 2))
        return fail(SA_ERR_DOMAIN, "x0 chain %lld parameter %d = %d", (long long)c, i, v);
    }

  auto *r = new sa_run();
  r->prob = p;
  r->desc = *desc;
  r->device = p->device;
  r->stream = s;
  const int S = desc->n_stages;
  std::vector<uint32_t> all_tau, tab;
  double T = desc->T0;
  for (int k = 0; k < desc->first_stage; ++k) T = T * desc->rho;
  for (int st = 0; st < S; ++st) {
    int32_t cap;
    tau_table(T, p->info.max_cost, tab, cap);
    r->tau_off.push_back(all_tau.size());
    r->dcap.push_back(cap);
    all_tau.insert(all_tau.end(), tab.begin(), tab.end());
    T = T * desc->rho;
  }
  hipError_t e = hipSuccess;
  auto alloc = [&](void **ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes ? bytes : 1);
  };
  alloc((void **)&r->x0, (size_t)(n * P));
  alloc((void **)&r->xbest, (size_t)(n * P));
  alloc((void **)&r->xwin, (size_t)P);
  alloc((void **)&r->cbest, (size_t)n * 4);
  alloc((void **)&r->cstats, (size_t)n * 16);
  alloc((void **)&r->tau, all_tau.size() * 4);
  alloc((void **)&r->rec, (size_t)std::max(S, 1) * sizeof(sa::StageRecord));
  for (int st = 0; st < S && desc->record_times && e == hipSuccess; ++st) {
    hipEvent_t a = nullptr, b = nullptr;
    e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    r->ev_start.push_back(a);
    r->ev_stop.push_back(b);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(r->x0, x0_dev, (size_t)(n * P), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess && !all_tau.empty())
    e = hipMemcpyAsync(r->tau, all_tau.data(), all_tau.size() * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && p->dev.hard) {
    // lambda >= 1, so V(x0) = 0 exactly when the cost with lambda equals the
    // cost with lambda = 0 (the mismatch alone)
    e = (hipError_t)sa::launch_eval(p->dev, r->x0, n, r->cbest, s);
    sa::DevProblem m = p->dev;
    m.lambda = 0;
    if (e == hipSuccess) e = (hipError_t)sa::launch_eval(m, r->x0, n, (int32_t *)r->cstats, s);
    std::vector<int32_t> c1((size_t)n), c0((size_t)n);
    if (e == hipSuccess) e = hipMemcpyAsync(c1.data(), r->cbest, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c0.data(), r->cstats, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
      for (int64_t c = 0; c < n; ++c)
        if (c1[(size_t)c] != c0[(size_t)c]) {
          free_run(r);
          return fail(SA_ERR_INFEASIBLE, "x0 of chain %lld breaks a structural constraint", (long long)c);
        }
  }
  if (e != hipSuccess) {
    free_run(r);
    return hip_fail(e, "run setup");
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
  const sa::DevProblem &pb = r->prob->dev;
  const int P = pb.P;
  for (int32_t i = 0; i < n_stages; ++i) {
    const int32_t st = r->launched;
    sa::StageArgs a{};
    a.n_chains = r->desc.n_chains;
    a.seed = r->desc.seed;
    a.net = 0;
    a.stage = r->desc.first_stage + st;
    a.L = r->desc.steps_per_stage;
    a.dcap = r->dcap[st];
    a.tau = r->tau + r->tau_off[st];
    a.x_start = st == 0 ? r->x0 : r->xwin;
    a.x_start_stride = st == 0 ? P : 0;
    a.xbest = r->xbest;
    a.cbest = r->cbest;
    a.cstats = r->cstats;
    const bool timed = !r->ev_start.empty();
    if (timed) SA_HIP(hipEventRecord(r->ev_start[st], (hipStream_t)stream), "event record");
    SA_HIP((hipError_t)sa::launch_stage(pb, a, stream), "stage launch");
    if (timed) SA_HIP(hipEventRecord(r->ev_stop[st], (hipStream_t)stream), "event record");
    sa::ReduceArgs ra{};
    ra.n_chains = r->desc.n_chains;
    ra.P = P;
    ra.cbest = r->cbest;
    ra.xbest = r->xbest;
    ra.cstats = r->cstats;
    ra.xwin = r->xwin;
    ra.rec = r->rec + st;
    SA_HIP((hipError_t)sa::launch_reduce(ra, stream), "reduce launch");
    r->launched++;
  }
  r->stream = (hipStream_t)stream;
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
  if (prob != 0) return fail(SA_ERR_ARG, "problem index %d out of range", prob);
  SA_HIP(hipSetDevice(r->device), "hipSetDevice");
  SA_HIP(hipStreamSynchronize(r->stream), "stream sync");
  return SA_OK;
}

extern "C" int sa_best(sa_run *r, int32_t prob, int8_t *x_host, int32_t *cost, int32_t *winner) {
  int rc = sync_run(r, prob);
  if (rc != SA_OK) return rc;
  if (r->launched == 0) return fail(SA_ERR_ARG, "no stage launched");
  sa::StageRecord rec;
  SA_HIP(hipMemcpy(&rec, r->rec + (r->launched - 1), sizeof(rec), hipMemcpyDeviceToHost), "copy record");
  if (x_host) SA_HIP(hipMemcpy(x_host, r->xwin, (size_t)r->prob->dev.P, hipMemcpyDeviceToHost), "copy best");
  if (cost) *cost = rec.best_cost;
  if (winner) *winner = rec.winner;
  return SA_OK;
}

extern "C" int sa_stats(sa_run *r, int32_t prob, sa_stage_stats *out) {
  int rc = sync_run(r, prob);
  if (rc != SA_OK) return rc;
  if (!out) return fail(SA_ERR_ARG, "out is NULL");
  std::vector<sa::StageRecord> rec((size_t)r->launched);
  if (r->launched)
    SA_HIP(hipMemcpy(rec.data(), r->rec, rec.size() * sizeof(sa::StageRecord), hipMemcpyDeviceToHost),
           "copy records");
  for (int32_t i = 0; i < r->launched; ++i) {
    out[i].best_cost = rec[i].best_cost;
    out[i].winner = rec[i].winner;
    out[i].accepted = rec[i].accepted;
    out[i].uphill = rec[i].uphill;
    out[i].neutral = rec[i].neutral;
    out[i].infeasible = rec[i].infeasible;
  }
  return SA_OK;
}

extern "C" int sa_chain_best(sa_run *r, int32_t prob, int32_t *cost, int8_t *x_host) {
  int rc = sync_run(r, prob);
  if (rc != SA_OK) return rc;
  const int64_t n = r->desc.n_chains;
  if (cost) SA_HIP(hipMemcpy(cost, r->cbest, (size_t)n * 4, hipMemcpyDeviceToHost), "copy chain costs");
  if (x_host)
    SA_HIP(hipMemcpy(x_host, r->xbest, (size_t)(n * r->prob->dev.P), hipMemcpyDeviceToHost), "copy chain bests");
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
