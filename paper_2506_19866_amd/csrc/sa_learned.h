// sa_learned.h -- the learned proposal inside the annealing loop.  An
// extension of Table 1's GetCandidate (not in the paper): every R steps a
// chain rebuilds a sampling table over its 2P single-parameter moves,
//   1. one extra simulation of its current vector (the MFMA simulation of
//      sa_device.h) that also sums, per node, the states, W*S and W*|S - R|
//      at the observed times;
//   2. the 32 features of every move (definitions below);
//   3. the network's score of every move, 16 moves per bf16 MFMA tile
//      (sa_mlp.h);
//   4. integer weights floor(exp(score - max) * 2^16), 0 for moves that would
//      break a structural constraint in hard mode, and their prefix sums;
// and each step draws its candidate from that table with the Philox words of
// the plain method (word 0 picks the move, word 3 decides the plain
// fallback).  Everything after the candidate -- constraints (§2.5.3), full
// simulation (§2.2), score (§2.3), Metropolis and restart (Table 1) -- is the
// plain chain loop of sa_chain.h, so the exact integer cost decides.
//
// Features of move p: old -> v (p an edge j -> i, or the threshold of i);
// float32 in this order of operations, then rounded to bf16:
//   0-2 one-hot code(old)   3-5 one-hot code(v)   6 threshold   7 e = (v-old)/2 (edge), (old-v)/2
//   8 i observed   9 eh_i   10 ah_i   11 msh_j   12 msh_i   13 e*eh_i   14 (e*msh_j)*eh_i (edge; else 13)
//   15 j observed   16 eh_j   17 in-degree(i)/8   18 out-degree(j)/8   19 ln(T)/5   20 M/sum W
//   21 raises V   22 (+1 in-edges of i)/8   23 (non-zero out-edges of j)/8   24-30 zero   31 one
// with msh = (sum of states)/(2 C K), eh = (sum W*R - sum W*S)/(2 sum W),
// ah = (sum W*|S-R|)/(2 sum W) over the node's observations (0 unobserved);
// edge-only features are 0 for a threshold.
#pragma once
#include "sa_chain.h"
#include "sa_mlp.h"

namespace sa {

// Table area of a wave: the 2P cumulative weights, or the 3 x 128*nk slot
// aggregates while a refresh runs.
__host__ __device__ inline int learned_tbl_words(const DevProblem &pb) {
  return 2 * pb.P > 3 * 128 * pb.nk ? 2 * pb.P : 3 * 128 * pb.nk;
}
// Feature rows of 32 moves staged between their computation and the tiles.
constexpr int kStageMoves = 16;
// LDS of one chain: the plain chain area, the vector at the last refresh
// [P4], the table, three float node features [N4] each, and the staged
// feature rows (32 x 64 bytes).
__host__ __device__ inline int learned_wave_bytes(const DevProblem &pb) {
  return chain_lds_bytes(pb) + round4(pb.P) + 4 * learned_tbl_words(pb) + 12 * round4(pb.N) + 64 * kStageMoves;
}

// nibble-wise w * v for nibbles w <= 3, v <= 2 (products <= 6: no carries)
__device__ __forceinline__ uint32_t nib_mul_small(uint32_t w, uint32_t v) {
  const uint32_t m1 = (v & kLowNibbles) * 0xfu, m2 = ((v >> 1) & kLowNibbles) * 0xfu;
  return (w & m1) + ((w << 1) & m2);
}

// The refresh simulation: simulates every condition for the vector in A and
// adds, per slot, the states (agg[0]), W*S (agg[1]) and W*|S - R| (agg[2])
// summed over observed times and conditions.  Per lane the sums of the even
// and of the odd nibbles stay in bytes (at most 6 per observed time:
// K <= 42), then the 16 condition lanes of a lane group are added in 16-bit
// halves.  Returns M = sum of W*|S - R|.
template <int NM, int NK, int D>
__device__ __forceinline__ int refresh_simulation(const ATile<NM, NK> &A, const DevProblem &pb, int lane,
                                                  const uint32_t *obs_r, const uint32_t *obs_w, uint32_t *agg) {
  constexpr int kSlots = 128 * NK;
  for (int i = lane; i < 3 * kSlots; i += kWave) agg[i] = 0u;
  wave_sync();
  const int g = lane >> 4;
  for (int cg = 0; cg < pb.CG; ++cg) {
    v4i B0[NK], B1[NK], CM[NK];
#pragma unroll
    for (int kt = 0; kt < NK; ++kt)
#pragma unroll
      for (int dw = 0; dw < 4; ++dw) {
        const int at = (cg * 4 * NK + kt * 4 + dw) * kWave + lane;
        B0[kt][dw] = (int)pb.b0[at];
        CM[kt][dw] = (int)pb.cmask[at];
      }
    const bool live = cg * 16 + (lane & 15) < pb.C;
    const uint32_t *rbase = obs_r + (size_t)cg * pb.K * pb.nd * kWave;
    const uint32_t *wbase = obs_w + (size_t)cg * pb.K * pb.nd * kWave;
    // [2 * q4 + parity]: sums of the even (0) and odd (1) nibbles of dword q4
    uint32_t aS[8 * NK], aWS[8 * NK], aWA[8 * NK];
#pragma unroll
    for (int q = 0; q < 8 * NK; ++q) aS[q] = aWS[q] = aWA[q] = 0u;
    auto add_nibbles = [](uint32_t *acc, int q4, uint32_t v) SA_INLINE {
      acc[2 * q4] += v & 0x0f0f0f0fu;
      acc[2 * q4 + 1] += (v >> 4) & 0x0f0f0f0fu;
    };
    int k = 0, tnext = load_uniform(pb.obs_t, 0);
    auto observe = [&](const v4i (&B)[NK], int t) SA_INLINE {
      if (t != tnext) return;
#pragma unroll
      for (int q4 = 0; q4 < 4 * NK; ++q4) {
        const uint32_t code = (uint32_t)B[q4 >> 2][q4 & 3];
        const uint32_t s = state_values(code);
        if (live) add_nibbles(aS, q4, s);
        if (q4 < pb.nd) {
          const uint32_t r = rbase[((size_t)k * pb.nd + q4) * kWave + lane];
          const uint32_t w = wbase[((size_t)k * pb.nd + q4) * kWave + lane];
          add_nibbles(aWA, q4, nib_mul_small(w, state_values(code ^ r)));  // |S - R| per nibble
          add_nibbles(aWS, q4, nib_mul_small(w, s));
        }
      }
      ++k;
      tnext = k < pb.K ? load_uniform(pb.obs_t, k) : -1;
    };
    observe(B0, 0);
    const int t_end = load_uniform(pb.obs_t, pb.K - 1);  // later states enter no aggregate
    int t = 1;
    for (; t + 1 <= t_end; t += 2) {
      time_step<NM, NM, NK, D>(A, B0, B1, CM);
      observe(B1, t);
      time_step<NM, NM, NK, D>(A, B1, B0, CM);
      observe(B0, t + 1);
    }
    if (t <= t_end) {
      time_step<NM, NM, NK, D>(A, B0, B1, CM);
      observe(B1, t);
    }
    // byte b of a parity-p accumulator holds nibble 2b + p: slot 8*q4 + 2b + p
    auto fold = [&](uint32_t v, uint32_t *dst) SA_INLINE {
      uint32_t lo = v & 0x00ff00ffu, hi = (v >> 8) & 0x00ff00ffu;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        lo += (uint32_t)__shfl_xor((int)lo, off, kWave);
        hi += (uint32_t)__shfl_xor((int)hi, off, kWave);
      }
      if ((lane & 15) == 0) {
        dst[0] += lo & 0xffffu;
        dst[2] += hi & 0xffffu;
        dst[4] += lo >> 16;
        dst[6] += hi >> 16;
      }
    };
#pragma unroll
    for (int q4 = 0; q4 < 4 * NK; ++q4)
#pragma unroll
      for (int par = 0; par < 2; ++par) {
        const int slot = g * 32 * NK + q4 * 8 + par;
        fold(aS[2 * q4 + par], agg + slot);
        fold(aWS[2 * q4 + par], agg + kSlots + slot);
        fold(aWA[2 * q4 + par], agg + 2 * kSlots + slot);
      }
    wave_sync();
  }
  int m = 0;
  for (int s = lane; s < kSlots; s += kWave) m += (int)agg[2 * kSlots + s];
  return uniform(wave_sum(m));
}

// Per-node float features of the refresh from the slot aggregates.
__device__ __forceinline__ void node_features(const DevProblem &pb, int lane, const uint32_t *agg, float *msh,
                                              float *eh, float *ah) {
  const int slots = 128 * pb.nk;
  const float den_s = (float)(2 * pb.C * pb.K);
  for (int i = lane; i < pb.N; i += kWave) {
    const int s = pb.node_slot[i];
    msh[i] = (float)(int)agg[s] / den_s;
    const int sw = pb.node_sw[i];
    float e = 0.f, a = 0.f;
    if (sw > 0) {
      const float den = (float)(2 * sw);
      e = (float)(pb.node_wr[i] - (int)agg[slots + s]) / den;
      a = (float)(int)agg[2 * slots + s] / den;
    }
    eh[i] = e;
    ah[i] = a;
  }
}

struct NodeFeatures {
  const float *msh, *eh, *ah;
  float lt, mn;
};

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
  const v2bf t = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, t);
}

// The 32 features of the move p: old -> v as bf16 pairs (feature 2q in the
// low half of word q), and whether the move raises V.
__device__ __forceinline__ void move_feature_words(int p, int old, int v, const uint32_t *pinfo, const NodeFeatures &nf,
                                                   const uint8_t *outnz, const uint8_t *inplus, bool &raises,
                                                   uint4 (&out)[4]) {
  const uint32_t info = pinfo[p];
  const int i = (int)(info & 127u), j = (int)((info >> 7) & 127u);
  const int indeg = (int)((info >> 14) & 127u), outdeg = (int)((info >> 21) & 127u);
  const bool edge = (info >> 28) & 1u, obs_i = (info >> 29) & 1u, obs_j = (info >> 30) & 1u;
  const int co = edge ? old + 1 : old, cn = edge ? v + 1 : v;
  const float e = edge ? (float)(v - old) / 2.f : (float)(old - v) / 2.f;
  const float eh_i = nf.eh[i], ah_i = nf.ah[i], msh_i = nf.msh[i];
  const float msh_j = edge ? nf.msh[j] : 0.f, eh_j = edge ? nf.eh[j] : 0.f;
  const float f13 = e * eh_i;
  const float f14 = edge ? (e * msh_j) * eh_i : f13;
  const int on_j = outnz[j], ip_i = inplus[i];
  const int on_new = on_j + (v != 0) - (old != 0), ip_new = ip_i + (v == 1) - (old == 1);
  raises = edge && ((on_new == 0 && on_j > 0) || (ip_new == 0 && ip_i > 0));
  out[0] = make_uint4(pack_bf16x2(co == 0 ? 1.f : 0.f, co == 1 ? 1.f : 0.f),
                      pack_bf16x2(co == 2 ? 1.f : 0.f, cn == 0 ? 1.f : 0.f),
                      pack_bf16x2(cn == 1 ? 1.f : 0.f, cn == 2 ? 1.f : 0.f), pack_bf16x2(edge ? 0.f : 1.f, e));
  out[1] = make_uint4(pack_bf16x2(obs_i ? 1.f : 0.f, eh_i), pack_bf16x2(ah_i, msh_j), pack_bf16x2(msh_i, f13),
                      pack_bf16x2(f14, obs_j ? 1.f : 0.f));
  out[2] = make_uint4(pack_bf16x2(eh_j, (float)indeg / 8.f), pack_bf16x2((float)outdeg / 8.f, nf.lt),
                      pack_bf16x2(nf.mn, raises ? 1.f : 0.f),
                      pack_bf16x2((float)ip_i / 8.f, edge ? (float)on_j / 8.f : 0.f));
  out[3] = make_uint4(0u, 0u, 0u, pack_bf16x2(0.f, 1.f));
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
  return v;
}

template <int NM, int NK, int D>
struct LearnedHooks {
  static constexpr bool kEnabled = true;
  const DevProblem *pb;
  LearnedArgs la;
  const uint32_t *pinfo;     // LDS copy of the parameter descriptors
  const uint4 *w1f, *w2f;    // the network fragments (global memory), or null
  uint8_t *xref;             // vector at the last refresh
  uint32_t *tbl;             // cumulative weights (or aggregates during a refresh)
  float *msh, *eh, *ah;
  uint4 *fst;                // staged feature rows [kStageMoves][4]
  float b2, mn;
  uint32_t total;
  TraceRecord *trace;        // this chain's records, or null

  __device__ __forceinline__ NodeFeatures nodes() const { return {msh, eh, ah, la.lt, mn}; }

  __device__ __forceinline__ void refresh(const ATile<NM, NK> &A, int it, const uint8_t *xcur, const uint8_t *outnz,
                                          const uint8_t *inplus, int, int, int lane, const uint32_t *lds_r,
                                          const uint32_t *lds_w) {
    if (it % la.refresh != 0) return;
    const int m = refresh_simulation<NM, NK, D>(A, *pb, lane, lds_r, lds_w, tbl);
    node_features(*pb, lane, tbl, msh, eh, ah);
    mn = (float)m / (float)pb->sum_w;
    wave_sync();
    if (!w1f) return;
    const int P = pb->P, E = pb->E, M2 = 2 * P;
    for (int i = lane; i < round4(P) / 4; i += kWave)
      reinterpret_cast<uint32_t *>(xref)[i] = reinterpret_cast<const uint32_t *>(xcur)[i];
    const int g = lane >> 4, r = lane & 15;
    const NodeFeatures nf = nodes();
    // scores of all moves; masked moves score -inf.  Lanes 0-31 compute the
    // feature rows of 32 moves once, the two tiles read them back as MFMA
    // operands; lane 16t + r holds move r of tile t, so it also stores that
    // move's score.
    for (int m0 = 0; m0 < M2; m0 += kStageMoves) {
      const int mm = m0 + lane;
      bool raises = false;
      if (lane < kStageMoves) {
        uint4 w[4] = {make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u),
                      make_uint4(0u, 0u, 0u, 0u)};
        if (mm < M2) {
          const int p = mm >> 1;
          const int old = (int)(int8_t)xcur[p];
          const bool edge = p < E;
          const int cn = ((edge ? old + 1 : old) + 1 + (mm & 1)) % 3;
          move_feature_words(p, old, edge ? cn - 1 : cn, pinfo, nf, outnz, inplus, raises, w);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) fst[lane * 4 + q] = w[q];
      }
      wave_sync();
#pragma unroll
      for (int t = 0; t < kStageMoves / 16; ++t) {
        if (m0 + 16 * t >= M2) break;
        const float l = mlp_tile_logit(as_v8bf(fst[(16 * t + r) * 4 + g]), w1f, w2f, lane, b2);
        if (g == t && mm < M2) tbl[mm] = __float_as_uint((pb->hard && raises) ? -INFINITY : l);
      }
      wave_sync();
    }
    // integer weights and their inclusive prefix sums, one contiguous chunk per lane
    float lmax = -INFINITY;
    for (int i = lane; i < M2; i += kWave) lmax = fmaxf(lmax, __uint_as_float(tbl[i]));
    lmax = wave_max_f(lmax);
    const int ch = (M2 + kWave - 1) / kWave;
    const int b0 = min(lane * ch, M2), b1 = min(b0 + ch, M2);
    uint32_t local = 0;
    for (int i = b0; i < b1; ++i) {
      const float l = __uint_as_float(tbl[i]);
      const uint32_t w = l == -INFINITY ? 0u : (uint32_t)floorf(expf(l - lmax) * 65536.f);
      tbl[i] = w;
      local += w;
    }
    uint32_t incl = local;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t t = (uint32_t)__shfl_up((int)incl, off, kWave);
      if (lane >= off) incl += t;
    }
    uint32_t run = incl - local;
    for (int i = b0; i < b1; ++i) {
      run += tbl[i];
      tbl[i] = run;
    }
    total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    wave_sync();
  }

  // Candidate from the table: the first move whose cumulative weight exceeds
  // ((word 0) * total) >> 32.  Declines (plain candidate) when no network is
  // loaded, when word 3 selects the plain fallback, when the table is empty,
  // or when the chain already holds the move's value.
  __device__ __forceinline__ bool select(uint32_t r0, uint32_t r3, const uint8_t *xcur, int &p, int &nv, int &source,
                                         int lane) {
    source = 0;
    if (!w1f || (uint64_t)r3 < la.eps_u) return false;
    if (total == 0u) {
      source = 3;
      return false;
    }
    const uint32_t rr = (uint32_t)(((uint64_t)r0 * (uint64_t)total) >> 32);
    const int M2 = 2 * pb->P, ch = (M2 + kWave - 1) / kWave;
    const int c0 = lane * ch;
    const bool hit = c0 < M2 && tbl[min(c0 + ch, M2) - 1] > rr;
    const int f = __ffsll((unsigned long long)__ballot(hit)) - 1;  // exists: the last entry is total > rr
    const int end = min(f * ch + ch, M2);
    int m = -1;
    for (int base = f * ch; m < 0; base += kWave) {
      const int idx = base + lane;
      const unsigned long long b = __ballot(idx < end && tbl[idx] > rr);
      if (b) m = base + __ffsll(b) - 1;
    }
    p = m >> 1;
    const int ref = (int)(int8_t)xref[p];
    const bool edge = p < pb->E;
    const int cn = ((edge ? ref + 1 : ref) + 1 + (m & 1)) % 3;
    const int v = edge ? cn - 1 : cn;
    if ((int)(int8_t)xcur[p] == v) {
      source = 2;
      return false;
    }
    nv = v;
    source = 1;
    return true;
  }

  __device__ __forceinline__ void record(uint64_t gstep, int p, int old, int nv, bool feasible, int delta,
                                         bool accept, int source, const uint8_t *outnz, const uint8_t *inplus,
                                         int lane) {
    if (!trace) return;
    const int64_t rel = (int64_t)gstep - la.trace_first;
    if (rel < 0 || rel % la.trace_every != 0) return;
    const int64_t slot = rel / la.trace_every;
    if (slot >= la.trace_cap) return;
    TraceRecord *rec = trace + slot;
    if (lane == 0) {
      bool raises;
      uint4 w[4];
      move_feature_words(p, old, nv, pinfo, nodes(), outnz, inplus, raises, w);
#pragma unroll
      for (int q = 0; q < 4; ++q) reinterpret_cast<uint4 *>(rec->features)[q] = w[q];
      rec->param = p;
      rec->value = nv;
      rec->delta = feasible ? delta : 0;
      rec->flags = (accept ? 1u : 0u) | (feasible ? 2u : 0u) | ((uint32_t)source << 2);
    }
  }
};

}  // namespace sa
