// sa_priority.h -- device building blocks of the paper's own model: weight,
// polarity and threshold per edge (image of §2.1), speed, memory and step size
// per node driving the priority update of §2.2, constraints of §2.5.3.
// Method: Reimer et al., arXiv 2506.19866.
//
// Layout: a chain owns a segment of LC lanes (LC = 16, 32 or 64, the smallest
// that holds its N nodes), so a wave runs 64 / LC chains side by side; node i
// lives on lane i of its segment.  A time step needs the states of a node's
// regulators.  They come from two wave ballots, [s >= 1] and [s >= 2], shifted
// to the segment: since s div 1 = [s >= 1] + [s >= 2] and s div 2 = [s >= 2],
// the image of node i is a signed sum of population counts of those two
// ballots under per-node regulator masks (set j belongs to a mask of node i
// when edge j -> i has the matching threshold and product w * p):
//   A1p/A2p/A1n/A2n: t = 1 and w*p >= 1 / = 2 / <= -1 / = -2   (against [s >= 1])
//   B1p/B2p/B1n/B2n: any t and the same products                (against [s >= 2])
//   K_i = |g1&A1p| + |g1&A2p| + |g2&B1p| + |g2&B2p|
//       - |g1&A1n| - |g1&A2n| - |g2&B1n| - |g2&B2n|.
// The highest priority of a step is a maximum over the segment (DPP within
// rows of 16 lanes, lane shuffles across rows).  No LDS traffic per time step
// beyond one byte of reference data.
#pragma once
#include "sa_device.h"

namespace sa {

template <int LC>
using SegMask = typename std::conditional<LC == 64, uint64_t, uint32_t>::type;

// Regulator masks of one node (plus nz: sources of its in-edges with w != 0).
template <int LC>
struct PrMasks {
  SegMask<LC> a1p, a2p, a1n, a2n, b1p, b2p, b1n, b2n, nz;
};

// Set or clear bit `bit` of every mask for an edge with weight w, polarity p
// and threshold t.
template <int LC>
__device__ __forceinline__ void pr_set_edge(PrMasks<LC> &m, SegMask<LC> bit, int w, int p, int t) {
  const int coef = w * p;
  const bool t1 = t == 1;
  auto put = [bit](SegMask<LC> &f, bool on) { f = (f & ~bit) | (on ? bit : (SegMask<LC>)0); };
  put(m.a1p, t1 && coef >= 1);
  put(m.a2p, t1 && coef == 2);
  put(m.a1n, t1 && coef <= -1);
  put(m.a2n, t1 && coef == -2);
  put(m.b1p, coef >= 1);
  put(m.b2p, coef == 2);
  put(m.b1n, coef <= -1);
  put(m.b2n, coef == -2);
  put(m.nz, w != 0);
}

template <int LC>
__device__ __forceinline__ int pr_popc(SegMask<LC> v) {
  if constexpr (LC == 64)
    return __builtin_popcountll(v);
  else
    return __builtin_popcount(v);
}

// Bits of the segment's lanes in a wave ballot, lane i of the segment at bit i.
template <int LC>
__device__ __forceinline__ SegMask<LC> seg_ballot(bool pred, int base) {
  const uint64_t b = __builtin_amdgcn_ballot_w64(pred);
  if constexpr (LC == 64)
    return b;
  else
    return (uint32_t)(b >> base);
}

// Maximum / sum / or over the LC lanes of the segment, in every lane of it:
// quad_perm swaps (lanes 1,0,3,2 and 2,3,0,1) and row rotations by 4 and 8
// give the maximum of each row of 16 lanes; shuffles across rows finish it.
template <int LC, typename Op>
__device__ __forceinline__ int seg_reduce(int v, Op op) {
  v = op(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
  v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
  v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, false));  // row_ror:4
  v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false));  // row_ror:8
  if constexpr (LC >= 32) v = op(v, __shfl_xor(v, 16));
  if constexpr (LC == 64) v = op(v, __shfl_xor(v, 32));
  return v;
}

template <int LC>
__device__ __forceinline__ int seg_max(int v) {
  return seg_reduce<LC>(v, [](int a, int b) { return a > b ? a : b; });
}
template <int LC>
__device__ __forceinline__ int seg_sum(int v) {
  return seg_reduce<LC>(v, [](int a, int b) { return a + b; });
}
template <int LC>
__device__ __forceinline__ SegMask<LC> seg_or(SegMask<LC> v) {
  auto orr = [](int a, int b) { return a | b; };
  if constexpr (LC == 64) {
    const uint32_t lo = (uint32_t)seg_reduce<LC>((int)(uint32_t)v, orr);
    const uint32_t hi = (uint32_t)seg_reduce<LC>((int)(uint32_t)(v >> 32), orr);
    return (uint64_t)hi << 32 | lo;
  } else {
    return (uint32_t)seg_reduce<LC>((int)v, orr);
  }
}

// Lane `base + j` of the segment's value v (j the same in every lane).
template <int LC>
__device__ __forceinline__ uint32_t seg_bcast(uint32_t v, int base, int j) {
  if constexpr (LC == 64)
    return (uint32_t)__builtin_amdgcn_readlane((int)v, j);
  else
    return (uint32_t)__shfl((int)v, base + j);
}

// Masks and node parameters of this lane's node from a parameter vector
// (xv(k) reads element k).
template <int LC, typename XV>
__device__ __forceinline__ void pr_build(const DevProblem &pb, int li, XV xv, PrMasks<LC> &m, int &u, int &mem,
                                         int &d) {
  m = PrMasks<LC>{};
  u = mem = d = 0;
  if (li >= pb.N) return;
  const int E = pb.E, N = pb.N;
  for (int e = pb.in_ptr[li]; e < pb.in_ptr[li + 1]; ++e)
    pr_set_edge<LC>(m, (SegMask<LC>)1 << pb.edge_src[e], xv(e), xv(E + e), xv(2 * E + e));
  u = xv(3 * E + li);
  mem = xv(3 * E + N + li);
  d = xv(3 * E + 2 * N + li);
}

// §2.5.3 for the segment: nodes without an in-edge with p = +1 and w != 0,
// plus nodes without an out-edge with w != 0 (a bit of some node's nz mask).
template <int LC>
__device__ __forceinline__ int pr_violations(const DevProblem &pb, int li, const PrMasks<LC> &m) {
  const SegMask<LC> sources = seg_or<LC>(m.nz);
  int v = 0;
  if (li < pb.N) v = (m.b1p == 0) + (int)(((sources >> li) & 1) == 0);
  return seg_sum<LC>(v);
}

// This lane's share of the weighted mismatch of §2.3 under every condition
// (the trajectory of §2.2's priority update); with TRAJ and a non-null traj
// the states of every step are written to traj[(c*(T+1) + t)*N + node].
// Every lane of the wave must call it together (ballots, reductions).
template <int LC, bool TRAJ>
__device__ __forceinline__ int pr_mismatch(const DevProblem &pb, int li, int base, const PrMasks<LC> &m, int u,
                                           int mem, int d, const uint8_t *start, const uint8_t *obs,
                                           int8_t *traj) {
  const int T = pb.T;
  int acc = 0;
  for (int c = 0; c < pb.C; ++c) {
    const int st = start[c * LC + li];
    int s = st & 3;
    const bool held = (st & 4) != 0;
    int idle = 0, streak = 0;
    const uint8_t *oc = obs + (size_t)c * (T + 1) * LC + li;
    {
      const int ob = oc[0];
      acc += (ob >> 2) * abs(s - (ob & 3));
    }
    if (TRAJ && traj && li < pb.N) traj[(size_t)c * (T + 1) * pb.N + li] = (int8_t)s;
    for (int t = 1; t <= T; ++t) {
      const SegMask<LC> g1 = seg_ballot<LC>(s >= 1, base), g2 = seg_ballot<LC>(s >= 2, base);
      const int img = pr_popc<LC>(g1 & m.a1p) + pr_popc<LC>(g1 & m.a2p) + pr_popc<LC>(g2 & m.b1p) +
                      pr_popc<LC>(g2 & m.b2p) - pr_popc<LC>(g1 & m.a1n) - pr_popc<LC>(g1 & m.a2n) -
                      pr_popc<LC>(g2 & m.b1n) - pr_popc<LC>(g2 & m.b2n);
      const int goal = img < 0 ? 0 : (img > 2 ? 2 : img);
      const bool told = !held && goal != s;
      idle += held ? 0 : 1;
      streak = told ? streak + 1 : 0;
      const int prio = (told && streak > mem) ? u * idle : 0;
      const int best = seg_max<LC>(prio);
      if (prio > 0 && prio == best) {
        const int gap = goal - s;
        const int step = min(abs(gap), d);
        s += gap > 0 ? step : -step;
        idle = 0;
        streak = 0;
      }
      const int ob = oc[(size_t)t * LC];
      acc += (ob >> 2) * abs(s - (ob & 3));
      if (TRAJ && traj && li < pb.N) traj[((size_t)c * (T + 1) + t) * pb.N + li] = (int8_t)s;
    }
  }
  return acc;
}

// Domain of element k of the priority model's vector: block 0 w, 1 p, 2 t
// (edges), 3 u, 4 m, 5 d (nodes); codes 0..size-1 in value order.
__device__ __forceinline__ int pr_block(int k, int E, int N) {
  return k < E ? 0 : k < 2 * E ? 1 : k < 3 * E ? 2 : k < 3 * E + N ? 3 : k < 3 * E + 2 * N ? 4 : 5;
}
__device__ __forceinline__ int pr_domain_size(int blk) { return blk == 3 ? 9 : (blk == 2 || blk == 5) ? 2 : 3; }
__device__ __forceinline__ int pr_code(int blk, int v) {
  switch (blk) {
    case 1: return v + 1;
    case 2: case 5: return v - 1;
    case 3: return v <= 6 ? v - 1 : v - 4;
    default: return v;
  }
}
__device__ __forceinline__ int pr_value(int blk, int code) {
  switch (blk) {
    case 1: return code - 1;
    case 2: case 5: return code + 1;
    case 3: return code < 6 ? code + 1 : code + 4;
    default: return code;
  }
}

}  // namespace sa
