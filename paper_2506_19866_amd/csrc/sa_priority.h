// sa_priority.h -- device building blocks of the paper's own model: weight,
// polarity and threshold per edge (image of §2.1), speed, memory and step size
// per node driving the priority update of §2.2, constraints of §2.5.3.
// Method: Reimer et al., arXiv 2506.19866.
//
// Layout: a chain owns a segment of LC lanes (LC = 16, 32 or 64, the smallest
// that holds its N nodes), so a wave runs 64 / LC chains side by side; node i
// lives on lane i of its segment and keeps its state, its idle and telling
// counts and its own parameters in registers.  A time step needs the states
// of a node's regulators, gathered in one of two ways (chosen per network):
//
//  * sparse (DMAX = 8 or 16 >= the largest in-degree): one slot per in-edge
//    holding the source lane's byte address and a table of the edge's three
//    possible contributions (s div t) * w * p for s = 0, 1, 2 as signed
//    bytes; every lane publishes its state as a one-hot byte code, a lane
//    permute (ds_bpermute) fetches it from each source lane and a 4-byte dot
//    product (v_dot4_i32_i8) with the table adds the contribution;
//  * dense (DMAX = 0): two wave ballots, [s >= 1] and [s >= 2], shifted to the
//    segment; since s div 1 = [s >= 1] + [s >= 2] and s div 2 = [s >= 2], the
//    image is a signed sum of population counts of those ballots under eight
//    per-node regulator masks (threshold 1 or any, w*p >= 1, = 2, <= -1, = -2).
//
// The highest priority of a step is a maximum over the segment: DPP within
// rows of 16 lanes, then gfx950's row swap (v_permlane16_swap) for a 32-lane
// segment, or the DPP row broadcasts and one lane read for a whole wave.  Two
// more masks per node (sources with w != 0, and whether an in-edge has p = +1
// and w != 0) give the constraint count.
#pragma once
#include <climits>

#include "sa_device.h"

namespace sa {

template <int LC>
using SegMask = typename std::conditional<LC == 64, uint64_t, uint32_t>::type;

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
  else if constexpr (LC == 32)
    return (uint32_t)(b >> base);
  else
    return (uint32_t)(b >> base) & 0xffffu;
}

// Maximum / sum / or over the LC lanes of the segment, in every lane of it:
// quad_perm swaps (lanes 1,0,3,2 and 2,3,0,1) and row rotations by 4 and 8
// reduce each row of 16 lanes.  A 32-lane segment then pairs rows 0-1 and
// 2-3 by the row swap.  A whole wave instead lets rows 1 and 3 take the last
// lane of the row before (row_bcast:15) and rows 2 and 3 lane 31
// (row_bcast:31), each fused into the operation, so that lane 63 holds the
// result, read into a scalar; `id` is the operation's identity, the value
// lanes of the rows a broadcast leaves out combine with.
template <int LC, typename Op>
__device__ __forceinline__ int seg_reduce(int v, Op op, int id) {
  v = op(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
  v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
  v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, false));  // row_ror:4
  v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false));  // row_ror:8
  if constexpr (LC == 32) {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    v = op((int)r[0], (int)r[1]);
  }
  if constexpr (LC == 64) {
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));  // row_bcast:15, rows 1 and 3
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));  // row_bcast:31, rows 2 and 3
    v = __builtin_amdgcn_readlane(v, 63);
  }
  return v;
}

template <int LC>
__device__ __forceinline__ int seg_max(int v) {
  return seg_reduce<LC>(v, [](int a, int b) { return a > b ? a : b; }, INT_MIN);
}
template <int LC>
__device__ __forceinline__ int seg_sum(int v) {
  return seg_reduce<LC>(v, [](int a, int b) { return a + b; }, 0);
}
template <int LC>
__device__ __forceinline__ SegMask<LC> seg_or(SegMask<LC> v) {
  auto orr = [](int a, int b) { return a | b; };
  if constexpr (LC == 64) {
    const uint32_t lo = (uint32_t)seg_reduce<LC>((int)(uint32_t)v, orr, 0);
    const uint32_t hi = (uint32_t)seg_reduce<LC>((int)(uint32_t)(v >> 32), orr, 0);
    return (uint64_t)hi << 32 | lo;
  } else {
    return (uint32_t)seg_reduce<LC>((int)v, orr, 0);
  }
}

// Lane `base + j` of the segment's value v (j the same in every lane).
template <int LC>
__device__ __forceinline__ uint32_t seg_bcast(uint32_t v, int base, int j) {
  if constexpr (LC == 64)
    return (uint32_t)__builtin_amdgcn_readlane((int)v, j);
  else
    return (uint32_t)__builtin_amdgcn_ds_bpermute((base + j) << 2, (int)v);
}

// Contributions (s div t) * w * p of an edge for s = 0, 1, 2 as signed bytes
// 0, 1 and 2 of a dword (byte 0 is always 0).
__device__ __forceinline__ uint32_t pr_edge_table(int w, int p, int t) {
  const int c = w * p;
  const int c1 = t == 1 ? c : 0, c2 = t == 1 ? 2 * c : c;
  return ((uint32_t)(c1 & 0xff) << 8) | ((uint32_t)(c2 & 0xff) << 16);
}

// What one lane knows about its node's regulation (the chain's current or
// candidate parameters).
template <int LC, int DMAX>
struct PrNode {
  static constexpr int kSlots = DMAX > 0 ? DMAX : 1;
  uint32_t tab[kSlots];                           // sparse: contribution table per in-edge slot
  SegMask<LC> a1p, a2p, a1n, a2n, b1p, b2p, b1n, b2n;  // dense: regulator masks (b1p also for V)
  SegMask<LC> nz;                                 // sources of in-edges with w != 0
  bool act;                                       // an in-edge with p = +1 and w != 0
  int u, mem, d;                                  // speed, memory, step size
};

// Source lane byte addresses of the sparse slots (fixed by the topology).
template <int DMAX>
struct PrAddr {
  static constexpr int kSlots = DMAX > 0 ? DMAX : 1;
  int addr[kSlots];
};

// The slot of edge e (source j, k-th in-edge of node i) now has weight w,
// polarity p and threshold t.
template <int LC, int DMAX>
__device__ __forceinline__ void pr_set_edge(PrNode<LC, DMAX> &nd, int slot, int j, int w, int p, int t) {
  const SegMask<LC> bit = (SegMask<LC>)1 << j;
  auto put = [bit](SegMask<LC> &f, bool on) { f = (f & ~bit) | (on ? bit : (SegMask<LC>)0); };
  const int coef = w * p;
  if constexpr (DMAX > 0) {
    const uint32_t tb = pr_edge_table(w, p, t);
#pragma unroll
    for (int k = 0; k < DMAX; ++k) nd.tab[k] = k == slot ? tb : nd.tab[k];
  } else {
    const bool t1 = t == 1;
    put(nd.a1p, t1 && coef >= 1);
    put(nd.a2p, t1 && coef == 2);
    put(nd.a1n, t1 && coef <= -1);
    put(nd.a2n, t1 && coef == -2);
    put(nd.b2p, coef == 2);
    put(nd.b1n, coef <= -1);
    put(nd.b2n, coef == -2);
  }
  put(nd.b1p, coef >= 1);
  put(nd.nz, w != 0);
  nd.act = nd.b1p != 0;
}

// Node state of lane li from a parameter vector (xv(k) reads element k).
template <int LC, int DMAX, typename XV>
__device__ __forceinline__ void pr_build(const DevProblem &pb, int li, int base, XV xv, PrNode<LC, DMAX> &nd,
                                         PrAddr<DMAX> &ad) {
  nd = PrNode<LC, DMAX>{};
#pragma unroll
  for (int k = 0; k < PrAddr<DMAX>::kSlots; ++k) ad.addr[k] = (base + li) << 2;
  if (li >= pb.N) return;
  const int E = pb.E, N = pb.N;
  const int e0 = pb.in_ptr[li], e1 = pb.in_ptr[li + 1];
  for (int e = e0; e < e1; ++e) {
    const int j = pb.edge_src[e];
    pr_set_edge<LC, DMAX>(nd, e - e0, j, xv(e), xv(E + e), xv(2 * E + e));
    if constexpr (DMAX > 0) {
#pragma unroll
      for (int k = 0; k < DMAX; ++k) ad.addr[k] = k == e - e0 ? (base + j) << 2 : ad.addr[k];
    }
  }
  nd.u = xv(3 * E + li);
  nd.mem = xv(3 * E + N + li);
  nd.d = xv(3 * E + 2 * N + li);
}

// §2.5.3 for the segment: nodes without an in-edge with p = +1 and w != 0,
// plus nodes without an out-edge with w != 0 (a bit of some node's nz mask).
template <int LC, int DMAX>
__device__ __forceinline__ int pr_violations(const DevProblem &pb, int li, const PrNode<LC, DMAX> &nd) {
  const SegMask<LC> sources = seg_or<LC>(nd.nz);
  int v = 0;
  if (li < pb.N) v = (int)!nd.act + (int)(((sources >> li) & 1) == 0);
  return seg_sum<LC>(v);
}

// Median of three integers, min(max(a, lo), hi) for lo <= hi, in one
// v_med3_i32 (the compiler forms it only for constant bounds).
__device__ __forceinline__ int med3(int a, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(lo), "v"(hi));
  return r;
}

// One-hot byte code of a state: byte s of the dword is 1.
__device__ __forceinline__ int pr_onehot(int s) { return 1 << (s << 3); }

// Image K_i of this lane's node from the states of its segment (s, and its
// one-hot code oh, in every lane): in the sparse form a lane permute fetches
// each source's one-hot code and a 4-byte dot product with the edge's table
// picks the contribution and accumulates it.
template <int LC, int DMAX>
__device__ __forceinline__ int pr_image(const PrNode<LC, DMAX> &nd, const PrAddr<DMAX> &ad, int s, int oh,
                                        int base) {
  if constexpr (DMAX > 0) {
    int img = 0;
#pragma unroll
    for (int k = 0; k < DMAX; ++k)
      img = __builtin_amdgcn_sdot4((int)nd.tab[k], __builtin_amdgcn_ds_bpermute(ad.addr[k], oh), img, false);
    return img;
  } else {
    const SegMask<LC> g1 = seg_ballot<LC>(s >= 1, base), g2 = seg_ballot<LC>(s >= 2, base);
    return pr_popc<LC>(g1 & nd.a1p) + pr_popc<LC>(g1 & nd.a2p) + pr_popc<LC>(g2 & nd.b1p) +
           pr_popc<LC>(g2 & nd.b2p) - pr_popc<LC>(g1 & nd.a1n) - pr_popc<LC>(g1 & nd.a2n) -
           pr_popc<LC>(g2 & nd.b1n) - pr_popc<LC>(g2 & nd.b2n);
  }
}

// This lane's share of the weighted mismatch of §2.3 under every condition
// (the trajectory of §2.2's priority update).  start: [C][LC] state | 4 if
// held; obs: [C][T+1][LC] dwords whose byte s is W * |s - R| (0 where
// nothing is observed).  With TRAJ and a non-null traj the states of every
// step are written to traj[(c*(T+1) + t)*N + node].  Every lane of the wave
// must call it together (ballots, lane permutes, reductions).
// act records, over all conditions and steps, whether the lane's node was
// ever told to change (bit 0), ever eligible (bit 1) and ever moved towards a
// goal two levels away (bit 2) -- its memory, speed and step size can only
// matter where these happen -- and whether it ever held the state 1 (bit 8)
// or 2 (bit 16), the only states in which its out-edges contribute.
constexpr uint32_t kPrTold = 1, kPrReady = 2, kPrFar = 4, kPrVisited = 0x10100u;

// Smallest and largest image K_i the node had at a step where it was free
// (its goal clamp(K_i, 0, 2) mattered), over every condition and step of a
// trajectory; kPrNoImage when it never was.  A change of K_i by at most
// [lo, hi] (lo <= 0 <= hi) leaves every goal, and so the trajectory, as it is
// when min + lo >= 2 or max + hi <= 0 (the image stays saturated).
constexpr int kPrNoImage = 1 << 20;
struct PrImageRange {
  int lo = kPrNoImage, hi = -kPrNoImage;
};

template <int LC, int DMAX, bool TRAJ>
__device__ __forceinline__ int pr_mismatch(const DevProblem &pb, int li, int base, const PrNode<LC, DMAX> &nd,
                                           const PrAddr<DMAX> &ad, const uint8_t *start, const uint32_t *obs,
                                           int8_t *traj, uint32_t *act = nullptr, PrImageRange *range = nullptr) {
  const int T = pb.T;
  int acc = 0;
  int klo = kPrNoImage, khi = -kPrNoImage;
  bool told_any = false, ready_any = false, far_any = false;
  int vis = 0;
  for (int c = 0; c < pb.C; ++c) {
    const int st = start[c * LC + li];
    int s = st & 3;
    const int inc = (st & 4) ? 0 : 1;  // held nodes never count idle steps, so never get a priority
    int idle = 0, streak = 0;
    const uint32_t *oc = obs + (size_t)c * (T + 1) * LC + li;
    int oh = pr_onehot(s);
    vis |= oh;
    acc = __builtin_amdgcn_sdot4((int)oc[0], oh, acc, false);  // picks W|s - R|
    if (TRAJ && traj && li < pb.N) traj[(size_t)c * (T + 1) * pb.N + li] = (int8_t)s;
    for (int t = 1; t <= T; ++t) {
      const int img = pr_image<LC, DMAX>(nd, ad, s, oh, base);
      if (range && inc) {
        klo = min(klo, img);
        khi = max(khi, img);
      }
      const int goal = min(max(img, 0), 2);
      const bool told = inc && goal != s;
      idle += inc;
      streak = told ? streak + 1 : 0;
      // u <= 12 and idle <= T: a 24-bit product
      const int prio = (told && streak > nd.mem) ? (int)__umul24((unsigned)nd.u, (unsigned)idle) : 0;
      const int best = seg_max<LC>(prio);
      told_any |= told;
      ready_any |= prio > 0;
      // the node of the step's highest priority moves towards the goal by at
      // most d (d >= 1).  One chain per wave: a branch around one median
      // (|goal - s| = 2 for states in {0, 1, 2} is goal ^ s = 2); several
      // chains per wave: the plain form, which the compiler turns into
      // selects (each form measured the faster one for its segment width).
      if constexpr (LC == 64) {
        if (prio > 0 && prio == best) {
          far_any |= (goal ^ s) == 2;
          s = med3(goal, s - nd.d, s + nd.d);
          idle = 0;
          streak = 0;
        }
      } else if (prio > 0 && prio == best) {
        far_any |= abs(goal - s) == 2;
        s = min(max(goal, s - nd.d), s + nd.d);
        idle = 0;
        streak = 0;
      }
      oh = pr_onehot(s);
      vis |= oh;
      acc = __builtin_amdgcn_sdot4((int)oc[(size_t)t * LC], oh, acc, false);
      if (TRAJ && traj && li < pb.N) traj[((size_t)c * (T + 1) + t) * pb.N + li] = (int8_t)s;
    }
  }
  if (act)
    *act = (told_any ? kPrTold : 0u) | (ready_any ? kPrReady : 0u) | (far_any ? kPrFar : 0u) |
           ((uint32_t)vis & kPrVisited);
  if (range) {
    range->lo = klo;
    range->hi = khi;
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
