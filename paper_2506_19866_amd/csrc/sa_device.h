// sa_device.h -- device building blocks shared by the kernels: Philox,
// register patching, the MFMA simulation of all conditions, the score and the
// constraint counts.  Method: Reimer et al., arXiv 2506.19866 (model §2.1
// with the synchronous update of §2.2, objective §2.3, constraints §2.5.3).
// The register layout is described in sa_internal.h.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "sa_internal.h"

namespace sa {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWavesPerBlock = 4;
constexpr uint32_t kLowBits = 0x01010101u;

__host__ __device__ inline int round4(int v) { return (v + 3) & ~3; }

// (m-tiles, k-tiles) of every instantiated register layout: nk = ceil(nm/4)
#define SA_FOR_TILES(X) X(1, 1) X(2, 1) X(3, 1) X(4, 1) X(5, 2) X(6, 2) X(7, 2) X(8, 2) X(9, 3) X(10, 3) X(11, 3) X(12, 3)

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock)); }

// ---------------------------------------------------------------------------
// wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of two 64x64->128
// multiplications by the Philox constants, the high halves mixed with the
// other two words and the round key, the key advanced by the Weyl constants.
// Returns the top 32 bits of the four words (the only bits a step uses; the
// plain proposal uses words 0-2, and the compiler drops word 3 there).
// ---------------------------------------------------------------------------
struct Draw {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Draw philox_top_words(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                 uint64_t k0, uint64_t k1) {
  constexpr uint64_t kMul0 = 0xD2E7470EE14C6C93ull, kMul1 = 0xCA5A826395121157ull;
  constexpr uint64_t kWeyl0 = 0x9E3779B97F4A7C15ull, kWeyl1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kWeyl0;
      k1 += kWeyl1;
    }
    const uint64_t lo0 = kMul0 * c0, hi0 = __umul64hi(kMul0, c0);
    const uint64_t lo1 = kMul1 * c2, hi1 = __umul64hi(kMul1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return {(uint32_t)(c0 >> 32), (uint32_t)(c1 >> 32), (uint32_t)(c2 >> 32), (uint32_t)(c3 >> 32)};
}

// ---------------------------------------------------------------------------
// compile-time loops: every register index below is a constant from the
// start, so each 16-register chunk stays an SSA value (never a stack array)
// ---------------------------------------------------------------------------
#define SA_INLINE __attribute__((always_inline))

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// The chain's parameter matrix in registers
// ---------------------------------------------------------------------------
// A operand dword `reg` = (mt*NK + kt)*4 + dw (16 bytes per lane per
// (m-tile, k-tile)) lives in chunk reg/16, element reg%16, so a fragment is
// four consecutive registers of one 16-register tuple.  Byte b of dword dw
// holds entry (row l%16 of m-tile mt, column of slot (l/16, 16*kt + 4*dw + b)).
// Each 16-register chunk is its own local variable in the kernel (declared by
// SA_DECLARE_A): an access with a dynamic element index then stays inside one
// small object that the compiler keeps in a register tuple.
struct AChunkRefs {
  v16i &c0, &c1, &c2, &c3, &c4, &c5, &c6, &c7, &c8;
};

template <int C>
__device__ __forceinline__ v16i &chunk_ref(const AChunkRefs &r) {
  static_assert(C >= 0 && C < 9, "at most 9 chunks (144 A registers)");
  if constexpr (C == 0) return r.c0;
  else if constexpr (C == 1) return r.c1;
  else if constexpr (C == 2) return r.c2;
  else if constexpr (C == 3) return r.c3;
  else if constexpr (C == 4) return r.c4;
  else if constexpr (C == 5) return r.c5;
  else if constexpr (C == 6) return r.c6;
  else if constexpr (C == 7) return r.c7;
  else return r.c8;
}

template <int NM, int NK>
struct ATile {
  static constexpr int NR = NM * NK * 4;
  static constexpr int NC = (NR + 15) / 16;
  AChunkRefs a;
};

template <int C, int NM, int NK>
__device__ __forceinline__ v16i &chunk(const ATile<NM, NK> &A) {
  return chunk_ref<C>(A.a);
}

#define SA_DECLARE_A(NAME, NM, NK)                                                              \
  v16i NAME##_c0 = {}, NAME##_c1 = {}, NAME##_c2 = {}, NAME##_c3 = {}, NAME##_c4 = {},          \
       NAME##_c5 = {}, NAME##_c6 = {}, NAME##_c7 = {}, NAME##_c8 = {};                          \
  ATile<NM, NK> NAME{{NAME##_c0, NAME##_c1, NAME##_c2, NAME##_c3, NAME##_c4, NAME##_c5, NAME##_c6, \
                      NAME##_c7, NAME##_c8}}

template <int MT, int KT, int NM, int NK>
__device__ __forceinline__ v4i afrag(const ATile<NM, NK> &A) {
  constexpr int r0 = (MT * NK + KT) * 4;
  const v16i &c = chunk<r0 / 16>(A);
  constexpr int o = r0 % 16;
  return __builtin_shufflevector(c, c, o, o + 1, o + 2, o + 3);
}

// Replaces the bytes selected by `mask` (non-zero in one lane only) of A
// register `reg` (wave-uniform) by `bits`.  Branch-free: every chunk does an
// indexed read-modify-write of element reg%16 (s_set_gpr_idx addressing) with
// a mask that is zero unless the chunk is reg/16.
// The element update works on a value, never through a pointer, so that the
// chunk stays in registers.
__device__ __forceinline__ v16i vpatch(v16i v, int off, uint32_t m, uint32_t bits) {
  const uint32_t old = (uint32_t)v[off];
  v[off] = (int)((old & ~m) | (bits & m));
  return v;
}

template <int NM, int NK>
__device__ __forceinline__ void patch_a(ATile<NM, NK> &A, int reg, uint32_t mask, uint32_t bits) {
  const int ch = reg >> 4, off = reg & 15;
  static_for<ATile<NM, NK>::NC>([&](auto cc) SA_INLINE {
    constexpr int C = decltype(cc)::value;
    v16i &v = chunk<C>(A);
    v = vpatch(v, off, (ch == C) ? mask : 0u, bits);
  });
}

// Writes parameter p's value v (edge value a, or theta) at its A position.
// param_pos[p] = lane | m-tile << 8 | k-tile << 12 | dword << 14 | byte << 16,
// independent of the register layout; the layout's NK turns it into the
// A register index (mt*NK + kt)*4 + dw.
template <int NK>
__device__ __forceinline__ void param_patch_args(const DevProblem &pb, int lane, int p, int v, int &reg,
                                                 uint32_t &mask, uint32_t &bits) {
  const uint32_t pos = pb.param_pos[p];
  const int a = p < pb.E ? v : -v;  // -theta in the bias column
  const int mt = (int)((pos >> 8) & 15u), kt = (int)((pos >> 12) & 3u), dw = (int)((pos >> 14) & 3u);
  reg = (mt * NK + kt) * 4 + dw;
  mask = (lane == (int)(pos & 63u)) ? (0xffu << (8 * ((pos >> 16) & 3u))) : 0u;
  bits = ((uint32_t)a & 0xffu) * kLowBits;
}

// A from a parameter vector: zero, then one patch per parameter.
template <int NM, int NK, typename XV>
__device__ __forceinline__ void build_a(ATile<NM, NK> &A, const DevProblem &pb, int lane, XV xv) {
  static_for<ATile<NM, NK>::NC>([&](auto cc) SA_INLINE {
    chunk<decltype(cc)::value>(A) = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  });
#pragma unroll 1
  for (int p = 0; p < pb.P; ++p) {
    const int v = uniform(xv(p));
    int reg;
    uint32_t mask, bits;
    param_patch_args<NK>(pb, lane, p, v, reg, mask, bits);
    patch_a(A, uniform(reg), mask, bits);
  }
}

// ---------------------------------------------------------------------------
// node update and score on packed states (4 conditions' bytes per dword)
// ---------------------------------------------------------------------------
// Packs clamp(t, 0, 2) of the four results of an m-tile into bytes: the
// image bounded by the state range (§2.1, §2.2).  v_perm_b32 takes bytes 0-3
// from its second operand and 4-7 from its first; 0x0c yields a zero byte.
__device__ __forceinline__ uint32_t pack_targets(v4i acc) {
  const uint32_t k0 = (uint32_t)min(max(acc[0], 0), 2);
  const uint32_t k1 = (uint32_t)min(max(acc[1], 0), 2);
  const uint32_t k2 = (uint32_t)min(max(acc[2], 0), 2);
  const uint32_t k3 = (uint32_t)min(max(acc[3], 0), 2);
  const uint32_t lo = __builtin_amdgcn_perm(k1, k0, 0x0c0c0400u);  // [k0, k1, 0, 0]
  const uint32_t hi = __builtin_amdgcn_perm(k3, k2, 0x04000c0cu);  // [0, 0, k2, k3]
  return lo | hi;
}

// d = 1: every byte moves one level towards its target, s' = s + sgn(k - s).
// Over s, k in {0,1,2} the index s + 2k in [0, 6] determines s' uniquely:
// index 0 1 2 3 4 5 6 -> 0 0 1 1 1 2 2 (pairs sharing an index agree, e.g.
// (s,k) = (2,0) and (0,1) both give 1), so the update is one byte lookup
// per condition, four per v_perm_b32.  k = s yields s (index 3s), which is
// how clamped bytes are held.
__device__ __forceinline__ uint32_t step_one_level(uint32_t k, uint32_t s) {
  const uint32_t idx = (k << 1) + s;  // bytes <= 6: no carries between bytes
  return __builtin_amdgcn_perm(0x00020201u, 0x01010000u, idx);
}

// Weighted Manhattan distance of the packed states against the reference:
// per byte |s - r| = x - 2*(x & x>>1) with x = s ^ r (s, r in {0,1,2}),
// weighted by W (0 where the slot is not observed) with byte dot products.
// r and w point at this observed time's [nd][64] tables.
template <int NK>
__device__ __forceinline__ int score(const v4i (&B)[NK], const uint32_t *__restrict__ r,
                                     const uint32_t *__restrict__ w, int nd, int lane) {
  uint32_t a1 = 0, a2 = 0;
#pragma unroll
  for (int q4 = 0; q4 < 4 * NK; ++q4) {
    if (q4 < nd) {
      const uint32_t s = (uint32_t)B[q4 >> 2][q4 & 3];
      const uint32_t x = s ^ r[q4 * kWave + lane];
      const uint32_t y = (x >> 1) & x;
      const uint32_t ww = w[q4 * kWave + lane];
      a1 = __builtin_amdgcn_udot4(x, ww, a1, false);
      a2 = __builtin_amdgcn_udot4(y, ww, a2, false);
    }
  }
  return (int)(a1 - 2u * a2);
}

template <int NK>
__device__ __forceinline__ void write_states(const v4i (&B)[NK], const DevProblem &pb, int lane, int c, int t,
                                             int8_t *__restrict__ traj) {
  if (c >= pb.C) return;
  const int g = lane >> 4;
#pragma unroll
  for (int q4 = 0; q4 < 4 * NK; ++q4)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int v = pb.slot_node[g * 16 * NK + q4 * 4 + b];
      if (v >= 0)
        traj[((size_t)c * (pb.T + 1) + t) * pb.N + v] = (int8_t)(((uint32_t)B[q4 >> 2][q4 & 3] >> (8 * b)) & 0xffu);
    }
}

// One synchronous time step (§2.2): every m-tile reads only the states of
// step t-1 (B) and writes those of step t (NB).  Clamped bytes (mask CM) get
// their old state as target, so they hold.  With RT only the first nm
// m-tiles and nk k-tiles are present (a smaller network in a larger layout).
template <int NM, int NK, int D, bool RT>
__device__ __forceinline__ void time_step(const ATile<NM, NK> &A, const v4i (&B)[NK], v4i (&NB)[NK],
                                          const v4i (&CM)[NK], int nm, int nk) {
  static_for<NM>([&](auto mtc) SA_INLINE {
    constexpr int mt = decltype(mtc)::value;
    if (RT && mt >= nm) {
      NB[mt >> 2][mt & 3] = B[mt >> 2][mt & 3];
      return;
    }
    v4i acc = {0, 0, 0, 0};
    static_for<NK>([&](auto ktc) SA_INLINE {
      constexpr int kt = decltype(ktc)::value;
      if (!RT || kt < nk) acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(afrag<mt, kt>(A), B[kt], acc, 0, 0, 0);
    });
    const uint32_t s = (uint32_t)B[mt >> 2][mt & 3];
    const uint32_t cm = (uint32_t)CM[mt >> 2][mt & 3];
    const uint32_t k = pack_targets(acc);
    // cm ? s : k bitwise, one v_bitop3_b32 (truth table indexed by
    // (k << 2) | (s << 1) | cm: set for 3, 4, 6, 7)
    const uint32_t target = __builtin_amdgcn_bitop3_b32(k, s, cm, 0xD8);
    NB[mt >> 2][mt & 3] = (int)(D == 1 ? step_one_level(target, s) : target);
  });
  // dwords without an m-tile (slots beyond the rows) carry over unchanged
  static_for<4 * NK>([&](auto qc) SA_INLINE {
    constexpr int q = decltype(qc)::value;
    if constexpr (q >= NM) NB[q >> 2][q & 3] = B[q >> 2][q & 3];
  });
  if constexpr (!RT) {
    // keep the whole step in one block and let the m-tiles' integer work run
    // under the next m-tile's matrix products
#pragma unroll
    for (int kt = 0; kt < NK; ++kt) asm volatile("" : "+v"(NB[kt]));
    __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
    static_for<NM - 1>([&](auto) SA_INLINE {
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);
    });
    __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
  }
}

// Simulates every condition for the chain whose parameters are in A and
// returns this lane's share of the mismatch M (§2.3).  obs_r/obs_w:
// [CG][K][nd][64] tables.  The two state buffers alternate between steps.
template <int NM, int NK, int D, bool TRAJ, bool RT = false>
__device__ __forceinline__ int lane_mismatch(const ATile<NM, NK> &A, const DevProblem &pb, int lane,
                                             const uint32_t *obs_r, const uint32_t *obs_w,
                                             int8_t *__restrict__ traj) {
  const int nm = RT ? pb.nm : NM, nk = RT ? pb.nk : NK;
  int total = 0;
  for (int cg = 0; cg < pb.CG; ++cg) {
    v4i B0[NK], B1[NK], CM[NK];
    const int base = cg * 4 * nk;
#pragma unroll
    for (int kt = 0; kt < NK; ++kt)
#pragma unroll
      for (int dw = 0; dw < 4; ++dw) {
        const bool present = !RT || kt < nk;
        const int at = (base + kt * 4 + dw) * kWave + lane;
        B0[kt][dw] = present ? (int)pb.b0[at] : 0;
        CM[kt][dw] = present ? (int)pb.cmask[at] : -1;
      }
    const int c = cg * 16 + (lane & 15);
    const uint32_t *rbase = obs_r + (size_t)cg * pb.K * pb.nd * kWave;
    const uint32_t *wbase = obs_w + (size_t)cg * pb.K * pb.nd * kWave;
    int k = 0;
    int tnext = pb.obs_t[0];
    auto observe = [&](const v4i (&B)[NK], int t) SA_INLINE {
      if (TRAJ) write_states<NK>(B, pb, lane, c, t, traj);
      if (t == tnext) {
        total += score<NK>(B, rbase + (size_t)k * pb.nd * kWave, wbase + (size_t)k * pb.nd * kWave, pb.nd, lane);
        ++k;
        tnext = k < pb.K ? pb.obs_t[k] : -1;
      }
    };
    observe(B0, 0);
    int t = 1;
    for (; t + 1 <= pb.T; t += 2) {
      time_step<NM, NK, D, RT>(A, B0, B1, CM, nm, nk);
      observe(B1, t);
      time_step<NM, NK, D, RT>(A, B1, B0, CM, nm, nk);
      observe(B0, t + 1);
    }
    if (t <= pb.T) {
      time_step<NM, NK, D, RT>(A, B0, B1, CM, nm, nk);
      observe(B1, t);
    }
  }
  return total;
}

// §2.5.3: this lane's share of V = #(no non-zero out-edge) + #(no +1 in-edge).
// Optionally records the per-node counts (non-zero out-edges, +1 in-edges).
template <typename XV>
__device__ __forceinline__ int lane_violations(const DevProblem &pb, int lane, XV xv, uint8_t *outnz,
                                               uint8_t *inplus) {
  int v = 0;
  for (int i = lane; i < pb.N; i += kWave) {
    int ip = 0, on = 0;
    for (int e = pb.in_ptr[i]; e < pb.in_ptr[i + 1]; ++e) ip += xv(e) == 1;
    for (int j = pb.out_ptr[i]; j < pb.out_ptr[i + 1]; ++j) on += xv(pb.out_eid[j]) != 0;
    if (outnz) {
      outnz[i] = (uint8_t)on;
      inplus[i] = (uint8_t)ip;
    }
    v += (ip == 0) + (on == 0);
  }
  return v;
}

}  // namespace sa
