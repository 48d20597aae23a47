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
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWavesPerBlock = 4;
constexpr uint32_t kLowNibbles = 0x11111111u;

__host__ __device__ inline int round4(int v) { return (v + 3) & ~3; }

// (m-tiles, k-fragments of 128) of every instantiated register layout
#define SA_FOR_TILES(X) X(1, 1) X(2, 1) X(3, 1) X(4, 1) X(5, 1) X(6, 1) X(7, 1) X(8, 1) X(9, 2) X(10, 2) X(11, 2) X(12, 2)

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kWavesPerBlock - 1) / kWavesPerBlock)); }

// ---------------------------------------------------------------------------
// wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the 64 lanes, returned wave-uniform.  Data-parallel-primitive
// (DPP) adds: an inclusive scan within each row of 16 lanes (row_shr 1, 2, 4,
// 8, shifted-out lanes read 0), then row 0's total is added into row 1 and
// row 2's into row 3 (row_bcast:15), then rows 0-1 into rows 2-3
// (row_bcast:31); lane 63 ends with the total.  No LDS round trips.
__device__ __forceinline__ int wave_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false); // row_bcast:15 into rows 1 and 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false); // row_bcast:31 into rows 2 and 3
  return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Element i (wave-uniform) of a table that nothing writes while a kernel
// runs, loaded through the scalar unit: the constant address space tells the
// compiler that the memory does not change, so the load becomes s_load
// instead of a vector load and a lane read.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *table, int i) {
  typedef const __attribute__((address_space(4))) T *ConstPtr;
  return ((ConstPtr)table)[i];
}

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
// A operand dword `reg` = (mt*NK + kf)*4 + dw (16 bytes = 32 nibbles per
// lane per (m-tile, k-fragment)) lives in chunk reg/16, element reg%16, so a
// fragment is four consecutive registers of one 16-register tuple.  Nibble n
// of dword dw holds entry (row l%16 of m-tile mt, column of slot
// (l/16, 32*kf + 8*dw + n)) as an fp4 (e2m1) code.
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

// The A operand of m-tile MT, k-fragment KF, widened to the 8 dwords the
// instruction takes (fp4 operands use the first 4).
template <int MT, int KF, int NM, int NK>
__device__ __forceinline__ v8i afrag(const ATile<NM, NK> &A) {
  constexpr int r0 = (MT * NK + KF) * 4;
  const v16i &c = chunk<r0 / 16>(A);
  constexpr int o = r0 % 16;
  return __builtin_shufflevector(c, c, o, o + 1, o + 2, o + 3, o, o + 1, o + 2, o + 3);
}

__device__ __forceinline__ v8i widen(v4i b) { return __builtin_shufflevector(b, b, 0, 1, 2, 3, 0, 1, 2, 3); }

// fp4 (e2m1) code of a small integer a in [-3, 3]: magnitude 1 -> 0x2,
// 2 -> 0x4, 3 -> 0x5, sign in bit 3
__device__ __forceinline__ uint32_t fp4_code(int a) {
  const uint32_t m = (uint32_t)abs(a);
  return (m == 3u ? 0x5u : m << 1) | (a < 0 ? 8u : 0u);
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

// A entry of parameter p holding value v (edge value a, or -theta - 1 in the
// bias column: the product is 2(h - 1)), replicated into every nibble.
__device__ __forceinline__ uint32_t param_bits(int p, int E, int v) {
  return fp4_code(p < E ? v : -v - 1) * kLowNibbles;
}

// Writes parameter p's value v (edge value a, or theta) at its A position.
// param_pos[p] = lane | m-tile << 8 | k-fragment << 12 | dword << 14 |
// nibble << 16, independent of the register layout; the layout's NK turns it
// into the A register index (mt*NK + kf)*4 + dw.
template <int NK>
__device__ __forceinline__ void param_patch_args(const DevProblem &pb, int lane, int p, int v, int &reg,
                                                 uint32_t &mask, uint32_t &bits) {
  const uint32_t pos = load_uniform(pb.param_pos, p);
  const int mt = (int)((pos >> 8) & 15u), kf = (int)((pos >> 12) & 3u), dw = (int)((pos >> 14) & 3u);
  reg = (mt * NK + kf) * 4 + dw;
  mask = (lane == (int)(pos & 63u)) ? (0xfu << (4 * ((pos >> 16) & 7u))) : 0u;
  bits = param_bits(p, pb.E, v);
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
// node update and score on packed states: 8 nodes' fp4 codes per dword
// ---------------------------------------------------------------------------
// States are stored as the fp4 codes of 2s (0, 2.0, 4.0 -> codes 0x0, 0x4,
// 0x6), a thermometer code: bit 2 = [s >= 1], bit 1 = [s >= 2].  The bias
// input is a state fixed at 1, so the unscaled product is 2(h - 1).
constexpr uint32_t kBit2 = 0x44444444u;  // bit 2 of every nibble

// Rows 4g .. 4g+3 of an m-tile for this lane's condition: x = 2(h - 1).
// Scale operands 0 select the unscaled form of the instruction (both scales
// 1), which holds the VALU issue for fewer cycles than the scaled form.
__device__ __forceinline__ v4f mfma_fp4(v8i a, v8i b, v4f acc) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, acc, 4, 4, 0, 0, 0, 0);
}

// Writes the fp4 codes of 8x for an m-tile's four results x = 2(h - 1) into
// bytes 2h and 2h+1 of `word` (h = m-tile parity).  The conversion saturates
// at 6, so every code is 0x0 (x = 0), 0x7 (x >= 2) or 0xf (x <= -2): bit 3 =
// [x < 0], bits 0-2 = [x != 0].  A zero result is +0 (the accumulators start
// from +0 or from a non-zero offset, and exact cancellation rounds to +0), so
// the code 0x8 of a signed zero does not occur.  With t = clamp(h, 0, 2)
// (§2.1, §2.2): [t >= 2] = bit 2 and not bit 3, [t >= 1] = not bit 3.
__device__ __forceinline__ uint32_t put_codes(uint32_t word, const v4f &acc, int h) {
  constexpr float kSaturate = 0.125f;  // the conversion divides by it
  if (h == 0) {
    word = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(word, acc[0], acc[1], kSaturate, 0);
    word = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(word, acc[2], acc[3], kSaturate, 1);
  } else {
    word = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(word, acc[0], acc[1], kSaturate, 2);
    word = __builtin_amdgcn_cvt_scalef32_pk_fp4_f32(word, acc[2], acc[3], kSaturate, 3);
  }
  return word;
}

// Next states of 8 nodes from the codes w of x = 2(h - 1) and the states s.
// d = 1 moves one level towards t = clamp(h, 0, 2):
//     [s' >= 1] = [t >= 1] or [s >= 2],   [s' >= 2] = [t >= 2] and [s >= 1];
// d >= 2 reaches t: s' = t.  Both thresholds are formed at bit 1 of every
// nibble, where w >> 2 holds [x < 0], w itself [x != 0], s [s >= 2] and
// s >> 1 [s >= 1], each masked to that bit; one shift-or then moves
// [s' >= 1] up to bit 2 and merges the two (v_lshl_or_b32).  Five integer
// instructions per 8 nodes for d = 1, four for d >= 2.  v_bitop3_b32 truth
// tables are indexed by (a << 2) | (b << 1) | c.
constexpr uint32_t kBit1 = 0x22222222u;  // bit 1 of every nibble
template <int D>
__device__ __forceinline__ uint32_t next_states(uint32_t w, uint32_t s) {
  const uint32_t n = w >> 2;
  uint32_t ge1, ge2;
  if constexpr (D == 1) {
    ge1 = __builtin_amdgcn_bitop3_b32(n, s, kBit1, 0x8A);       // (!a | b) & c
    ge2 = __builtin_amdgcn_bitop3_b32(n, w, s >> 1, 0x08);      // !a & b & c: bit 1 only
  } else {
    ge1 = __builtin_amdgcn_bitop3_b32(n, kBit1, 0u, 0x0C);      // !a & b
    ge2 = __builtin_amdgcn_bitop3_b32(n, w, kBit1, 0x08);       // !a & b & c
  }
  return (ge1 << 1) | ge2;
}

// Weighted Manhattan distance of the packed states against the reference:
// x = s ^ r has [s >= 1] != [r >= 1] at bit 2 and [s >= 2] != [r >= 2] at
// bit 1, so |s - r| is the number of set bits; with 4-bit dot products
// against W (0 where the slot is not observed), a1 = sum W (2 b1 + 4 b2) and
// a2 = sum 4 W b2 give sum W (b1 + b2) = (2 a1 - a2) / 4.  r and w point at
// this observed time's [nd][64] tables.
template <int NK>
__device__ __forceinline__ int score(const v4i (&B)[NK], const uint32_t *__restrict__ r,
                                     const uint32_t *__restrict__ w, int nd, int lane) {
  uint32_t a1 = 0, a2 = 0;
#pragma unroll
  for (int q4 = 0; q4 < 4 * NK; ++q4) {
    if (q4 < nd) {
      const uint32_t x = (uint32_t)B[q4 >> 2][q4 & 3] ^ r[q4 * kWave + lane];
      const uint32_t ww = w[q4 * kWave + lane];
      a1 = __builtin_amdgcn_udot8(x, ww, a1, false);
      a2 = __builtin_amdgcn_udot8(x & kBit2, ww, a2, false);
    }
  }
  return (int)((2u * a1 - a2) >> 2);
}

// State values (0, 1, 2) of 8 packed codes, one per nibble.
__device__ __forceinline__ uint32_t state_values(uint32_t s) {
  return ((s >> 1) & kLowNibbles) + ((s >> 2) & kLowNibbles);
}

template <int NK>
__device__ __forceinline__ void write_states(const v4i (&B)[NK], const DevProblem &pb, int lane, int c, int t,
                                             int8_t *__restrict__ traj) {
  if (c >= pb.C) return;
  const int g = lane >> 4;
#pragma unroll
  for (int q4 = 0; q4 < 4 * NK; ++q4)
#pragma unroll
    for (int n = 0; n < 8; ++n) {
      const int v = pb.slot_node[g * 32 * NK + q4 * 8 + n];
      if (v >= 0)
        traj[((size_t)c * (pb.T + 1) + t) * pb.N + v] =
            (int8_t)((state_values((uint32_t)B[q4 >> 2][q4 & 3]) >> (4 * n)) & 0xfu);
    }
}

// One synchronous time step (§2.2): every m-tile reads only the states of
// step t-1 (B) and writes those of step t (NB).  M-tile mt's four rows are
// nibbles 4mt .. 4mt+3 of its lane group's slots, so two m-tiles fill one
// dword, which then takes the clamp select (mask CM: clamped nodes get their
// old state as target, so they hold) and the step.  Only the first NMR
// m-tiles of the NM-tile layout hold nodes (a smaller network in a larger
// layout); dwords past them carry over.
// HOLD: held nodes keep their state through a per-dword select with CM;
// without HOLD, every clamped node is in the first dword, OF holds the
// accumulator offsets of m-tiles 0 and 1 (clamped nodes forced to their
// clamp value by the product, DevProblem::cofs) and no select is needed.
template <int NMR, int NM, int NK, int D, bool HOLD = true>
__device__ __forceinline__ void time_step(const ATile<NM, NK> &A, const v4i (&B)[NK], v4i (&NB)[NK],
                                          const v4i (&CM)[NK], const v4f *OF = nullptr) {
  static_assert(NMR >= 1 && NMR <= NM, "active m-tiles within the layout");
  v8i bw[NK];
#pragma unroll
  for (int kf = 0; kf < NK; ++kf) bw[kf] = widen(B[kf]);
  constexpr int NW = (NMR + 1) / 2;  // dwords holding m-tile rows
  static_for<NW>([&](auto wc) SA_INLINE {
    constexpr int w = decltype(wc)::value;
    constexpr int kf = w / 4, dw = w % 4;
    v4f acc[2];
    static_for<2>([&](auto hc) SA_INLINE {
      constexpr int h = decltype(hc)::value;
      constexpr int mt = 2 * w + h;
      if constexpr (mt < NMR) {
        acc[h] = v4f{0.f, 0.f, 0.f, 0.f};
        if constexpr (!HOLD && mt < 2) acc[h] = OF[mt];
        static_for<NK>([&](auto kc) SA_INLINE {
          constexpr int k = decltype(kc)::value;
          acc[h] = mfma_fp4(afrag<mt, k>(A), bw[k], acc[h]);
        });
      }
    });
    // The code word is built in the register of a spent result (no copy):
    // bytes no m-tile writes hold no node (or the bias) and are held.
    uint32_t x = __builtin_bit_cast(uint32_t, acc[0][0]);
    static_for<2>([&](auto hc) SA_INLINE {
      constexpr int h = decltype(hc)::value;
      if constexpr (2 * w + h < NMR) x = put_codes(x, acc[h], h);
    });
    const uint32_t s = (uint32_t)B[kf][dw];
    if constexpr (HOLD) {
      const uint32_t cm = (uint32_t)CM[kf][dw];
      // cm ? s : next bitwise, one v_bitop3_b32 (truth table indexed by
      // (next << 2) | (s << 1) | cm: set for 3, 4, 6, 7)
      NB[kf][dw] = (int)__builtin_amdgcn_bitop3_b32(next_states<D>(x, s), s, cm, 0xD8);
    } else if constexpr (2 * w + 1 >= NMR) {
      // the dword's second m-tile is beyond the rows: its nibbles (the bias
      // slot when the node count is a multiple of 16, else empty slots) hold
      NB[kf][dw] = (int)__builtin_amdgcn_bitop3_b32(next_states<D>(x, s), s, 0xFFFF0000u, 0xD8);
    } else {
      NB[kf][dw] = (int)next_states<D>(x, s);
    }
  });
  // dwords without m-tile rows (slots beyond the rows) carry over unchanged
  static_for<4 * NK>([&](auto qc) SA_INLINE {
    constexpr int q = decltype(qc)::value;
    if constexpr (q >= NW) NB[q >> 2][q & 3] = B[q >> 2][q & 3];
  });
  // keep the whole step in one block and let the m-tiles' integer work run
  // under the next m-tile's matrix products
#pragma unroll
  for (int kf = 0; kf < NK; ++kf) asm volatile("" : "+v"(NB[kf]));
  // integer instructions per dword: 4 conversions, the update, the select
  constexpr int kValu = (D == 1 ? 10 : 9) - (HOLD ? 0 : 1);
  __builtin_amdgcn_sched_group_barrier(0x008, 2 * NK, 0);
  static_for<NW - 1>([&](auto) SA_INLINE {
    __builtin_amdgcn_sched_group_barrier(0x008, 2 * NK, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, kValu, 0);
  });
  __builtin_amdgcn_sched_group_barrier(0x002, kValu + 2, 0);
}

// Simulates every condition for the chain whose parameters are in A, with
// NMR m-tiles holding nodes, and returns this lane's share of the mismatch M
// (§2.3).  obs_r/obs_w: [CG][K][nd][64] tables.  The two state buffers
// alternate between steps.  Without a trajectory to record, the simulation
// ends at the last observed time (later states do not enter M).
template <int NMR, int NM, int NK, int D, bool TRAJ, bool HOLD>
__device__ __forceinline__ int lane_mismatch_n(const ATile<NM, NK> &A, const DevProblem &pb, int lane,
                                               const uint32_t *obs_r, const uint32_t *obs_w,
                                               int8_t *__restrict__ traj) {
  int total = 0;
  for (int cg = 0; cg < pb.CG; ++cg) {
    v4i B0[NK], B1[NK], CM[NK];
    v4f OF[2];
    const int base = cg * 4 * NK;
#pragma unroll
    for (int kt = 0; kt < NK; ++kt)
#pragma unroll
      for (int dw = 0; dw < 4; ++dw) {
        const int at = (base + kt * 4 + dw) * kWave + lane;
        B0[kt][dw] = (int)pb.b0[at];
        if constexpr (HOLD) CM[kt][dw] = (int)pb.cmask[at];
      }
    if constexpr (!HOLD) {
      const v4f *of = reinterpret_cast<const v4f *>(pb.cofs) + (size_t)cg * 2 * kWave + lane;
#pragma unroll
      for (int mt = 0; mt < 2 && mt < NMR; ++mt) OF[mt] = of[(size_t)mt * kWave];
    }
    const int c = cg * 16 + (lane & 15);
    const uint32_t *rbase = obs_r + (size_t)cg * pb.K * pb.nd * kWave;
    const uint32_t *wbase = obs_w + (size_t)cg * pb.K * pb.nd * kWave;
    int k = 0;
    int tnext = load_uniform(pb.obs_t, 0);
    auto observe = [&](const v4i (&B)[NK], int t) SA_INLINE {
      if (TRAJ) write_states<NK>(B, pb, lane, c, t, traj);
      if (t == tnext) {
        total += score<NK>(B, rbase + (size_t)k * pb.nd * kWave, wbase + (size_t)k * pb.nd * kWave, pb.nd, lane);
        ++k;
        tnext = k < pb.K ? load_uniform(pb.obs_t, k) : -1;
      }
    };
    observe(B0, 0);
    const int t_end = TRAJ ? pb.T : load_uniform(pb.obs_t, pb.K - 1);
    int t = 1;
    for (; t + 1 <= t_end; t += 2) {
      time_step<NMR, NM, NK, D, HOLD>(A, B0, B1, CM, OF);
      observe(B1, t);
      time_step<NMR, NM, NK, D, HOLD>(A, B1, B0, CM, OF);
      observe(B0, t + 1);
    }
    if (t <= t_end) {
      time_step<NMR, NM, NK, D, HOLD>(A, B0, B1, CM, OF);
      observe(B1, t);
    }
  }
  return total;
}

// Smallest m-tile count a layout of NM m-tiles serves at run time (the size
// classes of the many-network kernel: 1-4, 5-8 and 9-10 m-tiles).
constexpr int rt_min_tiles(int nm) { return nm <= 4 ? 1 : nm <= 8 ? 5 : 9; }

// RT: the network may have fewer m-tiles than the layout (pb.nm, from
// rt_min_tiles(NM) to NM; its k-fragments always equal NK): the simulation
// runs the variant compiled for that count and for the network's way of
// holding clamped nodes (pb.hold_by_offset; HOLD is then unused), so the
// time step holds no run-time bound.
template <int NM, int NK, int D, bool TRAJ, bool RT = false, bool HOLD = true>
__device__ __forceinline__ int lane_mismatch(const ATile<NM, NK> &A, const DevProblem &pb, int lane,
                                             const uint32_t *obs_r, const uint32_t *obs_w,
                                             int8_t *__restrict__ traj) {
  if constexpr (!RT) {
    return lane_mismatch_n<NM, NM, NK, D, TRAJ, HOLD>(A, pb, lane, obs_r, obs_w, traj);
  } else {
    int total = 0;
    const int nm = pb.nm;
    const bool by_offset = pb.hold_by_offset != 0;
    static_for<NM - rt_min_tiles(NM) + 1>([&](auto ic) SA_INLINE {
      constexpr int NMR = rt_min_tiles(NM) + decltype(ic)::value;
      if (nm == NMR) {
        if (by_offset)
          total = lane_mismatch_n<NMR, NM, NK, D, TRAJ, false>(A, pb, lane, obs_r, obs_w, traj);
        else
          total = lane_mismatch_n<NMR, NM, NK, D, TRAJ, true>(A, pb, lane, obs_r, obs_w, traj);
      }
    });
    return total;
  }
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
