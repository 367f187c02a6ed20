// Device code of one int8-MFMA leaf tile, shared by the per-launch leaf kernel
// and the persistent batched kernel.  See leaf_mfma.hip for the method.
#pragma once

#include "bmm_internal.h"

namespace bmm {
namespace mfma {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Operand formats of the matrix cores.  I8: v_mfma_i32_32x32x32_i8, int32
// counts.  F4: v_mfma_scale_f32_32x32x64_f8f6f4 on E2M1 operands with unit
// scales; a set bit becomes the nibble 0x1 (the value 0.5), so every product
// is 0.25 and the fp32 accumulator holds count / 4 exactly while k < 2^24.
enum MfmaFormat { FMT_I8 = 0, FMT_F4 = 1 };

// Semiring template value meaning "given at run time": the main loop does not
// depend on the semiring (both feed exact 0/1 operands), only the epilogue's
// reduction does, so one kernel can serve both with a single copy of the loop.
constexpr int SEMI_ANY = -1;

// Operands and results live in device (global) memory.  Pointers typed so keep
// the loads and stores global even where the compiler cannot infer it (pointers
// read from a problem table in memory would otherwise become generic accesses).
#define BMM_GLOBAL __attribute__((address_space(1)))
typedef const BMM_GLOBAL uint64_t* gq_ptr;
typedef BMM_GLOBAL uint32_t* gd_ptr;
typedef BMM_GLOBAL uint64_t* gw_ptr;
typedef uint64_t cpair_t __attribute__((ext_vector_type(2)));
typedef BMM_GLOBAL cpair_t* gw2_ptr;

template <int FMT>
struct Acc;
template <>
struct Acc<FMT_I8> {
  using type = v16i;
};
template <>
struct Acc<FMT_F4> {
  using type = v16f;
};

// Eight E2M1 operand nibbles per dword: nibble j of dword d is bit 4j + d of x.
__device__ __forceinline__ v8i expand_f4(uint32_t x) {
  v8i o;
#pragma unroll
  for (int d = 0; d < 4; ++d) o[d] = (int)((x >> d) & 0x11111111u);
#pragma unroll
  for (int d = 4; d < 8; ++d) o[d] = 0;
  return o;
}

// Four int8 operand dwords from bits first .. first+3 of every byte of x: each
// byte becomes exactly 0 or 1.  (For GF(2) the parity of the count would only
// need the low bit of each byte, but bytes that keep the other random bits make
// the matrix cores switch far more and run slower on dense inputs.)
template <int SEMI>
__device__ __forceinline__ v4i expand4(uint32_t x, int first) {
  v4i o;
#pragma unroll
  for (int d = 0; d < 4; ++d) o[d] = (int)((x >> (first + d)) & 0x01010101u);
  return o;
}

// WIDE: expand the rows of one side of the tile with 64-bit shifts (below): the longer
// side, or with SHORT the shorter one, which holds fewer expanded rows in registers.  The
// LDS-staged 256 x 256 leaf widens its longer side (2-3% faster for E2M1 operands); the
// batched items widen their shorter side (3% faster for int8, 2% for E2M1; the longer
// side spills them); the register-fed fp4 tiles keep the 32-bit form, which either wide
// form would spill.  BOTH (int8): both sides wide, for the recursion's unrolled 128 x 64
// tile with two load buffers instead of three.
template <int SEMI, int RA, int RB, int FMT, bool WIDE = true, bool SHORT = false, bool BOTH = false>
__device__ __forceinline__ void mfma_word(const uint64_t (&xa)[RA], const uint64_t (&xb)[RB],
                                          typename Acc<FMT>::type (&acc)[RA][RB]) {
  if constexpr (FMT == FMT_F4 && WIDE) {
    // one MFMA per 32-bit half: 32 k values per lane, 64 per instruction; the rows of
    // the longer side expand both halves at once (a 64-bit shift and two masks give
    // dword d of each half, where the 32-bit form takes two shifts and two masks)
    constexpr bool BW = SHORT ? RB < RA : RB >= RA;
    constexpr int NW = BW ? RB : RA, NN = BW ? RA : RB;
    v8i ow[2][NW];
#pragma unroll
    for (int g = 0; g < NW; ++g) {
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const uint64_t y = ((BW ? xb[g] : xa[g]) >> d) & 0x1111111111111111ull;
        ow[0][g][d] = (int)(uint32_t)y;
        ow[1][g][d] = (int)(uint32_t)(y >> 32);
      }
#pragma unroll
      for (int d = 4; d < 8; ++d) ow[0][g][d] = ow[1][g][d] = 0;
    }
#pragma unroll
    for (int hw = 0; hw < 2; ++hw) {
      v8i on[NN];
#pragma unroll
      for (int f = 0; f < NN; ++f) on[f] = expand_f4((uint32_t)((BW ? xa[f] : xb[f]) >> (32 * hw)));
#pragma unroll
      for (int f = 0; f < RA; ++f)
#pragma unroll
        for (int g = 0; g < RB; ++g)
          acc[f][g] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              BW ? on[f] : ow[hw][f], BW ? ow[hw][g] : on[g], acc[f][g], 4, 4, 0, 127, 0, 127);
    }
    return;
  } else if constexpr (FMT == FMT_F4) {
    // one MFMA per 32-bit half: 32 k values per lane, 64 per instruction
#pragma unroll
    for (int hw = 0; hw < 2; ++hw) {
      v8i oa[RA], ob[RB];
#pragma unroll
      for (int f = 0; f < RA; ++f) oa[f] = expand_f4((uint32_t)(xa[f] >> (32 * hw)));
#pragma unroll
      for (int g = 0; g < RB; ++g) ob[g] = expand_f4((uint32_t)(xb[g] >> (32 * hw)));
#pragma unroll
      for (int f = 0; f < RA; ++f)
#pragma unroll
        for (int g = 0; g < RB; ++g)
          acc[f][g] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
              oa[f], ob[g], acc[f][g], 4, 4, 0, 127, 0, 127);
    }
    return;
  } else if constexpr (!WIDE) {
#pragma unroll
    for (int hw = 0; hw < 2; ++hw) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        v4i oa[RA], ob[RB];
#pragma unroll
        for (int f = 0; f < RA; ++f) oa[f] = expand4<SEMI>((uint32_t)(xa[f] >> (32 * hw)), 4 * s);
#pragma unroll
        for (int g = 0; g < RB; ++g) ob[g] = expand4<SEMI>((uint32_t)(xb[g] >> (32 * hw)), 4 * s);
#pragma unroll
        for (int f = 0; f < RA; ++f)
#pragma unroll
          for (int g = 0; g < RB; ++g)
            acc[f][g] = __builtin_amdgcn_mfma_i32_32x32x32_i8(oa[f], ob[g], acc[f][g], 0, 0, 0);
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if constexpr (BOTH) {
        // every row expands both halves at once (16 more registers than one side)
        v4i owa[2][RA], owb[2][RB];
#pragma unroll
        for (int f = 0; f < RA; ++f)
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            const uint64_t y = (xa[f] >> (4 * s + d)) & 0x0101010101010101ull;
            owa[0][f][d] = (int)(uint32_t)y;
            owa[1][f][d] = (int)(uint32_t)(y >> 32);
          }
#pragma unroll
        for (int g = 0; g < RB; ++g)
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            const uint64_t y = (xb[g] >> (4 * s + d)) & 0x0101010101010101ull;
            owb[0][g][d] = (int)(uint32_t)y;
            owb[1][g][d] = (int)(uint32_t)(y >> 32);
          }
#pragma unroll
        for (int hw = 0; hw < 2; ++hw)
#pragma unroll
          for (int f = 0; f < RA; ++f)
#pragma unroll
            for (int g = 0; g < RB; ++g)
              acc[f][g] = __builtin_amdgcn_mfma_i32_32x32x32_i8(owa[hw][f], owb[hw][g], acc[f][g],
                                                                0, 0, 0);
        continue;
      }
      // The rows of one side (the longer, or with SHORT the shorter) expand both 32-bit
      // halves of a word at once: one 64-bit shift and two masks give dword d of each
      // half, where the 32-bit form takes two shifts and two masks.  Holding both halves
      // for every row would need more registers than two waves per SIMD leave, so the
      // other side stays 32-bit.
      constexpr bool BW = SHORT ? RB < RA : RB >= RA;
      v4i ow[2][BW ? RB : RA];
#pragma unroll
      for (int g = 0; g < (BW ? RB : RA); ++g)
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const uint64_t y = ((BW ? xb[g] : xa[g]) >> (4 * s + d)) & 0x0101010101010101ull;
          ow[0][g][d] = (int)(uint32_t)y;
          ow[1][g][d] = (int)(uint32_t)(y >> 32);
        }
#pragma unroll
      for (int hw = 0; hw < 2; ++hw) {
        v4i on[BW ? RA : RB];
#pragma unroll
        for (int f = 0; f < (BW ? RA : RB); ++f)
          on[f] = expand4<SEMI>((uint32_t)((BW ? xa[f] : xb[f]) >> (32 * hw)), 4 * s);
#pragma unroll
        for (int f = 0; f < RA; ++f)
#pragma unroll
          for (int g = 0; g < RB; ++g)
            acc[f][g] = __builtin_amdgcn_mfma_i32_32x32x32_i8(BW ? on[f] : ow[hw][f],
                                                              BW ? ow[hw][g] : on[g], acc[f][g], 0, 0, 0);
      }
    }
  }
}

// Epilogue of a TM x TN wave tile (TM = 32*RA, TN = 32*RB) at tile coordinates
// (tm, tn): reduce counts to bits and pack 32 columns per dword with ballots.  A tile
// of TN = 128 owns two whole 64-bit words of every row: it stores them as one 16-byte
// piece where C's rows are 16-byte aligned (else as two words), so each C line is
// written in fewer, larger pieces.  Narrower tiles store each dword as it is formed
// (measured faster on the recursion's short 128 x 64 tiles than gathering the words).
template <int SEMI, int RA, int RB, int FMT>
__device__ __forceinline__ void epilogue(const typename Acc<FMT>::type (&acc)[RA][RB],
                                         uint64_t* __restrict__ Cm, int64_t ldc, int64_t m,
                                         int64_t n, int64_t tm, int64_t tn, int accumulate,
                                         int semiring = SEMI) {
  constexpr int TM = 32 * RA, TN = 32 * RB;
  const bool gf2 = SEMI == SEMI_ANY ? semiring == GF2 : SEMI == GF2;
  const int64_t n_words32 = ((n + 63) >> 6) * 2;  // dwords per C row incl. padding
  if constexpr (RB != 4) {
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int li = lane & 31;
    const gd_ptr C32 = (gd_ptr)Cm;
    const int64_t ldc32 = 2 * ldc;
    const int myv = ((li >> 3) << 2) | (li & 3);
    const int myhi = (li >> 2) & 1;
#pragma unroll
    for (int g = 0; g < RB; ++g) {
      const int64_t c0 = tn * TN + 32 * g;
      const int64_t cw = c0 >> 5;
      if (cw >= n_words32) continue;  // uniform
      const int64_t valid = n - c0;
      const uint32_t cmask = valid >= 32 ? 0xFFFFFFFFu : (valid > 0 ? ((1u << valid) - 1u) : 0u);
#pragma unroll
      for (int f = 0; f < RA; ++f) {
        uint32_t mine = 0;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          int cnt;
          if constexpr (FMT == FMT_F4)
            cnt = __float2int_rn(acc[f][g][v] * 4.0f);  // exact: a multiple of 0.25
          else
            cnt = acc[f][g][v];
          const bool bit = gf2 ? ((cnt & 1) != 0) : (cnt != 0);
          const uint64_t bal = __ballot(bit);
          const uint32_t word = myhi ? (uint32_t)(bal >> 32) : (uint32_t)bal;
          mine = (myv == v) ? word : mine;
        }
        mine &= cmask;
        const int64_t row = tm * TM + 32 * f + li;
        if (half == 0 && row < m) {
          const gd_ptr dst = C32 + row * ldc32 + cw;
          if (accumulate) mine = gf2 ? (mine ^ *dst) : (mine | *dst);
          *dst = mine;
        }
      }
    }
  } else {
    // the lane index is taken afresh here (not from the work-item id the main loop
    // used), so nothing derived from it has to stay live across the loop
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    const int half = lane >> 5;
    const int li = lane & 31;
    const int myv = ((li >> 3) << 2) | (li & 3);
    const int hshift = ((li >> 2) & 1) * 32;  // lanes 4..7 of every 8 take the upper half
    // the 32-column dword of block (f, g) for this lane's row (lane li of half 0 keeps
    // row 32 f + li)
    auto pack = [&](int f, int g) -> uint32_t {
      const int64_t valid = n - (tn * TN + 32 * g);
      const uint32_t cmask = valid >= 32 ? 0xFFFFFFFFu : (valid > 0 ? ((1u << valid) - 1u) : 0u);
      uint32_t mine = 0;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int cnt;
        if constexpr (FMT == FMT_F4)
          cnt = __float2int_rn(acc[f][g][v] * 4.0f);  // exact: a multiple of 0.25
        else
          cnt = acc[f][g][v];
        const bool bit = gf2 ? ((cnt & 1) != 0) : (cnt != 0);
        const uint64_t bal = __ballot(bit);
        const uint32_t word = (uint32_t)(bal >> hshift);  // one 64-bit shift per lane
        mine = (myv == v) ? word : mine;
      }
      return mine & cmask;
    };
    const gw_ptr C64 = (gw_ptr)Cm;
    const int64_t n_words = n_words32 >> 1;
    const int64_t w0 = tn * 2;  // first 64-bit word of the tile's columns
    if (w0 >= n_words) return;  // uniform
    const bool vec16 = w0 + 1 < n_words &&
                       ((reinterpret_cast<uintptr_t>(Cm) & 15) | (uintptr_t)(ldc & 1)) == 0;
#pragma unroll
    for (int f = 0; f < RA; ++f) {
      // one row block at a time: the scheduler would otherwise hoist every block's
      // ballots ahead of the stores and park the masks in VGPR lanes
      __builtin_amdgcn_sched_barrier(0);
      uint64_t word[2];
#pragma unroll
      for (int h = 0; h < 2; ++h)
        word[h] = (uint64_t)pack(f, 2 * h) | ((uint64_t)pack(f, 2 * h + 1) << 32);
      const int64_t row = tm * TM + 32 * f + li;
      if (half == 0 && row < m) {
        const gw_ptr dst = C64 + row * ldc + w0;
        if (vec16) {
          const gw2_ptr d2 = (gw2_ptr)dst;
          cpair_t x = {word[0], word[1]};
          if (accumulate) {
            const cpair_t old = *d2;
            x = gf2 ? (x ^ old) : (x | old);
          }
          *d2 = x;
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if (w0 + h >= n_words) break;  // uniform
            uint64_t x = word[h];
            if (accumulate) x = gf2 ? (x ^ dst[h]) : (x | dst[h]);
            dst[h] = x;
          }
        }
      }
    }
  }
}

// KV = 64-bit words per lane per load (1: 8-byte loads, 2: 16-byte loads when
// the operands are 16-byte aligned).  Lane half h takes words 2*KV*step + KV*h + v.
// STEPS > 0: the launch guarantees exactly STEPS full steps and no tail words
// (k = 128 * KV * STEPS bits); the loop then unrolls completely, so the
// compiler knows every load in flight, and NB register buffers keep the words
// of step st + NB - 1 in flight while step st computes.
template <int SEMI, int RA, int RB, int KV, int FMT, int NB = 2, int STEPS = 0, bool WIDE = true,
          bool SHORT = false, bool BOTH = false>
__device__ __forceinline__ void tile(const uint64_t* __restrict__ A, int64_t lda,
                                     const uint64_t* __restrict__ BT, int64_t ldbt,
                                     uint64_t* __restrict__ Cm, int64_t ldc, int64_t m,
                                     int64_t k, int64_t n, int64_t tm, int64_t tn,
                                     int accumulate, int semiring = SEMI) {
  constexpr int TM = 32 * RA, TN = 32 * RB;
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int li = lane & 31;
  const int64_t kw = (k + 63) >> 6;

  gq_ptr arow[RA];
  gq_ptr brow[RB];
#pragma unroll
  for (int f = 0; f < RA; ++f) {
    int64_t r = tm * TM + 32 * f + li;
    r = r < m ? r : m - 1;
    arow[f] = (gq_ptr)A + r * lda + KV * half;
  }
#pragma unroll
  for (int g = 0; g < RB; ++g) {
    int64_t c = tn * TN + 32 * g + li;
    c = c < n ? c : n - 1;
    brow[g] = (gq_ptr)BT + c * ldbt + KV * half;
  }

  using AccV = typename Acc<FMT>::type;
  AccV acc[RA][RB];
#pragma unroll
  for (int f = 0; f < RA; ++f)
#pragma unroll
    for (int g = 0; g < RB; ++g) acc[f][g] = AccV{};

  // Main loop over full steps of 2*KV words, software-pipelined: the words of
  // step st+1 are requested before the MFMAs of step st are issued, so the
  // memory latency hides behind a whole step of matrix-core work.
  // Two register buffers alternate (the loop is unrolled by two), so no copy
  // of a loaded buffer is ever needed inside the loop.
  const int64_t full_steps = kw / (2 * KV);
  uint64_t a0[KV][RA], b0[KV][RB], a1[KV][RA], b1[KV][RB];
  auto fetch = [&](int64_t st, uint64_t (&xa)[KV][RA], uint64_t (&xb)[KV][RB]) {
    const int64_t w = st * 2 * KV;
    if constexpr (KV == 2) {
#pragma unroll
      for (int f = 0; f < RA; ++f) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>((const uint64_t*)(arow[f] + w));
        xa[0][f] = v.x;
        xa[1][f] = v.y;
      }
#pragma unroll
      for (int g = 0; g < RB; ++g) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>((const uint64_t*)(brow[g] + w));
        xb[0][g] = v.x;
        xb[1][g] = v.y;
      }
    } else {
#pragma unroll
      for (int f = 0; f < RA; ++f) xa[0][f] = arow[f][w];
#pragma unroll
      for (int g = 0; g < RB; ++g) xb[0][g] = brow[g][w];
    }
  };
  auto compute = [&](const uint64_t (&xa)[KV][RA], const uint64_t (&xb)[KV][RB]) {
#pragma unroll
    for (int v = 0; v < KV; ++v) mfma_word<SEMI, RA, RB, FMT, WIDE, SHORT, BOTH>(xa[v], xb[v], acc);
  };
  if constexpr (STEPS > 0) {
    static_assert(STEPS >= NB, "an unrolled pipeline needs at least NB steps");
    uint64_t xa[NB][KV][RA], xb[NB][KV][RB];
#pragma unroll
    for (int i = 0; i + 1 < NB; ++i) fetch(i, xa[i], xb[i]);
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      if (s + NB - 1 < STEPS) fetch(s + NB - 1, xa[(s + NB - 1) % NB], xb[(s + NB - 1) % NB]);
      __builtin_amdgcn_sched_barrier(0);
      // a wave issuing its matrix-core block takes issue priority over the other wave
      // of its SIMD (which is then typically in its first loads or its epilogue); the
      // short tiles of the recursion gain from it, the long-k loop does not.  int8 only:
      // the E2M1 build of this pipeline (which spills) returned wrong words with two
      // waves per SIMD while it raised its priority, and exact ones without the raise.
      if constexpr (FMT == FMT_I8) __builtin_amdgcn_s_setprio(1);
      compute(xa[s % NB], xb[s % NB]);
      if constexpr (FMT == FMT_I8) __builtin_amdgcn_s_setprio(0);
    }
    epilogue<SEMI, RA, RB, FMT>(acc, Cm, ldc, m, n, tm, tn, accumulate, semiring);
    return;
  }
  // words by which the row pointers have been moved forward (the chunked loop below
  // advances them, so no copy of the original pointers stays live across it)
  int64_t adv = 0;
  if constexpr (STEPS < 0) {
    // Long k: a loop over chunks of CH = -STEPS steps, each fully unrolled, with NB
    // buffers rotating across chunk boundaries (CH is a multiple of NB, so every chunk
    // starts on buffer 0); the tail after the last whole chunk drains with guarded loads.
    // Steps are counted from the advanced pointers.
    constexpr int CH = -STEPS;
    static_assert(CH % NB == 0, "a chunk must hold whole rotations");
    uint64_t xa[NB][KV][RA], xb[NB][KV][RB];
    if (full_steps >= CH + NB) {
#pragma unroll
      for (int i = 0; i + 1 < NB; ++i) fetch(i, xa[i], xb[i]);
      int64_t st = 0;
      for (; st + CH + NB - 1 <= full_steps; st += CH) {
#pragma unroll
        for (int s = 0; s < CH; ++s) {
          fetch(s + NB - 1, xa[(s + NB - 1) % NB], xb[(s + NB - 1) % NB]);
          __builtin_amdgcn_sched_barrier(0);
          compute(xa[s % NB], xb[s % NB]);
        }
#pragma unroll
        for (int f = 0; f < RA; ++f) arow[f] += CH * 2 * KV;
#pragma unroll
        for (int g = 0; g < RB; ++g) brow[g] += CH * 2 * KV;
      }
      adv = st * 2 * KV;
#pragma unroll
      for (int s = 0; s < CH + NB - 1; ++s) {
        if (st + s < full_steps) {
          if (st + s + NB - 1 < full_steps)
            fetch(s + NB - 1, xa[(s + NB - 1) % NB], xb[(s + NB - 1) % NB]);
          __builtin_amdgcn_sched_barrier(0);
          compute(xa[s % NB], xb[s % NB]);
        }
      }
      // tail words, then the epilogue (below)
      goto tail;
    }
  }
  if (full_steps > 0) fetch(0, a0, b0);
  {
  int64_t st = 0;
  // sched_barrier(0) keeps the scheduler from sinking the loads below the MFMAs
  for (; st + 1 < full_steps; st += 2) {
    fetch(st + 1, a1, b1);
    __builtin_amdgcn_sched_barrier(0);
    compute(a0, b0);
    if (st + 2 < full_steps) fetch(st + 2, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    compute(a1, b1);
  }
  if (st < full_steps) compute(a0, b0);
  }
tail:
  // Tail: words past the end of the row read as zero.
  {
    const int64_t w = full_steps * 2 * KV;
    if (w < kw) {
#pragma unroll
      for (int v = 0; v < KV; ++v) {
        const int64_t wi = w + KV * half + v;
        uint64_t xa[RA], xb[RB];
#pragma unroll
        for (int f = 0; f < RA; ++f) xa[f] = wi < kw ? arow[f][w - adv + v] : 0ull;
#pragma unroll
        for (int g = 0; g < RB; ++g) xb[g] = wi < kw ? brow[g][w - adv + v] : 0ull;
        mfma_word<SEMI, RA, RB, FMT, WIDE, SHORT, BOTH>(xa, xb, acc);
      }
    }
  }

  epilogue<SEMI, RA, RB, FMT>(acc, Cm, ldc, m, n, tm, tn, accumulate, semiring);
}

// A workgroup item of 2 x 2 wave tiles of 128 x 64 (256 rows of A, 128 rows of B^T,
// item coordinates (im, in)) with its operand rows staged through LDS: per stage of 8
// words of k the four waves load those 384 rows once, with 16-byte coalesced loads,
// into LDS (rows padded to 80 bytes so the lanes of one 16-byte LDS read hit distinct
// banks), and every wave reads its own rows from there, so each operand row is fetched
// from L2 once per workgroup instead of once per wave that uses it.  The next stage is
// loaded into registers while the current one computes.  Words past the end of k read
// as zero; whole 4-word groups past it are skipped.  All four waves (w = 0..3) take
// part in the loads and barriers; waves whose tile lies outside the problem only skip
// the epilogue.  smem: kLdsItemBytes of LDS.
constexpr int kLdsKs = 8;                          // words of k per stage
constexpr int kLdsRowB = 80;                       // padded LDS row (64 data bytes + 16)
constexpr int kLdsRows = 256 + 128;                // A rows, then B^T rows
constexpr int kLdsPanel = kLdsRows * kLdsRowB;     // bytes per stage buffer
constexpr int kLdsChunks = kLdsRows * 4 / 256;     // 16-byte chunks per thread per stage
constexpr int kLdsItemBytes = 2 * kLdsPanel;

// A thread's share of an item's stage: chunk i is row (tid >> 2) + 64 i of the item's
// 384 rows, words 2 (tid & 3) and 2 (tid & 3) + 1 of the stage.
typedef uint64_t LdsStage[kLdsChunks][2];

__device__ __forceinline__ void lds_sources(const uint64_t* Ap, int64_t lda, const uint64_t* BTp,
                                            int64_t ldbt, int64_t m, int64_t n, int64_t im,
                                            int64_t in, gq_ptr (&src)[kLdsChunks]) {
  const int tid = threadIdx.x, part = tid & 3;
  const int64_t row0 = im * 256, col0 = in * 128;
#pragma unroll
  for (int i = 0; i < kLdsChunks; ++i) {
    const int r = (tid >> 2) + 64 * i;
    if (r < 256) {
      int64_t g = row0 + r;
      g = g < m ? g : m - 1;
      src[i] = (gq_ptr)Ap + g * lda + 2 * part;
    } else {
      int64_t g = col0 + (r - 256);
      g = g < n ? g : n - 1;
      src[i] = (gq_ptr)BTp + g * ldbt + 2 * part;
    }
  }
}

// Load the stage starting at word w0 (words at or past kw read as zero).
__device__ __forceinline__ void lds_load(const gq_ptr (&src)[kLdsChunks], int64_t w0, int64_t kw,
                                         bool aligned, LdsStage& stage) {
  const int64_t wd = w0 + 2 * (threadIdx.x & 3);
#pragma unroll
  for (int i = 0; i < kLdsChunks; ++i) {
    if (aligned && wd + 1 < kw) {
      const ulonglong2 v = *reinterpret_cast<const ulonglong2*>((const uint64_t*)(src[i] + w0));
      stage[i][0] = v.x;
      stage[i][1] = v.y;
    } else {
      stage[i][0] = wd < kw ? src[i][w0] : 0ull;
      stage[i][1] = wd + 1 < kw ? src[i][w0 + 1] : 0ull;
    }
  }
}

// The first stage of item (im, in), for a caller that overlaps it with other work.
__device__ __forceinline__ void lds_prefetch(const uint64_t* Ap, int64_t lda, const uint64_t* BTp,
                                             int64_t ldbt, int64_t m, int64_t k, int64_t n,
                                             int64_t im, int64_t in, bool aligned,
                                             LdsStage& stage) {
  gq_ptr src[kLdsChunks];
  lds_sources(Ap, lda, BTp, ldbt, m, n, im, in, src);
  lds_load(src, 0, (k + 63) >> 6, aligned, stage);
}

struct LdsNoNext {
  __device__ void operator()() const {}
  __device__ bool operator()(LdsStage&) const { return false; }
};

// preloaded: `stage` already holds the item's first stage (lds_prefetch).  at_last()
// runs on every wave just before the barrier that ends the last stage (a persistent
// caller's wave 0 names the next item there); after that barrier, before the epilogue,
// prefetch(stage) may load the next item's first stage into `stage` and returns whether
// it did, which lds_item returns.
template <int SEMI, int FMT, bool WIDE, bool SHORT = false, class AtLast = LdsNoNext,
          class Prefetch = LdsNoNext>
__device__ __forceinline__ bool lds_item(const uint64_t* Ap, int64_t lda, const uint64_t* BTp,
                                         int64_t ldbt, uint64_t* C, int64_t ldc, int64_t m,
                                         int64_t k, int64_t n, int64_t im, int64_t in,
                                         int64_t tiles_m, int64_t tiles_n, bool aligned,
                                         int accumulate, int semiring, int w,
                                         unsigned char* smem, LdsStage& stage,
                                         bool preloaded = false, AtLast at_last = AtLast(),
                                         Prefetch prefetch = Prefetch()) {
  constexpr int RA = 4, RB = 2;
  const int tid = threadIdx.x, lane = tid & 63, half = lane >> 5, li = lane & 31;
  const int64_t kw = (k + 63) >> 6;
  gq_ptr src[kLdsChunks];
  lds_sources(Ap, lda, BTp, ldbt, m, n, im, in, src);
  int soff[kLdsChunks];
#pragma unroll
  for (int i = 0; i < kLdsChunks; ++i) soff[i] = ((tid >> 2) + 64 * i) * kLdsRowB + (tid & 3) * 16;
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < kLdsChunks; ++i) {
      ulonglong2 v;
      v.x = stage[i][0];
      v.y = stage[i][1];
      *reinterpret_cast<ulonglong2*>(smem + buf * kLdsPanel + soff[i]) = v;
    }
  };
  using AccV = typename Acc<FMT>::type;
  AccV acc[RA][RB];
#pragma unroll
  for (int f = 0; f < RA; ++f)
#pragma unroll
    for (int g = 0; g < RB; ++g) acc[f][g] = AccV{};
  const int wy = w >> 1, wx = w & 1;
  int aoff[RA], boff[RB];
#pragma unroll
  for (int f = 0; f < RA; ++f) aoff[f] = (wy * 128 + 32 * f + li) * kLdsRowB + 16 * half;
#pragma unroll
  for (int g = 0; g < RB; ++g) boff[g] = (256 + wx * 64 + 32 * g + li) * kLdsRowB + 16 * half;

  const int64_t stages = (kw + kLdsKs - 1) / kLdsKs;
  if (!preloaded) lds_load(src, 0, kw, aligned, stage);
  store(0);
  __syncthreads();
  if (stages == 0) {
    at_last();
    __syncthreads();
  }
  for (int64_t st = 0; st < stages; ++st) {
    const int cur = (int)(st & 1);
    if (st + 1 < stages) lds_load(src, (st + 1) * kLdsKs, kw, aligned, stage);
    const unsigned char* base = smem + cur * kLdsPanel;
    // two groups of 4 words per stage: lane half h takes words 4s + 2h and 4s + 2h + 1
#pragma unroll
    for (int s2 = 0; s2 < kLdsKs / 4; ++s2) {
      if (st * kLdsKs + 4 * s2 >= kw) break;  // uniform: only zero words are left
      uint64_t xa[2][RA], xb[2][RB];
#pragma unroll
      for (int f = 0; f < RA; ++f) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(base + aoff[f] + 32 * s2);
        xa[0][f] = v.x;
        xa[1][f] = v.y;
      }
#pragma unroll
      for (int g = 0; g < RB; ++g) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(base + boff[g] + 32 * s2);
        xb[0][g] = v.x;
        xb[1][g] = v.y;
      }
      mfma_word<SEMI, RA, RB, FMT, WIDE, SHORT>(xa[0], xb[0], acc);
      mfma_word<SEMI, RA, RB, FMT, WIDE, SHORT>(xa[1], xb[1], acc);
    }
    if (st + 1 < stages)
      store(cur ^ 1);
    else
      at_last();
    __syncthreads();
  }
  // no wave reads this item's LDS panels any more: the next item's first stage can be
  // in flight during the epilogue
  const bool next = prefetch(stage);
  const int64_t tm = 2 * im + wy, tn = 2 * in + wx;
  if (tm < tiles_m && tn < tiles_n)
    epilogue<SEMI, RA, RB, FMT>(acc, C, ldc, m, n, tm, tn, accumulate, semiring);
  return next;
}

}  // namespace mfma
}  // namespace bmm
