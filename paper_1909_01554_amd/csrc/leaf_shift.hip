// The recursion's last level shifted into the int8 leaf (section 3.15, shifting
// levels between layers).
//
// Without the shift, the last parallel level of the recursion expands every
// parent's operands into seven children in HBM (T_h = sum_q alpha_hq T_q,
// S_h = sum_q beta_hq S_q), the batched leaf multiplies the children, and a
// compression combines the seven products into the parent's quadrants
// (Q_q = sum_h gamma_qh P_h).  Here one workgroup owns a tile position of a
// parent and runs all seven products for it: each child operand word is formed
// in registers as the XOR of the one or two parent quadrant words that alpha
// (beta) selects, and each product's bits, once reduced, are XORed in LDS into
// the parent quadrants gamma sends them to; the four quadrant tiles are written
// once at the end.  The children and their products never reach HBM, and the
// seven k-loops of a tile run back to back, the next product's first operand
// words loading while the current one finishes.
//
// Schemes whose alpha and beta rows have weight <= 2 (the self-inverse and the
// chaining alternative bases) are supported; Strassen-Winograd keeps the
// unshifted path.
#include "mfma_tile.h"
#include "scheme.h"

namespace bmm {
namespace {

using mfma::gd_ptr;
typedef const BMM_GLOBAL char* gc_ptr;
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

constexpr int RA = 4, RB = 2;        // 128 x 64 wave tile, as the recursion's int8 leaf

// Zero words that the second load of a weight-1 combination reads instead of a
// parent quadrant (one row of k <= 4096 bits; every lane reads the same few lines,
// so these loads hit in the vector L1 and cost no L2 traffic).
__device__ __align__(256) uint64_t zero_words[64];
constexpr int TM = 32 * RA, TN = 32 * RB;
constexpr int kWaves = 4;

// Coefficient masks of a scheme, read off its register programs run on bit masks
// (constant-folded): bit q of lhs(h) / rhs(h) selects stored quadrant q (order 00,
// 01, 10, 11) of the left / transposed right operand for product h; bit h of out(q)
// sends product h to result quadrant q.  h and q are wave-uniform, so the selection
// stays in scalar registers.
template <int SCH>
__device__ __forceinline__ uint32_t lhs_mask(int h) {
  uint64_t o[7];
  scheme::expand_one<SCH, 0>(1, 2, 4, 8, o);
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 7; ++i) r = i == h ? (uint32_t)o[i] : r;
  return r;
}
template <int SCH>
__device__ __forceinline__ uint32_t rhs_mask(int h) {
  uint64_t o[7];
  scheme::expand_one<SCH, 1>(1, 2, 4, 8, o);
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 7; ++i) r = i == h ? (uint32_t)o[i] : r;
  return r;
}
template <int SCH>
__device__ __forceinline__ uint32_t out_mask(int q) {
  const uint64_t in[7] = {1, 2, 4, 8, 16, 32, 64};
  uint64_t c[4];
  scheme::compress_one<SCH>(in, c[0], c[1], c[2], c[3]);
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) r = i == q ? (uint32_t)c[i] : r;
  return r;
}

// Word offsets of the (at most two) parent quadrants a child operand sums; mask1 is
// nonzero for weight 2 (the second quadrant is loaded and XORed in; for weight 1 the
// second load reads zero words).
struct Pick {
  int64_t off0, off1;
  uint64_t mask1;
};

__device__ __forceinline__ Pick pick(uint32_t qmask, int64_t rows, int64_t ld, int64_t kw) {
  const int q0 = __builtin_ctz(qmask);
  const int q1 = 31 - __builtin_clz(qmask);
  Pick p;
  p.off0 = (int64_t)(q0 >> 1) * rows * ld + (int64_t)(q0 & 1) * kw;
  p.off1 = (int64_t)(q1 >> 1) * rows * ld + (int64_t)(q1 & 1) * kw;
  p.mask1 = q1 != q0 ? ~0ull : 0ull;
  return p;
}

// KV: 64-bit words per lane per load (2: 16-byte loads); STEPS: steps of 2*KV words per
// product (k = 128 * KV * STEPS bits).  Loads run one step ahead: at the start of a step
// the raw words of that step are combined into its operands, the next step's loads (in
// the last step of a product: the next product's first) are issued into the freed raw
// registers, and then the step's MFMAs run.
template <int SCH, int KV, int STEPS, bool PREFETCH_NEXT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void leaf_shift_kernel(
    ShiftBatch p, int64_t tiles_m, int64_t tiles_n) {
  __shared__ uint32_t acc_bits[kWaves][4][RA * RB][32];
  const int64_t grid_m = (tiles_m + 1) >> 1, grid_n = (tiles_n + 1) >> 1;
  const TileCoord c = xcd_tile(blockIdx.x, gridDim.x, grid_m, grid_n);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
  const int64_t tm = 2 * c.tm + (w >> 1);
  const int64_t tn = 2 * c.tn + (w & 1);
  if (c.b >= p.parents || tm >= tiles_m || tn >= tiles_n) return;  // uniform per wave
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int li = lane & 31;
  const int64_t kw = p.k >> 6;

  // this lane's rows of the parent's top-left quadrant, as 32-bit word offsets from the
  // parent's (wave-uniform) base; quadrants are further uniform offsets, so every load
  // takes a scalar base and a per-lane 32-bit offset
  const uint64_t* tbase = p.T + c.b * p.strideT;
  const uint64_t* sbase = p.S + c.b * p.strideS;
  uint32_t arow[RA], brow[RB];  // byte offsets
#pragma unroll
  for (int f = 0; f < RA; ++f) {
    int64_t r = tm * TM + 32 * f + li;
    r = r < p.m ? r : p.m - 1;
    arow[f] = (uint32_t)((r * p.ldt + KV * half) * 8);
  }
#pragma unroll
  for (int g = 0; g < RB; ++g) {
    const int64_t col = tn * TN + 32 * g + li;  // n is a multiple of 64: in range
    brow[g] = (uint32_t)((col * p.lds + KV * half) * 8);
  }
  if (half == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int fg = 0; fg < RA * RB; ++fg) acc_bits[w][q][fg][li] = 0u;
  }

  using mfma::v16i;
  v16i acc[RA][RB];
  uint64_t ua[KV][RA], va[KV][RA], ub[KV][RB], vb[KV][RB];  // raw words in flight
  uint64_t xa[KV][RA], xb[KV][RB];                          // the step's operands

  const uint32_t zoff = (uint32_t)(KV * half * 8);
  auto fetch = [&](const Pick& pa, const Pick& pb, int st) {
    const int64_t wd = (int64_t)st * 2 * KV;
    const gc_ptr a0 = (gc_ptr)(tbase + pa.off0 + wd), b0 = (gc_ptr)(sbase + pb.off0 + wd);
    const gc_ptr a1 = pa.mask1 ? (gc_ptr)(tbase + pa.off1 + wd) : (gc_ptr)(zero_words + wd);
    const gc_ptr b1 = pb.mask1 ? (gc_ptr)(sbase + pb.off1 + wd) : (gc_ptr)(zero_words + wd);
#pragma unroll
    for (int f = 0; f < RA; ++f) {
      const uint32_t o1 = pa.mask1 ? arow[f] : zoff;
      if constexpr (KV == 2) {
        const u64x2 u = *reinterpret_cast<const BMM_GLOBAL u64x2*>(a0 + arow[f]);
        const u64x2 v = *reinterpret_cast<const BMM_GLOBAL u64x2*>(a1 + o1);
        ua[0][f] = u.x;
        ua[1][f] = u.y;
        va[0][f] = v.x;
        va[1][f] = v.y;
      } else {
        ua[0][f] = *reinterpret_cast<const BMM_GLOBAL uint64_t*>(a0 + arow[f]);
        va[0][f] = *reinterpret_cast<const BMM_GLOBAL uint64_t*>(a1 + o1);
      }
    }
#pragma unroll
    for (int g = 0; g < RB; ++g) {
      const uint32_t o1 = pb.mask1 ? brow[g] : zoff;
      if constexpr (KV == 2) {
        const u64x2 u = *reinterpret_cast<const BMM_GLOBAL u64x2*>(b0 + brow[g]);
        const u64x2 v = *reinterpret_cast<const BMM_GLOBAL u64x2*>(b1 + o1);
        ub[0][g] = u.x;
        ub[1][g] = u.y;
        vb[0][g] = v.x;
        vb[1][g] = v.y;
      } else {
        ub[0][g] = *reinterpret_cast<const BMM_GLOBAL uint64_t*>(b0 + brow[g]);
        vb[0][g] = *reinterpret_cast<const BMM_GLOBAL uint64_t*>(b1 + o1);
      }
    }
  };
  auto combine = [&](const Pick& pa, const Pick& pb) {
#pragma unroll
    for (int v = 0; v < KV; ++v) {
#pragma unroll
      for (int f = 0; f < RA; ++f) xa[v][f] = ua[v][f] ^ va[v][f];
#pragma unroll
      for (int g = 0; g < RB; ++g) xb[v][g] = ub[v][g] ^ vb[v][g];
    }
  };

  Pick ca = pick(lhs_mask<SCH>(0), p.m, p.ldt, kw), cb = pick(rhs_mask<SCH>(0), p.n, p.lds, kw);
  fetch(ca, cb, 0);
  for (int h = 0; h < 7; ++h) {
    const bool more = h + 1 < 7;
    const Pick na = more ? pick(lhs_mask<SCH>(h + 1), p.m, p.ldt, kw) : ca;
    const Pick nb = more ? pick(rhs_mask<SCH>(h + 1), p.n, p.lds, kw) : cb;
#pragma unroll
    for (int f = 0; f < RA; ++f)
#pragma unroll
      for (int g = 0; g < RB; ++g) acc[f][g] = v16i{};
#pragma unroll
    for (int s = 0; s < STEPS; ++s) {
      combine(ca, cb);
      if (s + 1 < STEPS) fetch(ca, cb, s + 1);
      if constexpr (PREFETCH_NEXT)
        if (s + 1 == STEPS && more) fetch(na, nb, 0);  // the next product's first words
      __builtin_amdgcn_sched_barrier(0);
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int v = 0; v < KV; ++v)
        mfma::mfma_word<GF2, RA, RB, mfma::FMT_I8, false>(xa[v], xb[v], acc);
      __builtin_amdgcn_s_setprio(0);
      __builtin_amdgcn_sched_barrier(0);
    }
    // reduce this product's counts to parity bits (ballots: lanes 0..31 end up with
    // one 32-column word of one row per 32 x 32 block) and XOR them into the parent
    // quadrants that gamma sends product h to
    const int myv = ((li >> 3) << 2) | (li & 3);
    const int myhi = (li >> 2) & 1;
    uint32_t qm[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) qm[q] = (out_mask<SCH>(q) >> h) & 1u;
#pragma unroll
    for (int f = 0; f < RA; ++f)
#pragma unroll
      for (int g = 0; g < RB; ++g) {
        uint32_t mine = 0;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const uint64_t bal = __ballot((acc[f][g][v] & 1) != 0);
          const uint32_t word = myhi ? (uint32_t)(bal >> 32) : (uint32_t)bal;
          mine = (myv == v) ? word : mine;
        }
        if (half == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (qm[q]) acc_bits[w][q][f * RB + g][li] ^= mine;
        }
      }
    ca = na;
    cb = nb;
    if constexpr (!PREFETCH_NEXT)
      if (more) fetch(ca, cb, 0);
  }

  // the four quadrant tiles of the parent's result
  if (half == 0) {
    const gd_ptr Q32 = (gd_ptr)(p.Q + c.b * p.strideQ);
    const int64_t ldq32 = 2 * p.ldq;
    const int64_t nw32 = p.n >> 5;
#pragma unroll
    for (int f = 0; f < RA; ++f) {
      const int64_t row = tm * TM + 32 * f + li;
      if (row >= p.m) continue;
#pragma unroll
      for (int g = 0; g < RB; ++g) {
        const int64_t cw = (tn * TN + 32 * g) >> 5;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const gd_ptr dst = Q32 + (row + (q >> 1) * p.m) * ldq32 + (q & 1) * nw32 + cw;
          uint32_t v = acc_bits[w][q][f * RB + g][li];
          if (p.accumulate) v ^= *dst;
          *dst = v;
        }
      }
    }
  }
}

template <int SCH, int KV, int STEPS>
hipError_t launch_k(const ShiftBatch& p, dim3 g, int64_t tiles_m, int64_t tiles_n,
                    hipStream_t s) {
  // the next product's first loads overlap the epilogue only where registers allow
  hipLaunchKernelGGL((leaf_shift_kernel<SCH, KV, STEPS, KV == 1>), g, dim3(256), 0, s, p,
                     tiles_m, tiles_n);
  return hipGetLastError();
}

template <int SCH>
hipError_t launch_sch(const ShiftBatch& p, dim3 g, int64_t tiles_m, int64_t tiles_n,
                      bool aligned16, hipStream_t s) {
  // steps of 2 * KV words: k = 2048 -> 8 (16-byte loads) or 16 (8-byte loads)
  if (p.k == 2048)
    return aligned16 ? launch_k<SCH, 2, 8>(p, g, tiles_m, tiles_n, s)
                     : launch_k<SCH, 1, 16>(p, g, tiles_m, tiles_n, s);
  return aligned16 ? launch_k<SCH, 2, 16>(p, g, tiles_m, tiles_n, s)
                   : launch_k<SCH, 1, 32>(p, g, tiles_m, tiles_n, s);
}

}  // namespace

bool leaf_shift_supported(int scheme, int64_t m, int64_t k, int64_t n) {
  return (scheme == BMM_SCHEME_SELF_INVERSE || scheme == BMM_SCHEME_CHAINING) && m > 0 &&
         (k == 2048 || k == 4096) && n > 0 && n % 64 == 0;
}

// Per-lane offsets are 32-bit byte offsets: a parent's rows must span fewer than 2^32 bytes.
bool leaf_shift_fits(int64_t rows, int64_t ld) {
  return rows > 0 && ld > 0 && 2 * rows * ld < ((int64_t)1 << 29);
}

hipError_t launch_leaf_shift(int scheme, const ShiftBatch& p, int kv, hipStream_t s) {
  if (p.parents <= 0 || p.m <= 0 || p.n <= 0) return hipSuccess;
  if (!leaf_shift_supported(scheme, p.m, p.k, p.n) || !leaf_shift_fits(p.m, p.ldt) ||
      !leaf_shift_fits(p.n, p.lds))
    return hipErrorInvalidValue;
  const int64_t tiles_m = (p.m + TM - 1) / TM, tiles_n = p.n / TN;
  const int64_t blocks = ((tiles_m + 1) / 2) * ((tiles_n + 1) / 2) * p.parents;
  if (!grid_fits(blocks, 256)) return kGridTooLarge;
  const bool aligned16 =
      kv == 2 &&
      ((reinterpret_cast<uintptr_t>(p.T) | reinterpret_cast<uintptr_t>(p.S)) & 15) == 0 &&
      ((p.ldt | p.lds | p.strideT | p.strideS | (p.k >> 6)) & 1) == 0;
  const dim3 g((unsigned)blocks);
  return scheme == BMM_SCHEME_CHAINING
             ? launch_sch<BMM_SCHEME_CHAINING>(p, g, tiles_m, tiles_n, aligned16, s)
             : launch_sch<BMM_SCHEME_SELF_INVERSE>(p, g, tiles_m, tiles_n, aligned16, s);
}

}  // namespace bmm
