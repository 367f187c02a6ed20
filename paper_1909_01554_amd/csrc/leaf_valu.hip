// Cubic leaf product on the vector ALUs of gfx950, bit-parallel over 32-bit words.
//
// C[i][k] = SUM_j A[i][j] B[j][k] is computed in dot-product form against B
// transposed: for row i of A and row k of BT, the partial word
// acc ^= a & b (GF(2)) or acc |= a & b (Boolean) is folded over the 32-bit
// words of the k dimension with one three-input v_bitop3_b32 per 32 bit
// products, and reduced at the end to parity(popcount(acc)) or (acc != 0).
//
// A 256-thread workgroup owns a 128 x 128 tile of C; each wave a 64 x 64
// sub-tile and each lane an 8 x 8 block of 32-bit accumulators (rows a + 8i,
// columns b + 8j for lane = a + 8b).  Word tiles of A and BT are staged in LDS
// (double buffered, 16-byte reads; rows padded so the eight distinct rows a
// wave reads at once fall in distinct banks).  Output bits are assembled into
// packed row words with three cross-lane XOR-shuffles.
#include "bmm_internal.h"

namespace bmm {
namespace {

constexpr int TM = 128;
constexpr int TN = 128;
constexpr int KC = 8;           // 64-bit words of k per LDS stage
constexpr int KCD = 2 * KC;     // the same in dwords
constexpr int STR = KCD + 4;    // LDS row stride in dwords

template <int SEMI>
__device__ __forceinline__ uint32_t fold(uint32_t a, uint32_t b, uint32_t acc) {
  // truth tables: (a & b) ^ acc = 0x6A, (a & b) | acc = 0xEA
  return __builtin_amdgcn_bitop3_b32(a, b, acc, SEMI == GF2 ? 0x6A : 0xEA);
}

template <int SEMI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void leaf_valu_kernel(LeafBatch p, int64_t tiles_m,
                                                        int64_t tiles_n) {
  __shared__ __attribute__((aligned(16))) uint32_t sA[2][TM * STR];
  __shared__ __attribute__((aligned(16))) uint32_t sB[2][TN * STR];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int a = lane & 7, bb = lane >> 3;

  // workgroups ordered for L2 reuse per XCD
  const TileCoord c = xcd_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n);
  const int64_t b = c.b;
  if (b >= p.batch) return;  // uniform per workgroup
  const int64_t tm = c.tm;
  const int64_t tn = c.tn;
  const uint64_t* A = p.A + b * p.strideA;
  const uint64_t* BT = p.BT + b * p.strideB;
  const int64_t kw = (p.k + 63) >> 6;

  // Global -> LDS staging: thread tid loads words 4*(tid&1) .. +3 of tile row tid>>1.
  const int lr = tid >> 1;
  const int lw = (tid & 1) * 4;
  int64_t ga = tm * TM + lr;
  ga = ga < p.m ? ga : p.m - 1;
  int64_t gb = tn * TN + lr;
  gb = gb < p.n ? gb : p.n - 1;
  const uint64_t* srcA = A + ga * p.lda;
  const uint64_t* srcB = BT + gb * p.ldbt;

  uint64_t ra[4], rb[4];
  auto load_stage = [&](int64_t w0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t w = w0 + lw + q;
      ra[q] = w < kw ? srcA[w] : 0ull;
      rb[q] = w < kw ? srcB[w] : 0ull;
    }
  };
  auto store_stage = [&](int buf) {
    uint32_t* da = &sA[buf][lr * STR + 2 * lw];
    uint32_t* db = &sB[buf][lr * STR + 2 * lw];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      da[2 * q] = (uint32_t)ra[q];
      da[2 * q + 1] = (uint32_t)(ra[q] >> 32);
      db[2 * q] = (uint32_t)rb[q];
      db[2 * q + 1] = (uint32_t)(rb[q] >> 32);
    }
  };

  uint32_t acc[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = 0u;

  const int64_t stages = (kw + KC - 1) / KC;
  if (stages > 0) {
    load_stage(0);
    store_stage(0);
  }
  __syncthreads();
  const int arow0 = (wy * 64 + a) * STR;
  const int brow0 = (wx * 64 + bb) * STR;
  for (int64_t st = 0; st < stages; ++st) {
    const int cur = (int)(st & 1);
    if (st + 1 < stages) load_stage((st + 1) * KC);
#pragma unroll 1
    for (int d = 0; d < KCD; d += 4) {
      // the eight BT rows' words stay in registers while the A rows stream by
      uint4 bv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        bv[j] = *reinterpret_cast<const uint4*>(&sB[cur][brow0 + 8 * j * STR + d]);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const uint4 av = *reinterpret_cast<const uint4*>(&sA[cur][arow0 + 8 * i * STR + d]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          acc[i][j] = fold<SEMI>(av.x, bv[j].x, acc[i][j]);
          acc[i][j] = fold<SEMI>(av.y, bv[j].y, acc[i][j]);
          acc[i][j] = fold<SEMI>(av.z, bv[j].z, acc[i][j]);
          acc[i][j] = fold<SEMI>(av.w, bv[j].w, acc[i][j]);
        }
      }
    }
    if (st + 1 < stages) store_stage(cur ^ 1);
    __syncthreads();
  }

  // Epilogue: lane (a, bb) holds rows a + 8i, columns bb + 8j of its wave tile.
  uint64_t keep = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint64_t word = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const uint32_t bit = (SEMI == GF2) ? (__popc(acc[i][j]) & 1u) : (acc[i][j] != 0u);
      word |= (uint64_t)bit << (bb + 8 * j);
    }
    word |= __shfl_xor(word, 8);
    word |= __shfl_xor(word, 16);
    word |= __shfl_xor(word, 32);
    keep = (bb == i) ? word : keep;
  }
  const int64_t row = tm * TM + wy * 64 + a + 8 * bb;
  const int64_t cword = tn * 2 + wx;
  const int64_t c0 = cword * 64;
  if (row < p.m && c0 < p.n) {
    const int64_t valid = p.n - c0;
    if (valid < 64) keep &= (1ull << valid) - 1ull;
    uint64_t* dst = p.C + b * p.strideC + row * p.ldc + cword;
    if (p.accumulate) keep = (SEMI == GF2) ? (keep ^ *dst) : (keep | *dst);
    *dst = keep;
  }
}

// Outer-product form (tile 2), for cubic products whose B is at hand row-major: every
// bit A[i][j] selects row j of B, C[i][.] ^= (A[i][j] ? B[j][.] : 0) (GF(2)) or |=
// (Boolean), 32 columns per v_bitop3_b32 with the selection as a sign-extended mask.  A
// wave owns 256 rows (four per lane) and 512 columns (16 dwords) of C; the words of row j
// of B that the wave needs are the same for all its lanes, so they are read with scalar
// loads into scalar registers and each fold reads one vector register besides its
// accumulator (no LDS).  The accumulators are the result bits themselves: no reduction.
// The four waves of a workgroup own 1024 rows over the same columns, so they read the
// same rows of B (scalar cache hits).  Scalar loads may complete out of order, so a use
// waits for every one in flight: row j + 1 is requested right after row j's first use,
// and its latency hides behind the rest of row j's folds and the other waves of the SIMD.
constexpr int OROWS = 4;             // rows per lane
constexpr int OCW = 16;              // C dwords (32 columns each) per wave
constexpr int OTM = 4 * 64 * OROWS;  // rows per workgroup
constexpr int OTN = 32 * OCW;        // columns per workgroup

template <bool FULL>
__device__ __forceinline__ void outer_row(const uint32_t* __restrict__ r, int ncw,
                                          uint32_t (&bw)[OCW]) {
#pragma unroll
  for (int c = 0; c < OCW; ++c) bw[c] = (FULL || c < ncw) ? r[c] : 0u;
}

// The steps of one k-dword a of A (min(left, 32) bits; left > 0): cur holds row j of B on
// entry and row j + 32 (or nothing past k) on exit; brow points at row j and advances.
template <int SEMI, bool FULL>
__device__ __forceinline__ void outer_dword(const uint32_t*& brow, int64_t ldb32, int64_t left,
                                            int ncw, const uint32_t (&a)[OROWS],
                                            uint32_t (&cur)[OCW], uint32_t (&acc)[OROWS][OCW]) {
  const int nsteps = (int)(left < 32 ? left : 32);
  for (int jb = 0; jb < nsteps; ++jb) {
    uint32_t msk[OROWS];
#pragma unroll
    for (int r = 0; r < OROWS; ++r) msk[r] = (uint32_t)__builtin_amdgcn_sbfe((int)a[r], jb, 1);
#pragma unroll
    for (int r = 0; r < OROWS; ++r) acc[r][0] = fold<SEMI>(msk[r], cur[0], acc[r][0]);
    __builtin_amdgcn_sched_barrier(0);
    brow += ldb32;
    uint32_t nxt[OCW];
    if (jb + 1 < left) outer_row<FULL>(brow, ncw, nxt);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 1; q < OCW; ++q)
#pragma unroll
      for (int r = 0; r < OROWS; ++r) acc[r][q] = fold<SEMI>(msk[r], cur[q], acc[r][q]);
#pragma unroll
    for (int q = 0; q < OCW; ++q) cur[q] = nxt[q];
  }
}

// FULL: the rows of B and C hold at least OCW dwords, so every wave reads a whole window
// of OCW dwords of row j (the last column tile's window is moved left to end at the row's
// end, and that wave stores only the columns of its own tile); otherwise (n < 512) the
// loads past the row read zero.
template <int SEMI, bool FULL>
__global__ __launch_bounds__(256) void leaf_valu_outer_kernel(
    const uint64_t* __restrict__ A, int64_t lda, const uint32_t* __restrict__ B, int64_t ldb32,
    uint64_t* __restrict__ C, int64_t ldc, int64_t m, int64_t k, int64_t n, int64_t tiles_m,
    int64_t tiles_n, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const TileCoord c = xcd_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n);
  const int64_t row0 = c.tm * OTM + wave * (64 * OROWS);
  const int64_t n32 = ((n + 63) >> 6) * 2;  // dwords per row of B and C (whole words)
  const int64_t own32 = c.tn * OCW;         // first C dword of the wave's own columns
  // first dword of the window the wave computes
  const int64_t col32 = FULL ? (own32 + OCW <= n32 ? own32 : n32 - OCW) : own32;
  const int ncw = (int)(n32 - col32 < OCW ? n32 - col32 : OCW);
  int64_t ri[OROWS];
  const uint32_t* arow[OROWS];
#pragma unroll
  for (int r = 0; r < OROWS; ++r) {
    ri[r] = row0 + 64 * r + lane;
    const int64_t g = ri[r] < m ? ri[r] : m - 1;
    arow[r] = reinterpret_cast<const uint32_t*>(A + g * lda);
  }
  uint32_t acc[OROWS][OCW];
#pragma unroll
  for (int r = 0; r < OROWS; ++r)
#pragma unroll
    for (int q = 0; q < OCW; ++q) acc[r][q] = 0u;
  // One step per bit j of k (outer_dword), 32 per k-dword of A. The k-dwords of A
  // alternate between two register sets, each loaded a whole k-dword ahead of its use
  // (the last one is reread rather than skipped, so no copy waits for a load).
  const int64_t k32 = (k + 31) >> 5;  // k-dwords of A
  const uint32_t* brow = B + col32;
  uint32_t a0[OROWS], a1[OROWS], cur[OCW];
#pragma unroll
  for (int r = 0; r < OROWS; ++r) a0[r] = arow[r][0];
  outer_row<FULL>(brow, ncw, cur);
  for (int64_t jw = 0; jw < k32; jw += 2) {
    const int64_t j1 = jw + 1 < k32 ? jw + 1 : k32 - 1;
#pragma unroll
    for (int r = 0; r < OROWS; ++r) a1[r] = arow[r][j1];
    outer_dword<SEMI, FULL>(brow, ldb32, k - 32 * jw, ncw, a0, cur, acc);
    if (jw + 1 >= k32) break;
    const int64_t j2 = jw + 2 < k32 ? jw + 2 : k32 - 1;
#pragma unroll
    for (int r = 0; r < OROWS; ++r) a0[r] = arow[r][j2];
    outer_dword<SEMI, FULL>(brow, ldb32, k - 32 * (jw + 1), ncw, a1, cur, acc);
  }
  // the accumulators are C's dwords: two make a 64-bit word of the row
  const int64_t nw = n32 >> 1, w0 = col32 >> 1, own = own32 >> 1;
#pragma unroll
  for (int r = 0; r < OROWS; ++r) {
    if (ri[r] >= m) continue;
    uint64_t* dst = C + ri[r] * ldc + w0;
#pragma unroll
    for (int w = 0; w < OCW / 2; ++w) {
      if (w0 + w >= nw) break;  // uniform
      if (w0 + w < own) continue;  // uniform: the previous tile's columns
      uint64_t x = (uint64_t)acc[r][2 * w] | ((uint64_t)acc[r][2 * w + 1] << 32);
      const int64_t c0 = (w0 + w) * 64;
      if (n - c0 < 64) x &= (1ull << (n - c0)) - 1ull;  // padding columns stay zero
      if (accumulate) x = (SEMI == GF2) ? (x ^ dst[w]) : (x | dst[w]);
      dst[w] = x;
    }
  }
}

}  // namespace

hipError_t launch_leaf_valu(int semiring, const LeafBatch& p, int /*tile*/, hipStream_t s) {
  if (p.m <= 0 || p.n <= 0 || p.batch <= 0) return hipSuccess;
  const int64_t tiles_m = (p.m + TM - 1) / TM;
  const int64_t tiles_n = (p.n + TN - 1) / TN;
  const int64_t blocks = tiles_m * tiles_n * p.batch;
  if (!grid_fits(blocks, 256)) return kGridTooLarge;
  if (semiring == GF2)
    hipLaunchKernelGGL(leaf_valu_kernel<GF2>, dim3((unsigned)blocks), dim3(256), 0, s, p,
                       tiles_m, tiles_n);
  else
    hipLaunchKernelGGL(leaf_valu_kernel<BOOLEAN>, dim3((unsigned)blocks), dim3(256), 0, s, p,
                       tiles_m, tiles_n);
  return hipGetLastError();
}

hipError_t launch_leaf_valu_outer(int semiring, const uint64_t* A, int64_t lda,
                                  const uint64_t* B, int64_t ldb, uint64_t* C, int64_t ldc,
                                  int64_t m, int64_t k, int64_t n, int accumulate,
                                  hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int64_t tiles_m = (m + OTM - 1) / OTM;
  const int64_t tiles_n = (((n + 63) / 64) * 64 + OTN - 1) / OTN;
  const int64_t blocks = tiles_m * tiles_n;
  if (!grid_fits(blocks, 256)) return kGridTooLarge;
  const uint32_t* B32 = reinterpret_cast<const uint32_t*>(B);
  const bool full = ((n + 63) / 64) * 2 >= OCW;
  const dim3 g((unsigned)blocks), b(256);
  if (semiring == GF2) {
    if (full)
      hipLaunchKernelGGL((leaf_valu_outer_kernel<GF2, true>), g, b, 0, s, A, lda, B32, 2 * ldb,
                         C, ldc, m, k, n, tiles_m, tiles_n, accumulate);
    else
      hipLaunchKernelGGL((leaf_valu_outer_kernel<GF2, false>), g, b, 0, s, A, lda, B32, 2 * ldb,
                         C, ldc, m, k, n, tiles_m, tiles_n, accumulate);
  } else {
    if (full)
      hipLaunchKernelGGL((leaf_valu_outer_kernel<BOOLEAN, true>), g, b, 0, s, A, lda, B32,
                         2 * ldb, C, ldc, m, k, n, tiles_m, tiles_n, accumulate);
    else
      hipLaunchKernelGGL((leaf_valu_outer_kernel<BOOLEAN, false>), g, b, 0, s, A, lda, B32,
                         2 * ldb, C, ldc, m, k, n, tiles_m, tiles_n, accumulate);
  }
  return hipGetLastError();
}

}  // namespace bmm
