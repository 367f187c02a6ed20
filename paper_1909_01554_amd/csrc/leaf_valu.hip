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

}  // namespace bmm
