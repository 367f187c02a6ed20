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
// (Boolean), 32 columns per v_bitop3_b32 with the bit as a sign-extended mask
// (v_bfe_i32).  The accumulators are the result bits themselves: no reduction.
//
// A wave owns 256 rows (four per lane) and 512 columns (16 dwords); a workgroup 2 x 2
// waves, 512 x 1024.  Row j's 16 words are the same for all lanes of a wave: they are read
// from LDS at one address for the whole wave (a broadcast) one step ahead, and each word
// feeds four folds, one per row of the lane: a lane receives one byte per fold, as in the
// dot-product form, but the wave's lanes all read the same address.  Stages of OST rows of B (the
// workgroup's 1024 columns, 8 KB) are double buffered in LDS and loaded one stage ahead
// into registers; the k-dwords of A are loaded a k-dword ahead.  128 registers leave four
// waves per SIMD, which the VALU needs to pair instructions: with eight rows per lane (two
// waves per SIMD) it issued 1.14 instead of 1.39 instructions per SIMD quad-cycle.
constexpr int OROWS = 4;             // rows per lane
constexpr int OCW = 16;              // C dwords (32 columns each) per wave
constexpr int OST = 64;              // rows of B per LDS stage
constexpr int OWG_CW = 2 * OCW;      // C dwords per workgroup row (two waves across)
constexpr int OTM = 2 * 64 * OROWS;  // rows per workgroup
constexpr int OTN = 32 * OWG_CW;     // columns per workgroup

template <int SEMI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void
leaf_valu_outer_kernel(const uint64_t* __restrict__ A, int64_t lda,
                       const uint32_t* __restrict__ B, int64_t ldb32, uint64_t* __restrict__ C,
                       int64_t ldc, int64_t m, int64_t k, int64_t n, int64_t tiles_m,
                       int64_t tiles_n, int accumulate) {
  // two spare rows per stage: the reads of the next two rows run ahead unconditionally
  __shared__ __attribute__((aligned(16))) uint32_t sB[2][(OST + 2) * OWG_CW];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wy = wave >> 1, wx = wave & 1;
  const TileCoord c = xcd_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n);
  const int64_t n32 = ((n + 63) >> 6) * 2;      // dwords per row of B and C (whole words)
  const int64_t wg32 = c.tn * OWG_CW;           // first C dword of the workgroup's columns
  const int64_t col32 = wg32 + wx * OCW;        // first C dword of the wave's columns
  const int64_t row0 = c.tm * OTM + wy * (64 * OROWS);
  // the lane's rows are row0 + lane + 64 r: one pointer and a uniform stride; rows past m
  // load nothing (their bits stay zero)
  const int64_t lda32 = 2 * lda, astride = 64 * lda32;
  const uint32_t* arow0 = reinterpret_cast<const uint32_t*>(A) + (row0 + lane) * lda32;
  int nrows = 0;  // how many of the lane's rows lie in A
#pragma unroll
  for (int r = 0; r < OROWS; ++r) nrows += row0 + 64 * r + lane < m;
  auto load_a = [&](int64_t jw, uint32_t (&dst)[OROWS]) {
#pragma unroll
    for (int r = 0; r < OROWS; ++r) dst[r] = r < nrows ? arow0[r * astride + jw] : 0u;
  };
  // stage loads: OST rows x 32 dwords = 2048 dwords per stage, 8 per thread: thread t
  // carries row t / 4, dwords 8 (t mod 4) .. + 7
  const int srow = tid >> 2, sd = (tid & 3) * 8;
  const int64_t sc = wg32 + sd;  // first B dword this thread stages
  auto stage_load = [&](int64_t j0, uint4 (&v)[2]) {
    const int64_t j = j0 + srow;
    if (j < k && sc + 8 <= n32) {
      const uint4* src = reinterpret_cast<const uint4*>(B + j * ldb32 + sc);
      v[0] = src[0];
      v[1] = src[1];
    } else {
      uint32_t t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = (j < k && sc + q < n32) ? B[j * ldb32 + sc + q] : 0u;
      v[0] = make_uint4(t[0], t[1], t[2], t[3]);
      v[1] = make_uint4(t[4], t[5], t[6], t[7]);
    }
  };
  auto stage_store = [&](int buf, const uint4 (&v)[2]) {
    uint4* dst = reinterpret_cast<uint4*>(&sB[buf][srow * OWG_CW + sd]);
    dst[0] = v[0];
    dst[1] = v[1];
  };
  uint32_t acc[OROWS][OCW];
#pragma unroll
  for (int r = 0; r < OROWS; ++r)
#pragma unroll
    for (int q = 0; q < OCW; ++q) acc[r][q] = 0u;
  const int64_t k32 = (k + 31) >> 5;
  uint32_t a[OROWS], an[OROWS];
#pragma unroll
  for (int r = 0; r < OROWS; ++r) an[r] = 0u;
  if (k > 0) load_a(0, an);
  uint4 sv[2];
  stage_load(0, sv);
  stage_store(0, sv);
  const int64_t stages = (k + OST - 1) / OST;
  if (stages > 1) stage_load(OST, sv);
  __syncthreads();
  // one step: the row masks of bit j of A, and the folds of row j of B (bw, 16 words)
  auto step = [&](int jb, const uint4 (&bv)[4]) {
    uint32_t msk[OROWS];
#pragma unroll
    for (int r = 0; r < OROWS; ++r) msk[r] = (uint32_t)__builtin_amdgcn_sbfe((int)a[r], jb, 1);
    const uint32_t bw[OCW] = {bv[0].x, bv[0].y, bv[0].z, bv[0].w, bv[1].x, bv[1].y,
                              bv[1].z, bv[1].w, bv[2].x, bv[2].y, bv[2].z, bv[2].w,
                              bv[3].x, bv[3].y, bv[3].z, bv[3].w};
#pragma unroll
    for (int q = 0; q < OCW; ++q)
#pragma unroll
      for (int r = 0; r < OROWS; ++r) acc[r][q] = fold<SEMI>(msk[r], bw[q], acc[r][q]);
  };
  auto read_row = [&](const uint32_t* rowp, uint4 (&bv)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) bv[q] = reinterpret_cast<const uint4*>(rowp)[q];
  };
  for (int64_t st = 0; st < stages; ++st) {
    const int cur = (int)(st & 1);
    const uint32_t* base = &sB[cur][wx * OCW];
    const int64_t j0 = st * OST;
    const int nsteps = (int)(k - j0 < OST ? k - j0 : OST);
    // two steps per iteration with two row buffers (no copies); rows j + 1 and j + 2 are
    // requested before row j's and row j + 1's folds (the spare rows absorb the overrun)
    uint4 b0[4], b1[4];
    read_row(base, b0);
    for (int jj = 0; jj < nsteps; jj += 2) {
      const int64_t j = j0 + jj;
      if ((j & 31) == 0) {  // uniform: this k-dword of A, and the next one requested
#pragma unroll
        for (int r = 0; r < OROWS; ++r) a[r] = an[r];
        load_a((j >> 5) + 1 < k32 ? (j >> 5) + 1 : k32 - 1, an);
      }
      read_row(base + (jj + 1) * OWG_CW, b1);
      step((int)(j & 31), b0);
      read_row(base + (jj + 2) * OWG_CW, b0);
      step((int)((j + 1) & 31), b1);  // row nsteps of a ragged last stage is zero
    }
    if (st + 1 < stages) {
      stage_store(cur ^ 1, sv);
      if (st + 2 < stages) stage_load((st + 2) * OST, sv);
    }
    __syncthreads();
  }
  // the accumulators are C's dwords: two make a 64-bit word of the row
  const int64_t nw = n32 >> 1, w0 = col32 >> 1;
#pragma unroll
  for (int r = 0; r < OROWS; ++r) {
    if (r >= nrows) continue;
    uint64_t* dst = C + (row0 + 64 * r + lane) * ldc + w0;
#pragma unroll
    for (int w = 0; w < OCW / 2; ++w) {
      if (w0 + w >= nw) break;  // uniform
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
  const dim3 g((unsigned)blocks), b(256);
  if (semiring == GF2)
    hipLaunchKernelGGL(leaf_valu_outer_kernel<GF2>, g, b, 0, s, A, lda, B32, 2 * ldb, C, ldc,
                       m, k, n, tiles_m, tiles_n, accumulate);
  else
    hipLaunchKernelGGL(leaf_valu_outer_kernel<BOOLEAN>, g, b, 0, s, A, lda, B32, 2 * ldb, C,
                       ldc, m, k, n, tiles_m, tiles_n, accumulate);
  return hipGetLastError();
}

}  // namespace bmm
