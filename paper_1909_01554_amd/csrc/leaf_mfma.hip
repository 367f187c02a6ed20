// Cubic leaf product on the int8 matrix cores of gfx950.
//
// The cubic product C[i][k] = SUM_j A[i][j] B[j][k] (GF(2): XOR, Boolean: OR)
// is an integer dot product reduced at the end: the int32 count of j with
// A[i][j] = B[j][k] = 1 gives the GF(2) bit as its parity and the Boolean bit
// as (count > 0).  Counts stay exact because k < 2^31.
//
// Each wave owns a TM x TN tile of C (TM = 32*RA, TN = 32*RB) and issues
// v_mfma_i32_32x32x32_i8 on RA x RB accumulator blocks held in registers.
// Operands never touch HBM as bytes: every lane reads 64-bit words of packed
// bits straight from its row of A (or of B transposed) and expands them in
// registers.  The order of k inside a dot product is free as long as A and B
// use the same one, so a 32-bit half x of a word yields the eight dwords
// (x >> d) & 0x01010101 (d = 0..7): byte e of dword d is bit 8e + d of x, 0 or
// 1 (for one side of the tile both halves at once, from a 64-bit shift).  GF(2) parity alone would only need the low bit of each byte, but
// operand bytes holding the other random bits too make the matrix cores
// switch far more on dense inputs and run at a lower rate, so both semirings
// feed exact 0/1 bytes.
//
// The result bits go back to packed rows with wave ballots: accumulator
// register v of a 32x32 block holds row 8*(v/4) + (v%4) in lanes 0..31 and
// row 8*(v/4) + 4 + (v%4) in lanes 32..63, one column per lane, so one ballot
// yields two 32-bit row words.
#include "mfma_tile.h"

namespace bmm {
namespace {

// Each workgroup owns 2 x 2 wave tiles; workgroups are ordered for L2 reuse per XCD.
template <int SEMI, int RA, int RB, int KV, int FMT, int NB = 2, int STEPS = 0, bool WIDE = true,
          bool SHORT = false, bool BOTH = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void leaf_mfma_kernel(
    LeafBatch p, int64_t tiles_m, int64_t tiles_n) {
  const int64_t grid_m = (tiles_m + 1) >> 1, grid_n = (tiles_n + 1) >> 1;
  const TileCoord c = xcd_tile(blockIdx.x, gridDim.x, grid_m, grid_n);
  // The wide tiles take the wave index as a uniform value (their tile coordinates then
  // live in scalar registers, which frees the vector registers the long-k loop spilled);
  // the narrower tiles keep the per-lane form, measured faster on the recursion's leaves.
  const int w = RB == 4 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : threadIdx.x >> 6;
  const int64_t tm = 2 * c.tm + (w >> 1);
  const int64_t tn = 2 * c.tn + (w & 1);
  if (c.b >= p.batch || tm >= tiles_m || tn >= tiles_n) return;  // uniform per wave
  const int64_t b = c.b;
  mfma::tile<SEMI, RA, RB, KV, FMT, NB, STEPS, WIDE, SHORT, BOTH>(p.A + b * p.strideA, p.lda, p.BT + b * p.strideB, p.ldbt,
                                    p.C + b * p.strideC, p.ldc, p.m, p.k, p.n, tm, tn,
                                    p.accumulate);
}

// The LDS-staged 2 x 2 wave item of mfma::lds_item, one per workgroup (tile 8): the
// same 256 x 128 workgroup tiles, in the same XCD-aware order, with the operand rows of
// each stage loaded once into LDS and shared by the four waves.
template <int SEMI, int FMT, bool WIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void leaf_mfma_lds4_kernel(
    LeafBatch p, int64_t tiles_m, int64_t tiles_n, int aligned) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[mfma::kLdsItemBytes];
  const int64_t grid_m = (tiles_m + 1) >> 1, grid_n = (tiles_n + 1) >> 1;
  const TileCoord c = xcd_tile(blockIdx.x, gridDim.x, grid_m, grid_n);
  if (c.b >= p.batch) return;  // uniform per workgroup
  mfma::LdsStage stage;
  mfma::lds_item<SEMI, FMT, WIDE>(p.A + c.b * p.strideA, p.lda, p.BT + c.b * p.strideB, p.ldbt,
                                  p.C + c.b * p.strideC, p.ldc, p.m, p.k, p.n, c.tm, c.tn,
                                  tiles_m, tiles_n, aligned != 0, p.accumulate, SEMI,
                                  __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), smem, stage);
}

template <int SEMI, int FMT>
hipError_t launch_lds4(const LeafBatch& p, hipStream_t s) {
  const int64_t tiles_m = (p.m + 127) / 128;
  const int64_t tiles_n = (((p.n + 63) / 64) * 64 + 63) / 64;
  const int64_t blocks = ((tiles_m + 1) / 2) * ((tiles_n + 1) / 2) * p.batch;
  if (blocks == 0) return hipSuccess;
  if (!grid_fits(blocks, 256)) return kGridTooLarge;
  const int aligned = ((reinterpret_cast<uintptr_t>(p.A) | reinterpret_cast<uintptr_t>(p.BT)) & 15) == 0 &&
                      ((p.lda | p.ldbt | p.strideA | p.strideB) & 1) == 0;
  hipLaunchKernelGGL((leaf_mfma_lds4_kernel<SEMI, FMT, FMT == mfma::FMT_I8>), dim3((unsigned)blocks),
                     dim3(256), 0, s, p, tiles_m, tiles_n, aligned);
  return hipGetLastError();
}

// DEEP: int8 leaves of the recursion's lengths (k = 2048 or 4096 bits, 16-byte
// aligned) run a fully unrolled load pipeline with two register buffers and both
// operand sides expanded by 64-bit shifts: 18% fewer VALU instructions than the 32-bit
// form, 13% fewer than widening the shorter side alone (with three buffers, which then
// measured 1-1.5% slower at k = 2048 and 3.4% slower at k = 4096; both sides wide with
// three buffers spill).  CHUNKED: aligned int8 leaves
// run the 2-deep pipeline as a loop over fully unrolled chunks of 12 steps, which
// leaves the compiler's conservative wait for outstanding loads at the loop's
// back edge once per chunk instead of once per step pair.  All else takes the
// 2-deep loop.
template <int SEMI, int RA, int RB, int FMT, bool DEEP = false, bool CHUNKED = false>
hipError_t launch_t(const LeafBatch& p, hipStream_t s) {
  constexpr int TM = 32 * RA, TN = 32 * RB;
  const int64_t tiles_m = (p.m + TM - 1) / TM;
  // cover whole 64-bit output words, so padding dwords are written (as zero)
  const int64_t tiles_n = (((p.n + 63) / 64) * 64 + TN - 1) / TN;
  const int64_t blocks = ((tiles_m + 1) / 2) * ((tiles_n + 1) / 2) * p.batch;
  if (blocks == 0) return hipSuccess;
  if (!grid_fits(blocks, 256)) return kGridTooLarge;
  const bool aligned16 = ((reinterpret_cast<uintptr_t>(p.A) | reinterpret_cast<uintptr_t>(p.BT)) & 15) == 0 &&
                         ((p.lda | p.ldbt | p.strideA | p.strideB) & 1) == 0;
  const dim3 g((unsigned)blocks), b(256);
  // the unrolled pipelines are built for the int8 format only: with fp4 operands they
  // spill 1.7-3.9 KB per lane and ran the n = 2^18 fp4 recursion 5.6x slower
  if constexpr (DEEP && FMT == mfma::FMT_I8) {
    if (aligned16 && p.k == 2048) {
      hipLaunchKernelGGL((leaf_mfma_kernel<SEMI, RA, RB, 2, FMT, 2, 8, true, false, true>), g, b, 0, s,
                         p, tiles_m, tiles_n);
      return hipGetLastError();
    }
    if (aligned16 && p.k == 4096) {
      hipLaunchKernelGGL((leaf_mfma_kernel<SEMI, RA, RB, 2, FMT, 2, 16, true, false, true>), g, b, 0,
                         s, p, tiles_m, tiles_n);
      return hipGetLastError();
    }
  }
  if constexpr (CHUNKED && FMT == mfma::FMT_I8) {
    if (aligned16) {
      hipLaunchKernelGGL((leaf_mfma_kernel<SEMI, RA, RB, 2, FMT, 2, -12>), g, b, 0, s, p,
                         tiles_m, tiles_n);
      return hipGetLastError();
    }
  }
  // int8: the 64-bit expansion; the 128 x 64 tile widens its shorter side (84 bytes of
  // spills per lane with the longer side, 28 with the shorter; the n = 65536 recursion at
  // depth 6, 1024^3 leaves, 4.5% faster).  fp4: the 32-bit form (the wide one spills).
  constexpr bool kWideForm = FMT == mfma::FMT_I8;
  constexpr bool kShort = RA > RB;
  if (aligned16)
    hipLaunchKernelGGL((leaf_mfma_kernel<SEMI, RA, RB, 2, FMT, 2, 0, kWideForm, kShort>),
                       dim3((unsigned)blocks), dim3(256), 0, s, p, tiles_m, tiles_n);
  else
    hipLaunchKernelGGL((leaf_mfma_kernel<SEMI, RA, RB, 1, FMT, 2, 0, kWideForm, kShort>),
                       dim3((unsigned)blocks), dim3(256), 0, s, p, tiles_m, tiles_n);
  return hipGetLastError();
}

template <int SEMI, int FMT>
hipError_t launch_semi(const LeafBatch& p, int tile, hipStream_t s) {
  switch (tile) {
    case MFMA_LDS_256x256: return launch_leaf_mfma_lds(SEMI, FMT, p, s);
    case MFMA_LDS4_256x128: return launch_lds4<SEMI, FMT>(p, s);
    case MFMA_DEEP_128x64: return launch_t<SEMI, 4, 2, FMT, true>(p, s);
    case MFMA_CHUNK_64x128: return launch_t<SEMI, 2, 4, FMT, false, true>(p, s);
    case MFMA_64x64: return launch_t<SEMI, 2, 2, FMT>(p, s);
    case MFMA_64x128: return launch_t<SEMI, 2, 4, FMT>(p, s);
    case MFMA_64x32: return launch_t<SEMI, 2, 1, FMT>(p, s);
    default: return launch_t<SEMI, 4, 2, FMT>(p, s);
  }
}

}  // namespace

int leaf_mfma_tile_rows(int tile) {
  switch (tile) {
    case MFMA_64x64: return 64;
    case MFMA_64x128: return 64;
    case MFMA_CHUNK_64x128: return 64;
    case MFMA_64x32: return 64;
    case MFMA_LDS_256x256: return 256;
    case MFMA_LDS4_256x128: return 256;
    default: return 128;
  }
}

int leaf_mfma_tile_cols(int tile) {
  switch (tile) {
    case MFMA_64x64: return 64;
    case MFMA_64x128: return 128;
    case MFMA_CHUNK_64x128: return 128;
    case MFMA_64x32: return 32;
    case MFMA_LDS_256x256: return 256;
    case MFMA_LDS4_256x128: return 128;
    default: return 64;
  }
}

hipError_t launch_leaf_mfma(int semiring, const LeafBatch& p, int tile, hipStream_t s) {
  if (p.m <= 0 || p.n <= 0 || p.batch <= 0) return hipSuccess;
  return semiring == GF2 ? launch_semi<GF2, mfma::FMT_I8>(p, tile, s)
                         : launch_semi<BOOLEAN, mfma::FMT_I8>(p, tile, s);
}

hipError_t launch_leaf_mfma_f4(int semiring, const LeafBatch& p, int tile, hipStream_t s) {
  if (p.m <= 0 || p.n <= 0 || p.batch <= 0) return hipSuccess;
  return semiring == GF2 ? launch_semi<GF2, mfma::FMT_F4>(p, tile, s)
                         : launch_semi<BOOLEAN, mfma::FMT_F4>(p, tile, s);
}

}  // namespace bmm
