// Internal interface between the C-ABI layer (api.cpp) and the HIP kernels.
//
// Layout everywhere: packed row-major uint64, bit j of a row at bit j % 64 of
// word j / 64.  "BT" operands are the right-hand operand stored transposed
// (one row per column of B, k bits long), which is what both leaf kernels read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmm {

enum Semiring { GF2 = 0, BOOLEAN = 1 };

// Record a message for bmm_last_error() (thread-local) and return `code`.
int set_error(int code, const char* fmt, ...);

// Every device allocation the library makes goes through here (hipMalloc, or a
// forced failure while bmm_debug_fail_allocations is armed).
hipError_t dev_malloc(void** p, size_t bytes);

// A dispatch covers fewer than 2^32 work-items (the grid size of an AQL packet is
// 32 bits).  Launchers whose grid would reach that return kGridTooLarge without
// launching; the entry points report it as BMM_E_UNSUPPORTED.
constexpr hipError_t kGridTooLarge = hipErrorInvalidConfiguration;
inline bool grid_fits(int64_t blocks, int64_t threads) {
  return blocks >= 0 && blocks * threads < ((int64_t)1 << 32) && blocks < ((int64_t)1 << 31);
}

// A batch of independent leaf products C_b (m x n) = A_b (m x k) * B_b (k x n),
// with B_b given transposed as BT_b (n x k).  Operand b starts at base + b*stride
// (strides in words).  accumulate: C ^= AB (GF(2)) or C |= AB (Boolean).
struct LeafBatch {
  const uint64_t* A;
  int64_t lda, strideA;
  const uint64_t* BT;
  int64_t ldbt, strideB;
  uint64_t* C;
  int64_t ldc, strideC;
  int64_t m, k, n, batch;
  int accumulate;
};

// XCD-aware order of workgroups over a batch of 2-D tile grids.  The hardware
// hands workgroup g to XCD g % 8 (round robin); remapping g so that each XCD
// owns one contiguous range of logical workgroups, walked in groups of
// kGroupRows tile rows, keeps the operand panels of the tiles that run
// together on one XCD inside that XCD's L2.  Any remapping is a bijection, so
// correctness never depends on the dispatch order.
constexpr int kXcds = 8;
constexpr int kGroupRows = 8;

struct TileCoord {
  int64_t b, tm, tn;
};

// Banded order of a grid_m x grid_n tile grid: bands of kGroupRows tile rows,
// each walked column by column, so consecutive tiles share operand panels.
__device__ __forceinline__ void band_coord(int64_t r, int64_t grid_m, int64_t grid_n,
                                           int64_t& tm, int64_t& tn) {
  const int64_t band = (int64_t)kGroupRows * grid_n;
  const int64_t first = (r / band) * kGroupRows;
  const int64_t rows = grid_m - first < kGroupRows ? grid_m - first : kGroupRows;
  const int64_t q = r - (r / band) * band;
  tm = first + q % rows;
  tn = q / rows;
}

__device__ __forceinline__ TileCoord xcd_tile(int64_t g, int64_t total, int64_t grid_m,
                                              int64_t grid_n) {
  const int64_t x = g % kXcds, j = g / kXcds;
  const int64_t per = total / kXcds, rem = total % kXcds;
  const int64_t t = x * per + (x < rem ? x : rem) + j;
  const int64_t per_item = grid_m * grid_n;
  TileCoord c;
  c.b = t / per_item;
  band_coord(t - c.b * per_item, grid_m, grid_n, c.tm, c.tn);
  return c;
}

// MFMA leaf variants (rows x cols of C per wave).
enum MfmaTile { MFMA_128x64 = 0, MFMA_64x64 = 1, MFMA_64x128 = 2, MFMA_64x32 = 3,
                MFMA_LDS_256x256 = 4,
                MFMA_DEEP_128x64 = 5,  // 128 x 64, 3-deep unrolled pipeline for k = 2048, 4096
                MFMA_CHUNK_64x128 = 6,  // 64 x 128, 2-deep pipeline in unrolled 12-step chunks
                MFMA_LDS4_256x128 = 7,  // 2 x 2 waves of 128 x 64, operand rows shared in LDS
                MFMA_NUM_TILES };

hipError_t launch_leaf_mfma(int semiring, const LeafBatch& p, int tile, hipStream_t s);
// The same tiles on E2M1 (fp4) operands with exact fp32 sums; requires k < 2^24.
hipError_t launch_leaf_mfma_f4(int semiring, const LeafBatch& p, int tile, hipStream_t s);
// The 8-wave workgroup variant that shares operand panels through LDS (fmt 0: int8, 1: fp4).
hipError_t launch_leaf_mfma_lds(int semiring, int fmt, const LeafBatch& p, hipStream_t s);
hipError_t launch_leaf_valu(int semiring, const LeafBatch& p, int tile, hipStream_t s);
// The VALU leaf in outer-product form (tile 2): B row-major (k x n, pitch ldb words), one
// product; k = 0 leaves C zero (or unchanged when accumulating).
hipError_t launch_leaf_valu_outer(int semiring, const uint64_t* A, int64_t lda,
                                  const uint64_t* B, int64_t ldb, uint64_t* C, int64_t ldc,
                                  int64_t m, int64_t k, int64_t n, int accumulate,
                                  hipStream_t s);
// The last recursion level shifted into the int8 leaf (leaf_shift.hip): for every
// parent p, the seven child products of its quadrants (alpha, beta of `scheme`) are
// formed, multiplied and combined by gamma into the parent's result quadrants.
// m, k, n: a CHILD product's sizes (parents are 2m x 2k and 2n x 2k transposed,
// results 2m x 2n); parent p at base + p * stride (words).  accumulate: Q ^= result.
struct ShiftBatch {
  const uint64_t* T;
  int64_t ldt, strideT;
  const uint64_t* S;
  int64_t lds, strideS;
  uint64_t* Q;
  int64_t ldq, strideQ;
  int64_t m, k, n, parents;
  int accumulate;
};
// Schemes with alpha/beta weights <= 2 (self-inverse, chaining), k = 2048 or 4096
// bits, n a multiple of 64.
bool leaf_shift_supported(int scheme, int64_t m, int64_t k, int64_t n);
// The kernel addresses a parent's rows with 32-bit byte offsets (2 * rows * ld < 2^29).
bool leaf_shift_fits(int64_t rows, int64_t ld);
// kv = 2: 16-byte operand loads where operands and pitches allow, else 8-byte loads.
hipError_t launch_leaf_shift(int scheme, const ShiftBatch& p, int kv, hipStream_t s);
int leaf_mfma_tile_rows(int tile);
int leaf_mfma_tile_cols(int tile);

// dst (cols x rows bits) = transpose of src (rows x cols bits), batched.
hipError_t launch_transpose(const uint64_t* src, int64_t lds, int64_t strideS,
                            uint64_t* dst, int64_t ldd, int64_t strideD,
                            int64_t rows, int64_t cols, int64_t batch, hipStream_t s);

// 2x2 basis change of a scheme (bmm_scheme) applied at the top `depth` levels
// of every matrix of a batch (rows and row words divisible by 2^depth), in
// place.  inverse = 0: the forward change (both operands; transposed = 1 for
// an operand stored transposed), 1: the inverse change (result).  The
// Winograd scheme has none (no-op).
hipError_t launch_basis(uint64_t* X, int64_t ld, int64_t stride, int64_t rows,
                        int64_t row_words, int64_t batch, int depth, int inverse,
                        hipStream_t s, int scheme = 0, int transposed = 0);

// One recursion level of a scheme (bmm_scheme).  Parent p of a batch (rows x
// words, pitch ldp, stride strideP) expands into 7 children stored
// contiguously: child (p, h) is
// matrix 7p + h of `dst`, each (rows/2) x (words/2) with pitch words/2.
// side 0: left operand (alpha), 1: right operand stored transposed (beta with
// the 01 and 10 quadrants swapped).
hipError_t launch_expand(int side, const uint64_t* src, int64_t ldp, int64_t strideP,
                         uint64_t* dst, int64_t rows, int64_t words, int64_t parents,
                         hipStream_t s, int scheme = 0);
// Two recursion levels at once (49 grandchildren per parent, index 49p + 7h1 + h2).
hipError_t launch_expand2(int side, const uint64_t* src, int64_t ldp, int64_t strideP,
                          uint64_t* dst, int64_t rows, int64_t words, int64_t parents,
                          hipStream_t s, int scheme = 0);
// Inverse of the above for the products: 7 children (compact, (rows/2) x
// (words/2)) of parent p combine by gamma into the parent's 4 quadrants
// (accumulate = 1: XORed into the parent instead of overwriting it).
hipError_t launch_compress(const uint64_t* src, uint64_t* dst, int64_t ldp, int64_t strideP,
                           int64_t rows, int64_t words, int64_t parents, hipStream_t s,
                           int accumulate = 0, int scheme = 0);
hipError_t launch_compress2(const uint64_t* src, uint64_t* dst, int64_t ldp,
                            int64_t strideP, int64_t rows, int64_t words, int64_t parents,
                            hipStream_t s, int accumulate = 0, int scheme = 0);

// One child at a time (the lean depth-first levels): child h of a parent (rows x words,
// pitch ldp) of side 0 (left) or 1 (right, stored transposed) into dst (pitch ldd); and
// product h (pitch lds) into the parent's result quadrants by gamma (accumulate = 1: every
// contribution is XORed in; else each quadrant's first product overwrites it).
uint32_t child_mask(int scheme, int side, int h);
hipError_t launch_child(int scheme, int side, int h, const uint64_t* src, int64_t ldp,
                        uint64_t* dst, int64_t ldd, int64_t rows, int64_t words, hipStream_t s);
hipError_t launch_gamma(int scheme, int h, const uint64_t* src, int64_t lds, uint64_t* dst,
                        int64_t ldp, int64_t rows, int64_t words, int accumulate,
                        hipStream_t s);

// Copy a batch of rows x words matrices (used to stage operands).
hipError_t launch_copy(const uint64_t* src, int64_t lds, uint64_t* dst, int64_t ldd,
                       int64_t rows, int64_t words, hipStream_t s);
// dst ^= src for rows x words matrices.
hipError_t launch_xor(const uint64_t* src, int64_t lds, uint64_t* dst, int64_t ldd, int64_t rows,
                      int64_t words, hipStream_t s);
// Fill `words` contiguous words with dense pseudo-random bits (autotuner buffers).
hipError_t launch_random(uint64_t* dst, int64_t words, uint64_t seed, hipStream_t s);
// Zero a rows x words matrix (a fill kernel, safe under graph capture).
hipError_t launch_zero(uint64_t* dst, int64_t ld, int64_t rows, int64_t words, hipStream_t s);

// VALU issue-rate calibration (calib.hip): `blocks` 256-thread workgroups fold
// calib_chains() independent chains with one v_bitop3_b32 each per round; every wave
// stores (core clock start, end, constant clock start, end) at stamps[4 * wave].
int calib_chains();
hipError_t launch_valu_rate(uint32_t seed, int64_t rounds, int blocks, uint32_t* sink,
                            long long* stamps, hipStream_t s);

// Persistent batched leaf over a device-resident problem table.  A work item is
// one workgroup's 2 x 2 wave tiles of one problem; a problem's items, in banded
// order, are split into contiguous ranges over kXcds queues (one per XCD), and
// a queue's items are listed as segments (problem, first item) at increasing
// queue positions.
struct BatchedDesc {
  const uint64_t* A;
  const uint64_t* BT;
  uint64_t* C;
  int64_t lda, ldbt, ldc;
  int64_t m, k, n;
  int32_t semiring;
  int32_t aligned;           // A, B^T 16-byte aligned with even pitches: 16-byte loads
  int32_t tiles_m, tiles_n;  // wave tiles (tiles_n covers C's padding words)
  int32_t items_m, items_n;  // work items (2 x 2 wave tiles)
};
struct BatchedSeg {
  uint32_t begin;    // queue position of the segment's first item
  uint32_t problem;  // index into the problem table
  uint32_t item_lo;  // the problem's item at that position
  uint32_t pad;
};
struct BatchedQueues {
  uint32_t seg_off[kXcds], seg_count[kXcds], items[kXcds];
};
constexpr int kBatchedCounterStride = 64;  // uint32s between queue counters (256 bytes)
// tile 1: 128 x 64 per wave, 2: 64 x 64, 3: 64 x 128; fmt: mfma::MfmaFormat (0 int8, 1 E2M1).
// counters: kXcds * kBatchedCounterStride uint32s, zeroed by the launch itself.
hipError_t launch_batched_persistent(const BatchedDesc* descs, const BatchedSeg* segs,
                                     const BatchedQueues& queues, unsigned int* counters,
                                     int grid, int tile, int fmt, hipStream_t s);
// Generation of the batched tuning records (changes whenever one is set or loaded).
uint64_t batched_tune_generation();
// Release bmm_batched's library-owned plans, graphs and staging buffers.
void batched_cache_clear();
int batched_tile_rows(int tile);
int batched_tile_cols(int tile);

// Batched-plan choices recorded by the autotuner (leaf kind, tile, persistent
// workgroups per CU), keyed by the problem count and the total work rounded to a
// power of two (kept with the other autotune tables).
bool batched_tuned(int64_t count, double ops, int* leaf, int* tile, int* wg_per_cu);
void batched_tune_set(int64_t count, double ops, int leaf, int tile, int wg_per_cu);
// Per size class of k (0: k < 1024, 1: < 4096, 2: else) within such plans: the leaf kind
// (VALU included) and tile the autotuner chose where a mix beat one choice for all.
bool batched_class_tuned(int64_t count, double ops, int kclass, int* leaf, int* tile);
void batched_class_set(int64_t count, double ops, int kclass, int leaf, int tile);
void batched_class_clear(int64_t count, double ops);

}  // namespace bmm

#include "../../include/bmm.h"

namespace bmm {

// Inverse of the result's basis change of a scheme (standard -> alternative basis).
// Leaf kind and tile of a product (options, then the autotune table, then the
// default rule), as every entry point chooses them.
void choose_leaf(int semiring, int64_t m, int64_t k, int64_t n, int64_t batch,
                 const bmm_options& o, int* leaf, int* tile);
// The cubic product behind bmm_gf2 / bmm_boolean.  B^T goes to the library's cached
// scratch, or, when caller_bt is given, to that fixed buffer (get() returns its
// device address, set up on first use): requests whose B^T does not fit are
// refused with BMM_E_UNSUPPORTED before any device work.
struct BtScratch {
  size_t bytes;
  int (*get)(void** out);
};
int cubic_product(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                  uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n,
                  const bmm_options* opt, void* stream, const BtScratch* caller_bt);
hipError_t to_alt_basis(uint64_t* C, int64_t ldc, int64_t rows, int64_t words, int depth,
                        int scheme, hipStream_t s);

// The recursion's core on operands already in the alternative basis (A, and B
// given transposed), for callers that stage their own operands (the
// out-of-core pipeline).  depth = -1 picks it as the public product does;
// strassen_alt_plan reports the workspace and the depth chosen.  accumulate = 1
// XORs the (alternative-basis) result into C.  Both return a bmm status.
int strassen_alt_plan(int64_t m, int64_t k, int64_t n, int depth, const bmm_options& o,
                      size_t* bytes, int* depth_out);
int strassen_alt(const uint64_t* Ahat, int64_t lda, const uint64_t* BThat, int64_t ldbt,
                 uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n, int depth,
                 void* ws, size_t bytes, const bmm_options& o, int accumulate, hipStream_t s);

}  // namespace bmm
