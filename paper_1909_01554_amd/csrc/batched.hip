// Persistent batched leaf: many independent products of uneven sizes in one
// launch.  A work item is a 2 x 2 group of wave tiles of one problem (128 x 64,
// 64 x 64 or 64 x 128 per wave; int8 or E2M1 operands, as the plan chose), so
// the four waves of a workgroup read shared operand rows together.  Items sit
// in kXcds queues, one per XCD: every problem's items, in banded order, are
// split into contiguous ranges over the queues, so the workgroups of one XCD
// walk neighbouring items and share that XCD's L2.  A workgroup takes items
// from the queue of its own XCD (the hardware hands workgroup g to XCD g % 8)
// and, once that queue is empty, from the others in turn; it exits when all
// are empty.  Which XCD runs an item never affects the result.
//
// Wave 0 of a workgroup pops items: lane 0 takes a queue position with one
// atomic add (issued before the current item's tile, so its latency hides
// behind the operand loads), then the wave finds the position's segment with a
// 64-way search over the queue's segment table and hands (problem, item) to the
// other waves through LDS.  A one-workgroup kernel zeroes the queue counters
// before each launch, so the pair can be captured into a HIP graph and
// replayed.
#include "mfma_tile.h"

namespace bmm {
namespace {

__global__ void reset_counters(unsigned int* counters) {
  if (threadIdx.x < kXcds) counters[threadIdx.x * kBatchedCounterStride] = 0u;
}

// Index of the last segment of a queue whose first position is <= t (every
// queue's first segment starts at 0 and t is below the queue's item count).
// Each round, the 64 lanes probe evenly spaced segments and a ballot narrows
// the range 64-fold; called by a whole wave.
__device__ __forceinline__ uint32_t find_segment(const BatchedSeg* __restrict__ segs,
                                                 uint32_t count, uint32_t t, int lane) {
  uint32_t lo = 0, hi = count;
  while (hi - lo > 1) {
    const uint32_t span = hi - lo;
    const uint32_t idx = lo + (uint32_t)(((uint64_t)span * lane) >> 6);
    const uint64_t le = __ballot(segs[idx].begin <= t);  // lanes 0..j, lane 0 always
    const int j = 63 - __builtin_clzll(le);
    const uint32_t nlo = lo + (uint32_t)(((uint64_t)span * j) >> 6);
    if (j < 63) hi = lo + (uint32_t)(((uint64_t)span * (j + 1)) >> 6);
    lo = nlo;
  }
  return lo;
}

// Wave 0: resolve the queue position t (already taken from queue q) into
// (problem, item) in slot[0..1], moving to the next queue while the current
// one is empty; problem -1 once every queue is empty.
__device__ __forceinline__ void resolve_item(const BatchedSeg* __restrict__ segs,
                                             const BatchedQueues& qs,
                                             unsigned int* __restrict__ counters, unsigned t,
                                             int& q, int& visited, int lane, int* slot) {
  while (t >= qs.items[q]) {
    if (++visited == kXcds) {
      if (lane == 0) slot[0] = -1;
      return;
    }
    q = (q + 1) % kXcds;
    unsigned v = 0;
    if (lane == 0) v = atomicAdd(&counters[q * kBatchedCounterStride], 1u);
    t = __shfl(v, 0);
  }
  const BatchedSeg* qsegs = segs + qs.seg_off[q];
  const uint32_t s = find_segment(qsegs, qs.seg_count[q], t, lane);
  if (lane == 0) {
    slot[0] = (int)qsegs[s].problem;
    slot[1] = (int)(qsegs[s].item_lo + (t - qsegs[s].begin));
  }
}

// The register-fed items keep the 32-bit operand expansion: the persistent loop's own
// state leaves no room for the wide form's registers.  The LDS-shared items widen their
// shorter side (its two B^T rows; int8 33.0 -> 32.1 ms, fp4 24.2 -> 23.8 ms).
constexpr bool kWide = false;

template <int RA, int RB, int FMT>
__device__ __forceinline__ void run_item(const BatchedDesc& d, int64_t item, int w) {
  int64_t im, in;
  band_coord(item, d.items_m, d.items_n, im, in);
  const int64_t tm = 2 * im + (w >> 1), tn = 2 * in + (w & 1);
  if (tm >= d.tiles_m || tn >= d.tiles_n) return;  // uniform per wave
  // (the tile reads and writes through global-memory pointers: the table's
  // pointers are device memory)
  const uint64_t* A = d.A;
  const uint64_t* BT = d.BT;
  uint64_t* C = d.C;
  // (the chunked long-k loop of the one-shot leaf measured no faster here: most
  // items are short, and its code doubles the kernel)
  if (d.aligned) {
    mfma::tile<mfma::SEMI_ANY, RA, RB, 2, FMT, 2, 0, kWide>(A, d.lda, BT, d.ldbt, C, d.ldc, d.m,
                                                          d.k, d.n, tm, tn, 0, d.semiring);
  } else {
    mfma::tile<mfma::SEMI_ANY, RA, RB, 1, FMT, 2, 0, kWide>(A, d.lda, BT, d.ldbt, C, d.ldc, d.m,
                                                          d.k, d.n, tm, tn, 0, d.semiring);
  }
}

// LDS-staged items (tile 4): mfma::lds_item (operand rows of the workgroup's 2 x 2
// wave tiles staged through LDS once per stage and shared by the four waves).  (Loading
// the next item's first stage during the current item's epilogue measured slower: wave
// 0 then has to name the next item before the last stage's barrier, which the other
// waves wait for.)
template <int FMT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void batched_lds_kernel(
    const BatchedDesc* __restrict__ descs, const BatchedSeg* __restrict__ segs,
    BatchedQueues qs, unsigned int* __restrict__ counters) {
  __shared__ int slots[2][2];
  __shared__ __attribute__((aligned(16))) unsigned char smem[mfma::kLdsItemBytes];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  int q = blockIdx.x % kXcds, visited = 0;  // wave 0's queue state
  if (w == 0) {
    unsigned v = 0;
    if (lane == 0) v = atomicAdd(&counters[q * kBatchedCounterStride], 1u);
    resolve_item(segs, qs, counters, __shfl(v, 0), q, visited, lane, slots[0]);
  }
  __syncthreads();
  mfma::LdsStage stage;
  for (int it = 0;; ++it) {
    const int* cur = slots[it & 1];
    const int p = __builtin_amdgcn_readfirstlane(cur[0]);
    if (p < 0) break;  // the same for every wave of the workgroup
    const int item = __builtin_amdgcn_readfirstlane(cur[1]);
    unsigned v = 0;
    if (w == 0 && lane == 0 && visited < kXcds)
      v = atomicAdd(&counters[q * kBatchedCounterStride], 1u);
    const BatchedDesc& d = descs[p];
    int64_t im, in;
    band_coord(item, d.items_m, d.items_n, im, in);
    mfma::lds_item<mfma::SEMI_ANY, FMT, true, true>(
        d.A, d.lda, d.BT, d.ldbt, d.C, d.ldc, d.m, d.k, d.n, im, in, d.tiles_m, d.tiles_n,
        d.aligned != 0, 0, d.semiring, w, smem, stage);
    if (w == 0) resolve_item(segs, qs, counters, __shfl(v, 0), q, visited, lane, slots[(it + 1) & 1]);
    __syncthreads();
  }
}

template <int RA, int RB, int FMT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void batched_kernel(
    const BatchedDesc* __restrict__ descs, const BatchedSeg* __restrict__ segs,
    BatchedQueues qs, unsigned int* __restrict__ counters) {
  // two (problem, item) slots: wave 0 fills one while the others read the other
  __shared__ int slots[2][2];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  int q = blockIdx.x % kXcds, visited = 0;  // wave 0's queue state
  if (w == 0) {
    unsigned v = 0;
    if (lane == 0) v = atomicAdd(&counters[q * kBatchedCounterStride], 1u);
    resolve_item(segs, qs, counters, __shfl(v, 0), q, visited, lane, slots[0]);
  }
  __syncthreads();
  for (int it = 0;; ++it) {
    const int* cur = slots[it & 1];
    const int p = __builtin_amdgcn_readfirstlane(cur[0]);
    if (p < 0) break;  // the same for every wave of the workgroup
    const int item = __builtin_amdgcn_readfirstlane(cur[1]);
    unsigned v = 0;
    if (w == 0 && lane == 0 && visited < kXcds)
      v = atomicAdd(&counters[q * kBatchedCounterStride], 1u);
    run_item<RA, RB, FMT>(descs[p], item, w);
    if (w == 0) resolve_item(segs, qs, counters, __shfl(v, 0), q, visited, lane, slots[(it + 1) & 1]);
    __syncthreads();
  }
}

template <int RA, int RB, int FMT>
void launch_k(const BatchedDesc* descs, const BatchedSeg* segs, const BatchedQueues& qs,
              unsigned int* counters, int grid, hipStream_t s) {
  hipLaunchKernelGGL((batched_kernel<RA, RB, FMT>), dim3((unsigned)grid), dim3(256), 0, s, descs,
                     segs, qs, counters);
}

template <int FMT>
void launch_fmt(const BatchedDesc* descs, const BatchedSeg* segs, const BatchedQueues& qs,
                unsigned int* counters, int grid, int tile, hipStream_t s) {
  if (tile == 4)
    hipLaunchKernelGGL((batched_lds_kernel<FMT>), dim3((unsigned)grid), dim3(256), 0, s, descs,
                       segs, qs, counters);
  else if (tile == 1) launch_k<4, 2, FMT>(descs, segs, qs, counters, grid, s);
  else if (tile == 3) launch_k<2, 4, FMT>(descs, segs, qs, counters, grid, s);
  else launch_k<2, 2, FMT>(descs, segs, qs, counters, grid, s);
}

}  // namespace

int batched_tile_rows(int tile) { return tile == 1 || tile == 4 ? 128 : 64; }
int batched_tile_cols(int tile) { return tile == 3 ? 128 : 64; }

hipError_t launch_batched_persistent(const BatchedDesc* descs, const BatchedSeg* segs,
                                     const BatchedQueues& queues, unsigned int* counters,
                                     int grid, int tile, int fmt, hipStream_t s) {
  uint64_t items = 0;
  for (int x = 0; x < kXcds; ++x) items += queues.items[x];
  if (items == 0 || grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, s, counters);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (fmt == mfma::FMT_F4)
    launch_fmt<mfma::FMT_F4>(descs, segs, queues, counters, grid, tile, s);
  else
    launch_fmt<mfma::FMT_I8>(descs, segs, queues, counters, grid, tile, s);
  return hipGetLastError();
}

}  // namespace bmm
