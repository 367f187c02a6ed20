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

// The 32-bit operand expansion: the persistent loop's own state leaves no room
// for the wide form's registers.
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

// LDS-staged item (tile 4): the workgroup's 2 x 2 wave tiles of 128 x 64 cover
// 256 rows of A and 128 rows of B^T; per stage of 8 words of k the four waves load
// those 384 rows once, with 16-byte coalesced loads, into LDS (rows padded to 80
// bytes so the lanes of one 16-byte LDS read hit distinct banks) and every wave reads
// its own rows from there: each operand row is fetched from L2 once per workgroup
// instead of once per wave that uses it.  The next stage is loaded into registers
// while the current one computes.  Words past the end of k read as zero; whole
// 4-word groups past it are skipped.  Every wave takes part in the loads and
// barriers; waves whose tile lies outside the problem only skip the epilogue.
constexpr int LS_KS = 8;                       // words of k per stage
constexpr int LS_ROWB = 80;                    // padded LDS row (64 data bytes + 16)
constexpr int LS_ROWS = 256 + 128;             // A rows, then B^T rows
constexpr int LS_PANEL = LS_ROWS * LS_ROWB;    // bytes per stage buffer
constexpr int LS_CHUNKS = LS_ROWS * 4 / 256;   // 16-byte chunks per thread per stage

template <int FMT>
__device__ __forceinline__ void run_item_lds(const BatchedDesc& d, int64_t item, int w,
                                             unsigned char* smem) {
  constexpr int RA = 4, RB = 2;
  int64_t im, in;
  band_coord(item, d.items_m, d.items_n, im, in);
  const int tid = threadIdx.x, lane = tid & 63, half = lane >> 5, li = lane & 31;
  const int64_t row0 = im * 256, col0 = in * 128;
  const mfma::gq_ptr A = (mfma::gq_ptr)d.A;
  const mfma::gq_ptr BT = (mfma::gq_ptr)d.BT;
  const int64_t kw = (d.k + 63) >> 6;
  // staging: chunk q = tid + 256 i covers row q >> 2, words 2 (q & 3) .. + 1 of a stage
  mfma::gq_ptr src[LS_CHUNKS];
  int soff[LS_CHUNKS], spart[LS_CHUNKS];
#pragma unroll
  for (int i = 0; i < LS_CHUNKS; ++i) {
    const int q = tid + 256 * i;
    const int r = q >> 2, part = q & 3;
    spart[i] = part;
    if (r < 256) {
      int64_t g = row0 + r;
      g = g < d.m ? g : d.m - 1;
      src[i] = A + g * d.lda + 2 * part;
    } else {
      int64_t g = col0 + (r - 256);
      g = g < d.n ? g : d.n - 1;
      src[i] = BT + g * d.ldbt + 2 * part;
    }
    soff[i] = r * LS_ROWB + part * 16;
  }
  uint64_t stage[LS_CHUNKS][2];
  auto load = [&](int64_t w0) {
#pragma unroll
    for (int i = 0; i < LS_CHUNKS; ++i) {
      const int64_t wd = w0 + 2 * spart[i];
      if (d.aligned && wd + 1 < kw) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>((const uint64_t*)(src[i] + w0));
        stage[i][0] = v.x;
        stage[i][1] = v.y;
      } else {
        stage[i][0] = wd < kw ? src[i][w0] : 0ull;
        stage[i][1] = wd + 1 < kw ? src[i][w0 + 1] : 0ull;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LS_CHUNKS; ++i) {
      ulonglong2 v;
      v.x = stage[i][0];
      v.y = stage[i][1];
      *reinterpret_cast<ulonglong2*>(smem + buf * LS_PANEL + soff[i]) = v;
    }
  };
  using AccV = typename mfma::Acc<FMT>::type;
  AccV acc[RA][RB];
#pragma unroll
  for (int f = 0; f < RA; ++f)
#pragma unroll
    for (int g = 0; g < RB; ++g) acc[f][g] = AccV{};
  const int wy = w >> 1, wx = w & 1;
  int aoff[RA], boff[RB];
#pragma unroll
  for (int f = 0; f < RA; ++f) aoff[f] = (wy * 128 + 32 * f + li) * LS_ROWB + 16 * half;
#pragma unroll
  for (int g = 0; g < RB; ++g) boff[g] = (256 + wx * 64 + 32 * g + li) * LS_ROWB + 16 * half;

  const int64_t stages = (kw + LS_KS - 1) / LS_KS;
  load(0);
  store(0);
  __syncthreads();
  for (int64_t st = 0; st < stages; ++st) {
    const int cur = (int)(st & 1);
    if (st + 1 < stages) load((st + 1) * LS_KS);
    const unsigned char* base = smem + cur * LS_PANEL;
    // two groups of 4 words per stage: lane half h takes words 4s + 2h and 4s + 2h + 1
#pragma unroll
    for (int s2 = 0; s2 < LS_KS / 4; ++s2) {
      if (st * LS_KS + 4 * s2 >= kw) break;  // uniform: only zero words are left
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
      mfma::mfma_word<mfma::SEMI_ANY, RA, RB, FMT, kWide>(xa[0], xb[0], acc);
      mfma::mfma_word<mfma::SEMI_ANY, RA, RB, FMT, kWide>(xa[1], xb[1], acc);
    }
    if (st + 1 < stages) store(cur ^ 1);
    __syncthreads();
  }
  const int64_t tm = 2 * im + wy, tn = 2 * in + wx;
  if (tm < d.tiles_m && tn < d.tiles_n)
    mfma::epilogue<mfma::SEMI_ANY, RA, RB, FMT>(acc, d.C, d.ldc, d.m, d.n, tm, tn, 0,
                                                d.semiring);
}

template <int FMT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void batched_lds_kernel(
    const BatchedDesc* __restrict__ descs, const BatchedSeg* __restrict__ segs,
    BatchedQueues qs, unsigned int* __restrict__ counters) {
  __shared__ int slots[2][2];
  __shared__ __attribute__((aligned(16))) unsigned char smem[2 * LS_PANEL];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
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
    run_item_lds<FMT>(descs[p], item, w, smem);
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
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
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
