// Persistent batched leaf: many independent products of uneven sizes in one
// launch.  Each wave pulls output tiles (128 x 64 or 64 x 64, int8 or E2M1
// operands, as the plan chose) from a device-wide counter until the queue is
// empty; a tile's problem is found by binary search over the per-problem tile
// prefix sums.  The tile itself is the matrix-core leaf (mfma_tile.h).  The
// plan orders problems by decreasing k (longest tiles first), so the queue
// drains with a short tail.  A separate one-thread kernel zeroes the counter
// before each launch, so the pair can be captured into a HIP graph and
// replayed.
#include "mfma_tile.h"

namespace bmm {
namespace {

__global__ void reset_counter(unsigned int* counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

template <int RA, int RB, int KV, int FMT>
__device__ __forceinline__ void run_tile(const BatchedDesc& d, int64_t tm, int64_t tn) {
  if (d.semiring == GF2)
    mfma::tile<GF2, RA, RB, KV, FMT>(d.A, d.lda, d.BT, d.ldbt, d.C, d.ldc, d.m, d.k, d.n, tm,
                                     tn, 0);
  else
    mfma::tile<BOOLEAN, RA, RB, KV, FMT>(d.A, d.lda, d.BT, d.ldbt, d.C, d.ldc, d.m, d.k, d.n,
                                         tm, tn, 0);
}

template <int RA, int RB, int FMT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void batched_kernel(
    const BatchedDesc* __restrict__ descs, const uint32_t* __restrict__ begins, int64_t count,
    int64_t total_tiles, unsigned int* __restrict__ counter, int cached) {
  // Each persistent workgroup copies the problems' first-tile indices into LDS
  // once (when they fit), so finding a tile's problem is an LDS binary search.
  extern __shared__ uint32_t sbeg[];
  if (cached) {
    for (int64_t i = threadIdx.x; i < count; i += blockDim.x) sbeg[i] = begins[i];
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  while (true) {
    unsigned int t = 0;
    if (lane == 0) t = atomicAdd(counter, 1u);
    t = __shfl(t, 0);
    if ((int64_t)t >= total_tiles) break;  // every wave exits once the queue is drained
    // binary search: last problem whose first tile is <= t
    int64_t lo = 0, hi = count - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      const uint32_t b = cached ? sbeg[mid] : begins[mid];
      if (b <= t) lo = mid;
      else hi = mid - 1;
    }
    const BatchedDesc d = descs[lo];
    const int64_t local = (int64_t)t - d.tile_begin;
    const int64_t tm = local / d.tiles_n;
    const int64_t tn = local - tm * d.tiles_n;
    const bool aligned = ((reinterpret_cast<uintptr_t>(d.A) | reinterpret_cast<uintptr_t>(d.BT)) & 15) == 0 &&
                         ((d.lda | d.ldbt) & 1) == 0;
    if (aligned) run_tile<RA, RB, 2, FMT>(d, tm, tn);
    else run_tile<RA, RB, 1, FMT>(d, tm, tn);
  }
}

template <int RA, int RB, int FMT>
void launch_k(const BatchedDesc* descs, const uint32_t* begins, int64_t count,
              int64_t total_tiles, unsigned int* counter, int grid, int cached, size_t lds,
              hipStream_t s) {
  hipLaunchKernelGGL((batched_kernel<RA, RB, FMT>), dim3((unsigned)grid), dim3(256), lds, s,
                     descs, begins, count, total_tiles, counter, cached);
}

}  // namespace

int batched_tile_rows(int tile) { return tile == 1 ? 128 : 64; }
int batched_tile_cols(int tile) { return tile == 1 ? 64 : 64; }

hipError_t launch_batched_persistent(const BatchedDesc* descs, const uint32_t* begins,
                                     int64_t count, int64_t total_tiles, unsigned int* counter,
                                     int grid, int tile, int fmt, hipStream_t s) {
  if (count <= 0 || total_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cached = count <= kBatchedLdsProblems ? 1 : 0;
  const size_t lds = cached ? (size_t)count * sizeof(uint32_t) : 0;
  if (tile == 1) {
    if (fmt == mfma::FMT_F4)
      launch_k<4, 2, mfma::FMT_F4>(descs, begins, count, total_tiles, counter, grid, cached, lds, s);
    else
      launch_k<4, 2, mfma::FMT_I8>(descs, begins, count, total_tiles, counter, grid, cached, lds, s);
  } else {
    if (fmt == mfma::FMT_F4)
      launch_k<2, 2, mfma::FMT_F4>(descs, begins, count, total_tiles, counter, grid, cached, lds, s);
    else
      launch_k<2, 2, mfma::FMT_I8>(descs, begins, count, total_tiles, counter, grid, cached, lds, s);
  }
  return hipGetLastError();
}

}  // namespace bmm
