// Persistent variant of the matrix-core leaf for launches of many short tiles
// (the batched leaf products of the recursion, k = 2048 or 4096 bits).
//
// Same arithmetic and tiles as leaf_mfma.hip (see mfma_tile.h), but the grid
// holds only as many workgroups as the chip runs at once, and each one walks
// the logical workgroups blockIdx.x, blockIdx.x + gridDim.x, ...  While a wave
// issues the matrix-core operations of its current tile's last step, it
// already requests the first words of its next tile, so the memory latency at
// the start of a tile hides behind work instead of stalling the wave (a short
// tile has only 8 or 16 steps, so that stall is a large share of its time).
// Logical workgroups go through the same XCD-aware order as the one-shot
// kernel; the grid is a multiple of 8, so every workgroup stays on one XCD's
// range.
#include <algorithm>

#include "mfma_tile.h"

namespace bmm {
namespace {

// Logical workgroup L -> (matrix, workgroup row, workgroup column): the same
// XCD-aware order as xcd_tile, in 32-bit arithmetic (launches here hold fewer
// than 2^31 workgroups).
struct Pos {
  int b, tm, tn;
  bool valid;
};

template <int SEMI, int RA, int RB, int KV, int FMT, bool EDGE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void leaf_mfma_persist_kernel(
    LeafBatch p, int tiles_m, int tiles_n, int total_wg) {
  constexpr int TM = 32 * RA, TN = 32 * RB;
  const int grid_m = (tiles_m + 1) >> 1, grid_n = (tiles_n + 1) >> 1;
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int li = lane & 31;
  const int64_t kw = (p.k + 63) >> 6;
  const int64_t full_steps = kw / (2 * KV);
  // the next tile's first step can ride in the current tile's last pair of steps only
  // when every tile ends on a whole pair and has no tail words
  const bool chain = full_steps >= 2 && (full_steps & 1) == 0 && kw % (2 * KV) == 0;

  auto locate = [&](int L) {
    const int x = L % kXcds, j = L / kXcds;
    const int per = total_wg / kXcds, rem = total_wg % kXcds;
    const int t = x * per + (x < rem ? x : rem) + j;
    const int per_item = grid_m * grid_n;
    Pos q;
    q.b = t / per_item;
    const int r = t - q.b * per_item;
    const int band = kGroupRows * grid_n;
    const int first = (r / band) * kGroupRows;
    const int rows = grid_m - first < kGroupRows ? grid_m - first : kGroupRows;
    const int qq = r - (r / band) * band;
    q.tm = 2 * (first + qq % rows) + (w >> 1);
    q.tn = 2 * (qq / rows) + (w & 1);
    q.valid = q.b < p.batch && q.tm < tiles_m && q.tn < tiles_n;  // uniform per wave
    return q;
  };
  // per-lane row pointers at word KV * half of the tile's first row of A / column of B
  auto base_a = [&](const Pos& q) {
    return p.A + (int64_t)q.b * p.strideA + ((int64_t)q.tm * TM + li) * p.lda + KV * half;
  };
  auto base_b = [&](const Pos& q) {
    return p.BT + (int64_t)q.b * p.strideB + ((int64_t)q.tn * TN + li) * p.ldbt + KV * half;
  };
  auto fetch = [&](const Pos& q, const uint64_t* pa, const uint64_t* pb, int64_t st,
                   uint64_t (&xa)[KV][RA], uint64_t (&xb)[KV][RB]) {
    const int64_t wd = st * 2 * KV;
#pragma unroll
    for (int f = 0; f < RA; ++f) {
      const uint64_t* src = pa + (int64_t)(32 * f) * p.lda + wd;
      if constexpr (EDGE) {  // rows past the end repeat the last row (results discarded)
        int64_t r = (int64_t)q.tm * TM + 32 * f + li;
        r = r < p.m ? r : p.m - 1;
        src = p.A + (int64_t)q.b * p.strideA + r * p.lda + KV * half + wd;
      }
      if constexpr (KV == 2) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(src);
        xa[0][f] = v.x;
        xa[1][f] = v.y;
      } else {
        xa[0][f] = *src;
      }
    }
#pragma unroll
    for (int g = 0; g < RB; ++g) {
      const uint64_t* src = pb + (int64_t)(32 * g) * p.ldbt + wd;
      if constexpr (EDGE) {
        int64_t c = (int64_t)q.tn * TN + 32 * g + li;
        c = c < p.n ? c : p.n - 1;
        src = p.BT + (int64_t)q.b * p.strideB + c * p.ldbt + KV * half + wd;
      }
      if constexpr (KV == 2) {
        const ulonglong2 v = *reinterpret_cast<const ulonglong2*>(src);
        xb[0][g] = v.x;
        xb[1][g] = v.y;
      } else {
        xb[0][g] = *src;
      }
    }
  };

  using AccV = typename mfma::Acc<FMT>::type;
  AccV acc[RA][RB];
  auto compute = [&](const uint64_t (&xa)[KV][RA], const uint64_t (&xb)[KV][RB]) {
#pragma unroll
    for (int v = 0; v < KV; ++v) mfma::mfma_word<SEMI, RA, RB, FMT>(xa[v], xb[v], acc);
  };

  int L = blockIdx.x;
  if (L >= total_wg) return;
  Pos cur = locate(L);
  const uint64_t* pa = base_a(cur);
  const uint64_t* pb = base_b(cur);
  uint64_t a0[KV][RA], b0[KV][RB], a1[KV][RA], b1[KV][RB];
  if (cur.valid && full_steps > 0) fetch(cur, pa, pb, 0, a0, b0);
  while (true) {
    const int Ln = L + (int)gridDim.x;
    const bool has_next = Ln < total_wg;
    const Pos nxt = has_next ? locate(Ln) : Pos{0, 0, 0, false};
    const uint64_t* na = base_a(nxt);
    const uint64_t* nb = base_b(nxt);
    const bool chained = chain && cur.valid && nxt.valid;
    if (cur.valid) {
#pragma unroll
      for (int f = 0; f < RA; ++f)
#pragma unroll
        for (int g = 0; g < RB; ++g) acc[f][g] = AccV{};
      int64_t st = 0;
      // all pairs but the last: the words of step st+1 (then st+2) are requested
      // before the matrix-core work of step st (then st+1) is issued
      for (; st + 3 < full_steps; st += 2) {
        fetch(cur, pa, pb, st + 1, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        compute(a0, b0);
        fetch(cur, pa, pb, st + 2, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        compute(a1, b1);
      }
      if (st + 1 < full_steps) {
        // the last pair: its second half carries the next tile's first step
        fetch(cur, pa, pb, st + 1, a1, b1);
        __builtin_amdgcn_sched_barrier(0);
        compute(a0, b0);
        if (chained)
          fetch(nxt, na, nb, 0, a0, b0);
        else if (st + 2 < full_steps)
          fetch(cur, pa, pb, st + 2, a0, b0);
        __builtin_amdgcn_sched_barrier(0);
        compute(a1, b1);
        st += 2;
      }
      if (st < full_steps) compute(a0, b0);
      // tail: words past the end of the row read as zero
      const int64_t wt = full_steps * 2 * KV;
      if (wt < kw) {
#pragma unroll
        for (int v = 0; v < KV; ++v) {
          const bool in = wt + KV * half + v < kw;
          uint64_t xa[RA], xb[RB];
#pragma unroll
          for (int f = 0; f < RA; ++f) {
            int64_t r = (int64_t)cur.tm * TM + 32 * f + li;
            r = r < p.m ? r : p.m - 1;
            xa[f] = in ? p.A[(int64_t)cur.b * p.strideA + r * p.lda + wt + v + KV * half] : 0ull;
          }
#pragma unroll
          for (int g = 0; g < RB; ++g) {
            int64_t c = (int64_t)cur.tn * TN + 32 * g + li;
            c = c < p.n ? c : p.n - 1;
            xb[g] = in ? p.BT[(int64_t)cur.b * p.strideB + c * p.ldbt + wt + v + KV * half] : 0ull;
          }
          mfma::mfma_word<SEMI, RA, RB, FMT>(xa, xb, acc);
        }
      }
      mfma::epilogue<SEMI, RA, RB, FMT>(acc, p.C + (int64_t)cur.b * p.strideC, p.ldc, p.m, p.n,
                                        cur.tm, cur.tn, p.accumulate);
    }
    if (!has_next) break;
    if (!chained && nxt.valid && full_steps > 0) fetch(nxt, na, nb, 0, a0, b0);
    cur = nxt;
    pa = na;
    pb = nb;
    L = Ln;
  }
}

int persistent_grid() {
  static int grid = 0;
  if (grid == 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // two 4-wave workgroups per CU (two waves per SIMD), a multiple of 8
    grid = ((cus * 2 + 7) / 8) * 8;
  }
  return grid;
}

template <int SEMI, int RA, int RB, int KV, int FMT>
void launch_kv(const LeafBatch& p, int tiles_m, int tiles_n, int total_wg, int grid,
               hipStream_t s) {
  constexpr int TM = 32 * RA, TN = 32 * RB;
  // edge tiles exist when a row or column tile runs past the end of the operand
  const bool edge = p.m % TM != 0 || p.n % TN != 0;
  if (edge)
    hipLaunchKernelGGL((leaf_mfma_persist_kernel<SEMI, RA, RB, KV, FMT, true>), dim3(grid),
                       dim3(256), 0, s, p, tiles_m, tiles_n, total_wg);
  else
    hipLaunchKernelGGL((leaf_mfma_persist_kernel<SEMI, RA, RB, KV, FMT, false>), dim3(grid),
                       dim3(256), 0, s, p, tiles_m, tiles_n, total_wg);
}

template <int SEMI, int RA, int RB, int FMT>
hipError_t launch_p(const LeafBatch& p, hipStream_t s) {
  constexpr int TM = 32 * RA, TN = 32 * RB;
  const int64_t tiles_m = (p.m + TM - 1) / TM;
  const int64_t tiles_n = (((p.n + 63) / 64) * 64 + TN - 1) / TN;
  const int64_t total_wg = ((tiles_m + 1) / 2) * ((tiles_n + 1) / 2) * p.batch;
  if (total_wg == 0) return hipSuccess;
  if (total_wg >= ((int64_t)1 << 31) - persistent_grid()) return hipErrorInvalidValue;
  const int grid = (int)std::min<int64_t>(total_wg, persistent_grid());
  const bool aligned16 = ((reinterpret_cast<uintptr_t>(p.A) | reinterpret_cast<uintptr_t>(p.BT)) & 15) == 0 &&
                         ((p.lda | p.ldbt | p.strideA | p.strideB) & 1) == 0;
  if (aligned16)
    launch_kv<SEMI, RA, RB, 2, FMT>(p, (int)tiles_m, (int)tiles_n, (int)total_wg, grid, s);
  else
    launch_kv<SEMI, RA, RB, 1, FMT>(p, (int)tiles_m, (int)tiles_n, (int)total_wg, grid, s);
  return hipGetLastError();
}

template <int SEMI, int FMT>
hipError_t launch_shape(const LeafBatch& p, int tile, hipStream_t s) {
  if (tile == MFMA_P_64x128) return launch_p<SEMI, 2, 4, FMT>(p, s);
  return launch_p<SEMI, 4, 2, FMT>(p, s);
}

}  // namespace

hipError_t launch_leaf_mfma_persist(int semiring, int fmt, const LeafBatch& p, int tile,
                                    hipStream_t s) {
  if (p.m <= 0 || p.n <= 0 || p.batch <= 0) return hipSuccess;
  if (fmt == mfma::FMT_F4)
    return semiring == GF2 ? launch_shape<GF2, mfma::FMT_F4>(p, tile, s)
                           : launch_shape<BOOLEAN, mfma::FMT_F4>(p, tile, s);
  return semiring == GF2 ? launch_shape<GF2, mfma::FMT_I8>(p, tile, s)
                         : launch_shape<BOOLEAN, mfma::FMT_I8>(p, tile, s);
}

}  // namespace bmm
