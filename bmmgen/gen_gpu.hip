// GPU implementation of the seeded bit-matrix generator (spec in gen_spec.h).
// One thread per output word; a grid-stride loop covers any size.
#include <hip/hip_runtime.h>
#include "gen_spec.h"

namespace {

__device__ __forceinline__ uint64_t sm(uint64_t x) {
  uint64_t z = x + BMMGEN_GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void fill_kernel(uint64_t* __restrict__ dst, int64_t rows, int64_t nwords,
                            int64_t ld, int64_t row0, int64_t w0, int64_t cols,
                            uint64_t base, int kind, uint64_t param) {
  const int64_t row_words = (cols + 63) / 64;
  const int64_t total = rows * nwords;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / nwords;
    const int64_t w = e - r * nwords;
    const int64_t gw = w0 + w;
    uint64_t v = 0;
    if (gw < row_words) {
      const uint64_t rowkey = sm(base ^ (uint64_t)(row0 + r));
      const uint64_t wk = (uint64_t)gw << 8;
      if (kind == BMMGEN_HALF) {
        v = sm(rowkey ^ wk);
      } else if (kind == BMMGEN_POW2) {
        v = ~0ull;
        for (uint64_t t = 0; t < param; ++t) v &= sm(rowkey ^ (wk | t));
      } else {
        for (int b = 0; b < 64; b += 2) {
          const uint64_t h = sm(rowkey ^ (wk | (uint64_t)(1 + b / 2)));
          if ((h & 0xFFFFFFFFull) < param) v |= 1ull << b;
          if ((h >> 32) < param) v |= 1ull << (b + 1);
        }
      }
      const int64_t tail = cols - gw * 64;
      if (tail < 64) v &= (1ull << tail) - 1ull;
    }
    dst[r * ld + w] = v;
  }
}

uint64_t host_sm(uint64_t x) {
  uint64_t z = x + BMMGEN_GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

// Device-memory counterpart of bmmgen_fill_cpu, enqueued on `stream`.
// Returns 0 on success, -1 on bad arguments, -2 on a launch error.
extern "C" int bmmgen_fill_gpu(uint64_t* dst, int64_t rows, int64_t nwords, int64_t ld,
                               int64_t row0, int64_t w0, int64_t cols, uint64_t seed,
                               uint64_t tag, int kind, uint64_t param, void* stream) {
  if (!dst || rows < 0 || nwords < 0 || ld < nwords || row0 < 0 || w0 < 0 || cols < 0)
    return -1;
  if (kind < 0 || kind > 2) return -1;
  if (kind == BMMGEN_POW2 && (param < 1 || param > 32)) return -1;
  if (kind == BMMGEN_THRESH && param > 0xFFFFFFFFull) return -1;
  const int64_t total = rows * nwords;
  if (total == 0) return 0;
  const int threads = 256;
  int64_t blocks = (total + threads - 1) / threads;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(threads), 0,
                     (hipStream_t)stream, dst, rows, nwords, ld, row0, w0, cols,
                     host_sm(seed ^ tag), kind, param);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
