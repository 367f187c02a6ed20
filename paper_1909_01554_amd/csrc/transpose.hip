// Bit-matrix transpose: one wave per 64 x 64 bit block.
//
// Lane l loads word (row 64*rb + l, word column wc); six butterfly stages
// (distance 32, 16, ..., 1) exchange the off-diagonal halves of ever smaller
// sub-blocks through cross-lane shuffles, after which lane l holds column
// 64*wc + l as a 64-bit word over the block's rows.  Bits of rows past the end
// read as zero, so the padding of the transposed rows is zero.
#include "bmm_internal.h"

namespace bmm {
namespace {

__device__ __forceinline__ uint64_t swap_stage(uint64_t x, int lane, int j, uint64_t m) {
  const uint64_t y = __shfl_xor(x, j);
  if ((lane & j) == 0) {
    // this lane is row k, the partner row k + j: take the partner's low part
    const uint64_t t = ((x >> j) ^ y) & m;
    return x ^ (t << j);
  }
  const uint64_t t = ((y >> j) ^ x) & m;
  return x ^ t;
}

__global__ __launch_bounds__(256) void transpose_kernel(const uint64_t* __restrict__ src,
                                                        int64_t lds, int64_t strideS,
                                                        uint64_t* __restrict__ dst, int64_t ldd,
                                                        int64_t strideD, int64_t rows,
                                                        int64_t cols, int64_t n_rb,
                                                        int64_t n_wc, int64_t batch) {
  const int lane = threadIdx.x & 63;
  const int64_t blk = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t per = n_rb * n_wc;
  const int64_t b = blk / per;
  if (b >= batch) return;
  const int64_t t = blk - b * per;
  const int64_t rb = t / n_wc;
  const int64_t wc = t - rb * n_wc;
  const int64_t r = rb * 64 + lane;
  uint64_t x = r < rows ? src[b * strideS + r * lds + wc] : 0ull;
  x = swap_stage(x, lane, 32, 0x00000000FFFFFFFFull);
  x = swap_stage(x, lane, 16, 0x0000FFFF0000FFFFull);
  x = swap_stage(x, lane, 8, 0x00FF00FF00FF00FFull);
  x = swap_stage(x, lane, 4, 0x0F0F0F0F0F0F0F0Full);
  x = swap_stage(x, lane, 2, 0x3333333333333333ull);
  x = swap_stage(x, lane, 1, 0x5555555555555555ull);
  const int64_t c = wc * 64 + lane;
  if (c < cols) dst[b * strideD + c * ldd + rb] = x;
}

}  // namespace

hipError_t launch_transpose(const uint64_t* src, int64_t lds, int64_t strideS, uint64_t* dst,
                            int64_t ldd, int64_t strideD, int64_t rows, int64_t cols,
                            int64_t batch, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || batch <= 0) return hipSuccess;
  const int64_t n_rb = (rows + 63) / 64;
  const int64_t n_wc = (cols + 63) / 64;
  const int64_t total = n_rb * n_wc * batch;
  const int64_t blocks = (total + 3) / 4;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, lds,
                     strideS, dst, ldd, strideD, rows, cols, n_rb, n_wc, batch);
  return hipGetLastError();
}

}  // namespace bmm
