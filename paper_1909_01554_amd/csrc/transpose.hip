// Bit-matrix transpose in 64 x 64 bit blocks.
//
// Lane l holds word (row 64*rb + l, word column wc) of a block; six butterfly stages
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

// A workgroup transposes a tile of 512 rows x 8 words (8 x 8 blocks of 64 x 64
// bits) through LDS, so global reads and writes move 64 contiguous bytes per
// eight threads; each wave transposes 16 of the blocks in registers.
constexpr int TR_ROWS = 512, TR_WORDS = 8, TR_STR = 9;  // padded LDS row (in words)

__global__ __launch_bounds__(256) void transpose_kernel(const uint64_t* __restrict__ src,
                                                        int64_t lds, int64_t strideS,
                                                        uint64_t* __restrict__ dst, int64_t ldd,
                                                        int64_t strideD, int64_t rows,
                                                        int64_t cols, int64_t n_rt,
                                                        int64_t n_wt, int64_t batch) {
  __shared__ uint64_t tile[TR_ROWS * TR_STR];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int64_t per = n_rt * n_wt;
  const int64_t b = (int64_t)blockIdx.x / per;
  if (b >= batch) return;  // uniform per workgroup
  const int64_t t = (int64_t)blockIdx.x - b * per;
  const int64_t r0 = (t / n_wt) * TR_ROWS;
  const int64_t w0 = (t % n_wt) * TR_WORDS;
  const int64_t src_words = (cols + 63) >> 6;
  const int64_t dst_words = (rows + 63) >> 6;
  const uint64_t* S = src + b * strideS;
  uint64_t* D = dst + b * strideD;
  const int sub_r = tid >> 3, sub_w = tid & 7;
#pragma unroll 4
  for (int it = 0; it < TR_ROWS / 32; ++it) {
    const int lr = it * 32 + sub_r;
    const int64_t r = r0 + lr, w = w0 + sub_w;
    tile[lr * TR_STR + sub_w] = (r < rows && w < src_words) ? S[r * lds + w] : 0ull;
  }
  __syncthreads();
  uint64_t res[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int blk = wave * 16 + i;
    const int rb = blk >> 3, wc = blk & 7;
    uint64_t x = tile[(rb * 64 + lane) * TR_STR + wc];
    x = swap_stage(x, lane, 32, 0x00000000FFFFFFFFull);
    x = swap_stage(x, lane, 16, 0x0000FFFF0000FFFFull);
    x = swap_stage(x, lane, 8, 0x00FF00FF00FF00FFull);
    x = swap_stage(x, lane, 4, 0x0F0F0F0F0F0F0F0Full);
    x = swap_stage(x, lane, 2, 0x3333333333333333ull);
    x = swap_stage(x, lane, 1, 0x5555555555555555ull);
    res[i] = x;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int blk = wave * 16 + i;
    const int rb = blk >> 3, wc = blk & 7;
    // lane now holds output row (64 * (w0 + wc) + lane), word (r0 / 64 + rb)
    tile[(wc * 64 + lane) * TR_STR + rb] = res[i];
  }
  __syncthreads();
#pragma unroll 4
  for (int it = 0; it < TR_ROWS / 32; ++it) {
    const int orow = it * 32 + sub_r;
    const int64_t c = w0 * 64 + orow, wd = r0 / 64 + sub_w;
    if (c < cols && wd < dst_words) D[c * ldd + wd] = tile[orow * TR_STR + sub_w];
  }
}

}  // namespace

hipError_t launch_transpose(const uint64_t* src, int64_t lds, int64_t strideS, uint64_t* dst,
                            int64_t ldd, int64_t strideD, int64_t rows, int64_t cols,
                            int64_t batch, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || batch <= 0) return hipSuccess;
  const int64_t n_rt = (rows + TR_ROWS - 1) / TR_ROWS;
  const int64_t n_wt = ((cols + 63) / 64 + TR_WORDS - 1) / TR_WORDS;
  const int64_t blocks = n_rt * n_wt * batch;
  if (!grid_fits(blocks, 256)) return kGridTooLarge;
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, lds,
                     strideS, dst, ldd, strideD, rows, cols, n_rt, n_wt, batch);
  return hipGetLastError();
}

}  // namespace bmm
