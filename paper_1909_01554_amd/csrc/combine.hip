// Expanding and compressing levels of the recursion (sections 3.8, 3.9, 3.11;
// Algorithms 1 and 2 of the paper) for every 2 x 2 scheme in scheme.h: the
// self-inverse design (eqs. mb-tsrecurrence and mb-qrecurrence, matrix form
// eq. mb-albega), the chaining design (eqs. ab-tsrecurrence and
// ab-qrecurrence) and Strassen-Winograd (eqs. sw-input and sw-output).
//
// The right operand is kept transposed throughout (its quadrant (j, k) lives
// at (k, j)), so the right expansion reads the stored 01 quadrant as B10 and
// the stored 10 quadrant as B01; each S_h is then produced already transposed.
//
// Every thread owns one 64-bit word position of a child (or grandchild) and
// moves it through registers: one level reads 4 words and writes 7 (expand)
// or reads 7 and writes 4 (compress); the merged two-level kernels read 16 and
// write 49, or read 49 and write 16, so the intermediate level never goes to
// HBM (section 3.15, merging levels).  Children of parent p are matrices
// 7p + h, grandchildren 49p + 7h1 + h2, stored compactly one after another.
#include "bmm_internal.h"
#include "scheme.h"

namespace bmm {
namespace {

using scheme::compress_one;
using scheme::expand_one;

template <int SCH, int SIDE>
__global__ __launch_bounds__(256) void expand_kernel(const uint64_t* __restrict__ src,
                                                     int64_t ldp, int64_t strideP,
                                                     uint64_t* __restrict__ dst, int64_t rows,
                                                     int64_t words, int64_t parents) {
  const int64_t hr = rows >> 1, hw = words >> 1;
  const int64_t csize = hr * hw;
  const int64_t total = csize * parents;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t p = e / csize;
    const int64_t q = e - p * csize;
    const int64_t r = q / hw;
    const int64_t w = q - r * hw;
    const uint64_t* P = src + p * strideP;
    const uint64_t q00 = P[r * ldp + w];
    const uint64_t q01 = P[r * ldp + hw + w];
    const uint64_t q10 = P[(r + hr) * ldp + w];
    const uint64_t q11 = P[(r + hr) * ldp + hw + w];
    uint64_t o[7];
    expand_one<SCH, SIDE>(q00, q01, q10, q11, o);
    uint64_t* D = dst + 7 * p * csize + q;
#pragma unroll
    for (int h = 0; h < 7; ++h) D[h * csize] = o[h];
  }
}

template <int SCH, int SIDE>
__global__ __launch_bounds__(256) void expand2_kernel(const uint64_t* __restrict__ src,
                                                      int64_t ldp, int64_t strideP,
                                                      uint64_t* __restrict__ dst, int64_t rows,
                                                      int64_t words, int64_t parents) {
  const int64_t qr = rows >> 2, qw = words >> 2;
  const int64_t gsize = qr * qw;
  const int64_t total = gsize * parents;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t p = e / gsize;
    const int64_t q = e - p * gsize;
    const int64_t r = q / qw;
    const int64_t w = q - r * qw;
    const uint64_t* P = src + p * strideP + r * ldp + w;
    // x[i1][j1][i2][j2] at row i1*2qr + i2*qr + r, word j1*2qw + j2*qw + w
    uint64_t x[2][2][2][2];
#pragma unroll
    for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
      for (int j1 = 0; j1 < 2; ++j1)
#pragma unroll
        for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
          for (int j2 = 0; j2 < 2; ++j2)
            x[i1][j1][i2][j2] = P[(i1 * 2 * qr + i2 * qr) * ldp + j1 * 2 * qw + j2 * qw];
    // first level: for each inner quadrant (i2, j2), expand over (i1, j1)
    uint64_t t[7][2][2];
#pragma unroll
    for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
      for (int j2 = 0; j2 < 2; ++j2) {
        uint64_t o[7];
        expand_one<SCH, SIDE>(x[0][0][i2][j2], x[0][1][i2][j2], x[1][0][i2][j2], x[1][1][i2][j2], o);
#pragma unroll
        for (int h = 0; h < 7; ++h) t[h][i2][j2] = o[h];
      }
    uint64_t* D = dst + 49 * p * gsize + q;
#pragma unroll
    for (int h1 = 0; h1 < 7; ++h1) {
      uint64_t o[7];
      expand_one<SCH, SIDE>(t[h1][0][0], t[h1][0][1], t[h1][1][0], t[h1][1][1], o);
#pragma unroll
      for (int h2 = 0; h2 < 7; ++h2) D[(7 * h1 + h2) * gsize] = o[h2];
    }
  }
}

template <int ACC>
__device__ __forceinline__ void put(uint64_t& d, uint64_t v) {
  if (ACC)
    d ^= v;
  else
    d = v;
}

// ACC = 1: the parent quadrants are XORed into dst instead of overwriting it.
template <int SCH, int ACC>
__global__ __launch_bounds__(256) void compress_kernel(const uint64_t* __restrict__ src,
                                                       uint64_t* __restrict__ dst, int64_t ldp,
                                                       int64_t strideP, int64_t rows,
                                                       int64_t words, int64_t parents) {
  const int64_t hr = rows >> 1, hw = words >> 1;
  const int64_t csize = hr * hw;
  const int64_t total = csize * parents;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t p = e / csize;
    const int64_t q = e - p * csize;
    const int64_t r = q / hw;
    const int64_t w = q - r * hw;
    const uint64_t* S = src + 7 * p * csize + q;
    uint64_t v[7];
#pragma unroll
    for (int h = 0; h < 7; ++h) v[h] = S[h * csize];
    uint64_t c00, c01, c10, c11;
    compress_one<SCH>(v, c00, c01, c10, c11);
    uint64_t* P = dst + p * strideP;
    put<ACC>(P[r * ldp + w], c00);
    put<ACC>(P[r * ldp + hw + w], c01);
    put<ACC>(P[(r + hr) * ldp + w], c10);
    put<ACC>(P[(r + hr) * ldp + hw + w], c11);
  }
}

template <int SCH, int ACC>
__global__ __launch_bounds__(256) void compress2_kernel(const uint64_t* __restrict__ src,
                                                        uint64_t* __restrict__ dst, int64_t ldp,
                                                        int64_t strideP, int64_t rows,
                                                        int64_t words, int64_t parents) {
  const int64_t qr = rows >> 2, qw = words >> 2;
  const int64_t gsize = qr * qw;
  const int64_t total = gsize * parents;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t p = e / gsize;
    const int64_t q = e - p * gsize;
    const int64_t r = q / qw;
    const int64_t w = q - r * qw;
    const uint64_t* S = src + 49 * p * gsize + q;
    // inner level: for each h1, combine the seven h2 products into quadrants (i2, k2)
    uint64_t c[7][2][2];
#pragma unroll
    for (int h1 = 0; h1 < 7; ++h1) {
      uint64_t v[7];
#pragma unroll
      for (int h2 = 0; h2 < 7; ++h2) v[h2] = S[(7 * h1 + h2) * gsize];
      compress_one<SCH>(v, c[h1][0][0], c[h1][0][1], c[h1][1][0], c[h1][1][1]);
    }
    uint64_t* P = dst + p * strideP + r * ldp + w;
#pragma unroll
    for (int i2 = 0; i2 < 2; ++i2)
#pragma unroll
      for (int k2 = 0; k2 < 2; ++k2) {
        uint64_t v[7];
#pragma unroll
        for (int h1 = 0; h1 < 7; ++h1) v[h1] = c[h1][i2][k2];
        uint64_t c00, c01, c10, c11;
        compress_one<SCH>(v, c00, c01, c10, c11);
        const int64_t off = i2 * qr * ldp + k2 * qw;
        put<ACC>(P[off], c00);
        put<ACC>(P[off + 2 * qw], c01);
        put<ACC>(P[off + 2 * qr * ldp], c10);
        put<ACC>(P[off + 2 * qr * ldp + 2 * qw], c11);
      }
  }
}

// One child of one parent (rows x words, pitch ldp): dst (rows/2 x words/2, pitch ldd)
// = XOR of the parent quadrants in `mask` (bit q: quadrant q in the order 00, 01, 10, 11).
__global__ __launch_bounds__(256) void child_kernel(const uint64_t* __restrict__ src,
                                                    int64_t ldp, uint64_t* __restrict__ dst,
                                                    int64_t ldd, int64_t rows, int64_t words,
                                                    uint32_t mask) {
  const int64_t hr = rows >> 1, hw = words >> 1;
  const int64_t total = hr * hw;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t r = e / hw;
    const int64_t w = e - r * hw;
    uint64_t v = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if ((mask >> q) & 1u) v ^= src[(r + (q >> 1) * hr) * ldp + (q & 1) * hw + w];
    dst[r * ldd + w] = v;
  }
}

// One product (rows/2 x words/2, pitch lds) into the parent's result quadrants in
// `targets`: overwriting those in `overwrite`, XORed into the others.
__global__ __launch_bounds__(256) void gamma_kernel(const uint64_t* __restrict__ src,
                                                    int64_t lds, uint64_t* __restrict__ dst,
                                                    int64_t ldp, int64_t rows, int64_t words,
                                                    uint32_t targets, uint32_t overwrite) {
  const int64_t hr = rows >> 1, hw = words >> 1;
  const int64_t total = hr * hw;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t r = e / hw;
    const int64_t w = e - r * hw;
    const uint64_t v = src[r * lds + w];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((targets >> q) & 1u)) continue;
      uint64_t& d = dst[(r + (q >> 1) * hr) * ldp + (q & 1) * hw + w];
      d = ((overwrite >> q) & 1u) ? v : (d ^ v);
    }
  }
}

__global__ __launch_bounds__(256) void copy_kernel(const uint64_t* __restrict__ src, int64_t lds,
                                                   uint64_t* __restrict__ dst, int64_t ldd,
                                                   int64_t rows, int64_t words) {
  const int64_t total = rows * words;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t r = e / words;
    const int64_t w = e - r * words;
    dst[r * ldd + w] = src[r * lds + w];
  }
}

__global__ __launch_bounds__(256) void xor_kernel(const uint64_t* __restrict__ src, int64_t lds,
                                                  uint64_t* __restrict__ dst, int64_t ldd,
                                                  int64_t rows, int64_t words) {
  const int64_t total = rows * words;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t r = e / words;
    const int64_t w = e - r * words;
    dst[r * ldd + w] ^= src[r * lds + w];
  }
}

// Pseudo-random words for the autotuner's timing buffers (the matrix cores' rate
// depends on how many operand bits switch, so tuning runs on dense random bits):
// the 64-bit finalizer of MurmurHash3 applied to seed + index.
__global__ __launch_bounds__(256) void random_kernel(uint64_t* __restrict__ dst, int64_t words,
                                                     uint64_t seed) {
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < words; e += gstride) {
    uint64_t z = seed + (uint64_t)e;
    z ^= z >> 33;
    z *= 0xFF51AFD7ED558CCDull;
    z ^= z >> 33;
    z *= 0xC4CEB9FE1A85EC53ull;
    z ^= z >> 33;
    dst[e] = z;
  }
}

__global__ __launch_bounds__(256) void zero_kernel(uint64_t* __restrict__ dst, int64_t ld,
                                                   int64_t rows, int64_t words) {
  const int64_t total = rows * words;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t r = e / words;
    const int64_t w = e - r * words;
    dst[r * ld + w] = 0ull;
  }
}

inline unsigned grid_for(int64_t total) {
  int64_t blocks = (total + 255) / 256;
  if (blocks > 32768) blocks = 32768;
  if (blocks < 1) blocks = 1;
  return (unsigned)blocks;
}

template <int SCH>
hipError_t expand_sch(int side, int levels, const uint64_t* src, int64_t ldp, int64_t strideP,
                      uint64_t* dst, int64_t rows, int64_t words, int64_t parents,
                      hipStream_t s) {
  const int sh = levels == 2 ? 2 : 1;
  const int64_t total = (rows >> sh) * (words >> sh) * parents;
  if (total <= 0) return hipSuccess;
  const dim3 g(grid_for(total)), b(256);
  if (levels == 2) {
    if (side == 0)
      hipLaunchKernelGGL((expand2_kernel<SCH, 0>), g, b, 0, s, src, ldp, strideP, dst, rows,
                         words, parents);
    else
      hipLaunchKernelGGL((expand2_kernel<SCH, 1>), g, b, 0, s, src, ldp, strideP, dst, rows,
                         words, parents);
  } else {
    if (side == 0)
      hipLaunchKernelGGL((expand_kernel<SCH, 0>), g, b, 0, s, src, ldp, strideP, dst, rows,
                         words, parents);
    else
      hipLaunchKernelGGL((expand_kernel<SCH, 1>), g, b, 0, s, src, ldp, strideP, dst, rows,
                         words, parents);
  }
  return hipGetLastError();
}

template <int SCH>
hipError_t compress_sch(int levels, const uint64_t* src, uint64_t* dst, int64_t ldp,
                        int64_t strideP, int64_t rows, int64_t words, int64_t parents,
                        hipStream_t s, int accumulate) {
  const int sh = levels == 2 ? 2 : 1;
  const int64_t total = (rows >> sh) * (words >> sh) * parents;
  if (total <= 0) return hipSuccess;
  const dim3 g(grid_for(total)), b(256);
  if (levels == 2) {
    if (accumulate)
      hipLaunchKernelGGL((compress2_kernel<SCH, 1>), g, b, 0, s, src, dst, ldp, strideP, rows,
                         words, parents);
    else
      hipLaunchKernelGGL((compress2_kernel<SCH, 0>), g, b, 0, s, src, dst, ldp, strideP, rows,
                         words, parents);
  } else {
    if (accumulate)
      hipLaunchKernelGGL((compress_kernel<SCH, 1>), g, b, 0, s, src, dst, ldp, strideP, rows,
                         words, parents);
    else
      hipLaunchKernelGGL((compress_kernel<SCH, 0>), g, b, 0, s, src, dst, ldp, strideP, rows,
                         words, parents);
  }
  return hipGetLastError();
}

hipError_t expand_any(int scheme, int side, int levels, const uint64_t* src, int64_t ldp,
                      int64_t strideP, uint64_t* dst, int64_t rows, int64_t words,
                      int64_t parents, hipStream_t s) {
  switch (scheme) {
    case BMM_SCHEME_CHAINING:
      return expand_sch<BMM_SCHEME_CHAINING>(side, levels, src, ldp, strideP, dst, rows, words,
                                             parents, s);
    case BMM_SCHEME_WINOGRAD:
      return expand_sch<BMM_SCHEME_WINOGRAD>(side, levels, src, ldp, strideP, dst, rows, words,
                                             parents, s);
    default:
      return expand_sch<BMM_SCHEME_SELF_INVERSE>(side, levels, src, ldp, strideP, dst, rows,
                                                 words, parents, s);
  }
}

hipError_t compress_any(int scheme, int levels, const uint64_t* src, uint64_t* dst, int64_t ldp,
                        int64_t strideP, int64_t rows, int64_t words, int64_t parents,
                        hipStream_t s, int accumulate) {
  switch (scheme) {
    case BMM_SCHEME_CHAINING:
      return compress_sch<BMM_SCHEME_CHAINING>(levels, src, dst, ldp, strideP, rows, words,
                                               parents, s, accumulate);
    case BMM_SCHEME_WINOGRAD:
      return compress_sch<BMM_SCHEME_WINOGRAD>(levels, src, dst, ldp, strideP, rows, words,
                                               parents, s, accumulate);
    default:
      return compress_sch<BMM_SCHEME_SELF_INVERSE>(levels, src, dst, ldp, strideP, rows, words,
                                                   parents, s, accumulate);
  }
}

// Coefficient masks of a scheme, from its own programs run on bit masks: the stored
// quadrants child h of side `side` sums, and the products result quadrant q sums.
template <int SCH>
uint32_t child_mask_of(int side, int h) {
  uint64_t o[7];
  if (side == 0)
    scheme::expand_one<SCH, 0>(1, 2, 4, 8, o);
  else
    scheme::expand_one<SCH, 1>(1, 2, 4, 8, o);
  return (uint32_t)o[h];
}
template <int SCH>
void gamma_masks_of(uint32_t (&g)[4]) {
  const uint64_t in[7] = {1, 2, 4, 8, 16, 32, 64};
  uint64_t c[4];
  scheme::compress_one<SCH>(in, c[0], c[1], c[2], c[3]);
  for (int q = 0; q < 4; ++q) g[q] = (uint32_t)c[q];
}

}  // namespace

uint32_t child_mask(int scheme, int side, int h) {
  if (scheme == BMM_SCHEME_CHAINING) return child_mask_of<BMM_SCHEME_CHAINING>(side, h);
  if (scheme == BMM_SCHEME_WINOGRAD) return child_mask_of<BMM_SCHEME_WINOGRAD>(side, h);
  return child_mask_of<BMM_SCHEME_SELF_INVERSE>(side, h);
}

hipError_t launch_child(int scheme, int side, int h, const uint64_t* src, int64_t ldp,
                        uint64_t* dst, int64_t ldd, int64_t rows, int64_t words, hipStream_t s) {
  const int64_t total = (rows >> 1) * (words >> 1);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(child_kernel, dim3(grid_for(total)), dim3(256), 0, s, src, ldp, dst, ldd,
                     rows, words, child_mask(scheme, side, h));
  return hipGetLastError();
}

hipError_t launch_gamma(int scheme, int h, const uint64_t* src, int64_t lds, uint64_t* dst,
                        int64_t ldp, int64_t rows, int64_t words, int accumulate,
                        hipStream_t s) {
  const int64_t total = (rows >> 1) * (words >> 1);
  if (total <= 0) return hipSuccess;
  uint32_t g[4];
  if (scheme == BMM_SCHEME_CHAINING)
    gamma_masks_of<BMM_SCHEME_CHAINING>(g);
  else if (scheme == BMM_SCHEME_WINOGRAD)
    gamma_masks_of<BMM_SCHEME_WINOGRAD>(g);
  else
    gamma_masks_of<BMM_SCHEME_SELF_INVERSE>(g);
  uint32_t targets = 0, overwrite = 0;
  for (int q = 0; q < 4; ++q) {
    if (!((g[q] >> h) & 1u)) continue;
    targets |= 1u << q;
    // the first product of a quadrant overwrites it, unless the result accumulates
    if (!accumulate && (g[q] & ((1u << h) - 1u)) == 0) overwrite |= 1u << q;
  }
  hipLaunchKernelGGL(gamma_kernel, dim3(grid_for(total)), dim3(256), 0, s, src, lds, dst, ldp,
                     rows, words, targets, overwrite);
  return hipGetLastError();
}

hipError_t launch_expand(int side, const uint64_t* src, int64_t ldp, int64_t strideP,
                         uint64_t* dst, int64_t rows, int64_t words, int64_t parents,
                         hipStream_t s, int scheme) {
  return expand_any(scheme, side, 1, src, ldp, strideP, dst, rows, words, parents, s);
}

hipError_t launch_expand2(int side, const uint64_t* src, int64_t ldp, int64_t strideP,
                          uint64_t* dst, int64_t rows, int64_t words, int64_t parents,
                          hipStream_t s, int scheme) {
  return expand_any(scheme, side, 2, src, ldp, strideP, dst, rows, words, parents, s);
}

hipError_t launch_compress(const uint64_t* src, uint64_t* dst, int64_t ldp, int64_t strideP,
                           int64_t rows, int64_t words, int64_t parents, hipStream_t s,
                           int accumulate, int scheme) {
  return compress_any(scheme, 1, src, dst, ldp, strideP, rows, words, parents, s, accumulate);
}

hipError_t launch_compress2(const uint64_t* src, uint64_t* dst, int64_t ldp, int64_t strideP,
                            int64_t rows, int64_t words, int64_t parents, hipStream_t s,
                            int accumulate, int scheme) {
  return compress_any(scheme, 2, src, dst, ldp, strideP, rows, words, parents, s, accumulate);
}

hipError_t launch_copy(const uint64_t* src, int64_t lds, uint64_t* dst, int64_t ldd,
                       int64_t rows, int64_t words, hipStream_t s) {
  const int64_t total = rows * words;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(total)), dim3(256), 0, s, src, lds, dst, ldd,
                     rows, words);
  return hipGetLastError();
}

hipError_t launch_xor(const uint64_t* src, int64_t lds, uint64_t* dst, int64_t ldd, int64_t rows,
                      int64_t words, hipStream_t s) {
  const int64_t total = rows * words;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(xor_kernel, dim3(grid_for(total)), dim3(256), 0, s, src, lds, dst, ldd, rows,
                     words);
  return hipGetLastError();
}

hipError_t launch_random(uint64_t* dst, int64_t words, uint64_t seed, hipStream_t s) {
  if (words <= 0) return hipSuccess;
  hipLaunchKernelGGL(random_kernel, dim3(grid_for(words)), dim3(256), 0, s, dst, words, seed);
  return hipGetLastError();
}

hipError_t launch_zero(uint64_t* dst, int64_t ld, int64_t rows, int64_t words, hipStream_t s) {
  const int64_t total = rows * words;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(total)), dim3(256), 0, s, dst, ld, rows, words);
  return hipGetLastError();
}

}  // namespace bmm
