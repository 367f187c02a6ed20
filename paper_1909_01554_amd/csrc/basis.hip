// Basis changes of the alternative-basis designs (sections 2.2 and 2.3; the
// 2 x 2 programs are in scheme.h).
//
// The change of basis for d recursion levels is the Kronecker power
// phi x ... x phi x I_leaf, applied one level at a time (Yates's algorithm,
// section 2.6), in place.  On a right-hand operand stored transposed the
// program reads its stored 01 quadrant as the 10 quadrant and vice versa at
// every level (the self-inverse change is symmetric in the two).
//
// The work is HBM-bound, so R <= 3 consecutive levels are fused per pass:
// each thread loads the 4^R words that one word position takes in the 2^R x 2^R
// sub-blocks of those levels, applies the R levels in registers and stores only
// the words of quadrants that some level writes.
#include "bmm_internal.h"
#include "scheme.h"

namespace bmm {
namespace {

// SCH: bmm_scheme; INV: 0 forward, 1 inverse; T: 1 for a transposed operand.
template <int R, int SCH, int INV, int T>
__global__ __launch_bounds__(256) void basis_kernel(uint64_t* __restrict__ X, int64_t ld,
                                                    int64_t stride, int64_t rows,
                                                    int64_t row_words, int64_t batch,
                                                    int level0) {
  constexpr int S = 1 << R;  // sub-blocks per side in this pass
  constexpr int W = scheme::written<SCH, INV, T>();
  // level0 = index (0-based, 0 = top) of the first level in this pass
  const int64_t outer_rows = rows >> level0;       // size of one outer block
  const int64_t outer_words = row_words >> level0;
  const int64_t IR = outer_rows >> R;               // inner block size
  const int64_t IW = outer_words >> R;
  const int64_t n_outer = (int64_t)1 << level0;    // outer blocks per side
  const int64_t per = n_outer * n_outer * IR * IW;
  const int64_t total = per * batch;
  const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gstride) {
    const int64_t b = e / per;
    int64_t q = e - b * per;
    const int64_t iw = q % IW;
    q /= IW;
    const int64_t ir = q % IR;
    q /= IR;
    const int64_t oc = q % n_outer;
    const int64_t orr = q / n_outer;
    uint64_t* base = X + b * stride + (orr * outer_rows + ir) * ld + oc * outer_words + iw;
    uint64_t x[S][S];
#pragma unroll
    for (int I = 0; I < S; ++I)
#pragma unroll
      for (int J = 0; J < S; ++J) x[I][J] = base[(int64_t)I * IR * ld + (int64_t)J * IW];
#pragma unroll
    for (int lv = 0; lv < R; ++lv) {
      const int bit = 1 << (R - 1 - lv);
#pragma unroll
      for (int I = 0; I < S; ++I) {
        if (I & bit) continue;
#pragma unroll
        for (int J = 0; J < S; ++J) {
          if (J & bit) continue;
          uint64_t& x00 = x[I][J];
          uint64_t& s01 = x[I][J | bit];
          uint64_t& s10 = x[I | bit][J];
          uint64_t& x11 = x[I | bit][J | bit];
          uint64_t& x01 = T ? s10 : s01;
          uint64_t& x10 = T ? s01 : s10;
          if (INV == 0)
            scheme::fwd<SCH>(x00, x01, x10, x11);
          else
            scheme::inv<SCH>(x00, x01, x10, x11);
        }
      }
    }
#pragma unroll
    for (int I = 0; I < S; ++I)
#pragma unroll
      for (int J = 0; J < S; ++J) {
        // written if at some level this word sits in a quadrant the program writes
        bool changed = false;
#pragma unroll
        for (int lv = 0; lv < R; ++lv) {
          const int bit = 1 << (R - 1 - lv);
          const int quad = ((I & bit) ? 2 : 0) | ((J & bit) ? 1 : 0);
          changed = changed || ((W >> quad) & 1);
        }
        if (changed) base[(int64_t)I * IR * ld + (int64_t)J * IW] = x[I][J];
      }
  }
}

template <int R, int SCH, int INV, int T>
hipError_t launch_pass4(uint64_t* X, int64_t ld, int64_t stride, int64_t rows,
                        int64_t row_words, int64_t batch, int level0, hipStream_t s) {
  const int64_t total = ((rows * row_words) >> (2 * R)) * batch;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((basis_kernel<R, SCH, INV, T>), dim3((unsigned)blocks), dim3(256), 0, s, X,
                     ld, stride, rows, row_words, batch, level0);
  return hipGetLastError();
}

template <int R>
hipError_t launch_pass(uint64_t* X, int64_t ld, int64_t stride, int64_t rows, int64_t row_words,
                       int64_t batch, int level0, int inverse, int sch, int transposed,
                       hipStream_t s) {
  if (sch == BMM_SCHEME_CHAINING) {
    // the chaining programs are not symmetric in the 01 and 10 quadrants, so a transposed
    // operand takes its own instantiation in both directions
    if (inverse && transposed)
      return launch_pass4<R, BMM_SCHEME_CHAINING, 1, 1>(X, ld, stride, rows, row_words, batch,
                                                        level0, s);
    if (inverse)
      return launch_pass4<R, BMM_SCHEME_CHAINING, 1, 0>(X, ld, stride, rows, row_words, batch,
                                                        level0, s);
    if (transposed)
      return launch_pass4<R, BMM_SCHEME_CHAINING, 0, 1>(X, ld, stride, rows, row_words, batch,
                                                        level0, s);
    return launch_pass4<R, BMM_SCHEME_CHAINING, 0, 0>(X, ld, stride, rows, row_words, batch,
                                                      level0, s);
  }
  // self-inverse: both programs are symmetric in the 01 and 10 quadrants
  if (inverse)
    return launch_pass4<R, BMM_SCHEME_SELF_INVERSE, 1, 0>(X, ld, stride, rows, row_words, batch,
                                                          level0, s);
  return launch_pass4<R, BMM_SCHEME_SELF_INVERSE, 0, 0>(X, ld, stride, rows, row_words, batch,
                                                        level0, s);
}

}  // namespace

hipError_t launch_basis(uint64_t* X, int64_t ld, int64_t stride, int64_t rows,
                        int64_t row_words, int64_t batch, int depth, int inverse,
                        hipStream_t s, int scheme, int transposed) {
  if (depth <= 0 || rows <= 0 || row_words <= 0 || batch <= 0) return hipSuccess;
  if (scheme == BMM_SCHEME_WINOGRAD) return hipSuccess;  // the standard basis
  int level = 0;
  while (level < depth) {
    const int left = depth - level;
    // split into passes of at most three levels, as even as possible
    const int passes_left = (left + 2) / 3;
    const int r = (left + passes_left - 1) / passes_left;
    hipError_t err;
    if (r == 3)
      err = launch_pass<3>(X, ld, stride, rows, row_words, batch, level, inverse, scheme,
                           transposed, s);
    else if (r == 2)
      err = launch_pass<2>(X, ld, stride, rows, row_words, batch, level, inverse, scheme,
                           transposed, s);
    else
      err = launch_pass<1>(X, ld, stride, rows, row_words, batch, level, inverse, scheme,
                           transposed, s);
    if (err != hipSuccess) return err;
    level += r;
  }
  return hipSuccess;
}

}  // namespace bmm
