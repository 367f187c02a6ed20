/* Oracle for the bit-matrix product: TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code with the GPU library.
 *
 * Definition (paper, section 2.4, the product of an s x t and a t x u matrix;
 * introduction: the Boolean algebra (0,1,OR,AND) and the binary field
 * (0,1,+,*)):
 *     C[i][k] = SUM_j A[i][j] * B[j][k]
 * with SUM = XOR over GF(2) and SUM = OR over the Boolean algebra.
 *
 * Written out plainly: row i of C is the XOR (or OR) of the rows j of B for
 * which bit A[i][j] is set.  Matrices are packed row-major uint64, bit j of a
 * row at bit j % 64 of word j / 64.  No blocking beyond splitting the work
 * over threads.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define ORACLE_GF2 0
#define ORACLE_BOOLEAN 1

static inline int get_bit(const uint64_t* row, int64_t j) {
  return (int)((row[j >> 6] >> (j & 63)) & 1ull);
}

/* Rows of C for R given rows of A.  Each thread owns a slice of output words
 * of every row, so B is streamed once per call. */
int oracle_rows(int semiring, const uint64_t* Arows, int64_t lda, int64_t R,
                const uint64_t* B, int64_t ldb, uint64_t* Crows, int64_t ldc,
                int64_t k, int64_t n) {
  if (semiring != ORACLE_GF2 && semiring != ORACLE_BOOLEAN) return -1;
  if (R < 0 || k < 0 || n < 0) return -1;
  const int64_t nw = (n + 63) / 64;
  if (lda < (k + 63) / 64 || ldb < nw || ldc < nw) return -1;
  for (int64_t r = 0; r < R; ++r) memset(Crows + (size_t)r * ldc, 0, sizeof(uint64_t) * nw);
  const int64_t slice = 64; /* words per work item */
  const int64_t nslices = (nw + slice - 1) / slice;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < nslices; ++s) {
    const int64_t w0 = s * slice;
    const int64_t w1 = (w0 + slice < nw) ? w0 + slice : nw;
    for (int64_t j = 0; j < k; ++j) {
      const uint64_t* brow = B + (size_t)j * ldb;
      for (int64_t r = 0; r < R; ++r) {
        if (!get_bit(Arows + (size_t)r * lda, j)) continue;
        uint64_t* crow = Crows + (size_t)r * ldc;
        if (semiring == ORACLE_GF2) {
          for (int64_t w = w0; w < w1; ++w) crow[w] ^= brow[w];
        } else {
          for (int64_t w = w0; w < w1; ++w) crow[w] |= brow[w];
        }
      }
    }
  }
  return 0;
}

/* The full product C = AB (m x k times k x n). */
int oracle_mul(int semiring, const uint64_t* A, int64_t lda, const uint64_t* B,
               int64_t ldb, uint64_t* C, int64_t ldc, int64_t m, int64_t k, int64_t n) {
  if (m < 0) return -1;
  /* Row blocks keep the per-call accumulator set small. */
  const int64_t blk = 256;
  for (int64_t i0 = 0; i0 < m; i0 += blk) {
    const int64_t R = (m - i0 < blk) ? m - i0 : blk;
    int rc = oracle_rows(semiring, A + (size_t)i0 * lda, lda, R, B, ldb,
                         C + (size_t)i0 * ldc, ldc, k, n);
    if (rc) return rc;
  }
  return 0;
}

/* y = x^T M over GF(2) for a bit vector x of length `rows`: the XOR of the
 * rows i of M with bit i of x set (used by Freivalds's check). */
int oracle_vecmat(const uint64_t* x, const uint64_t* M, int64_t ldm, int64_t rows,
                  int64_t cols, uint64_t* y) {
  if (rows < 0 || cols < 0) return -1;
  const int64_t nw = (cols + 63) / 64;
  if (ldm < nw) return -1;
  memset(y, 0, sizeof(uint64_t) * nw);
  const int64_t slice = 256;
  const int64_t nslices = (nw + slice - 1) / slice;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t s = 0; s < nslices; ++s) {
    const int64_t w0 = s * slice;
    const int64_t w1 = (w0 + slice < nw) ? w0 + slice : nw;
    for (int64_t i = 0; i < rows; ++i) {
      if (!get_bit(x, i)) continue;
      const uint64_t* mrow = M + (size_t)i * ldm;
      for (int64_t w = w0; w < w1; ++w) y[w] ^= mrow[w];
    }
  }
  return 0;
}
