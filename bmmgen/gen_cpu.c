/* CPU implementation of the seeded bit-matrix generator (spec in gen_spec.h). */
#include "gen_spec.h"
#include <stddef.h>

static inline uint64_t sm(uint64_t x) {
  uint64_t z = x + BMMGEN_GOLDEN;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t bmmgen_hash(uint64_t x) { return sm(x); }

static inline uint64_t gen_word(uint64_t rowkey, uint64_t w, int kind, uint64_t param) {
  if (kind == BMMGEN_HALF) return sm(rowkey ^ (w << 8));
  if (kind == BMMGEN_POW2) {
    uint64_t v = ~0ull;
    for (uint64_t t = 0; t < param; ++t) v &= sm(rowkey ^ ((w << 8) | t));
    return v;
  }
  /* BMMGEN_THRESH */
  uint64_t v = 0;
  for (int b = 0; b < 64; b += 2) {
    uint64_t h = sm(rowkey ^ ((w << 8) | (uint64_t)(1 + b / 2)));
    if ((h & 0xFFFFFFFFull) < param) v |= 1ull << b;
    if ((h >> 32) < param) v |= 1ull << (b + 1);
  }
  return v;
}

/* Fill rows [row0, row0 + rows) and words [w0, w0 + nwords) of a matrix with
 * `cols` columns in total into dst (row pitch ld words).  Returns 0 on
 * success, -1 on bad arguments. */
int bmmgen_fill_cpu(uint64_t* dst, int64_t rows, int64_t nwords, int64_t ld,
                    int64_t row0, int64_t w0, int64_t cols, uint64_t seed,
                    uint64_t tag, int kind, uint64_t param) {
  if (!dst || rows < 0 || nwords < 0 || ld < nwords || row0 < 0 || w0 < 0 || cols < 0)
    return -1;
  if (kind < 0 || kind > 2) return -1;
  if (kind == BMMGEN_POW2 && (param < 1 || param > 32)) return -1;
  if (kind == BMMGEN_THRESH && param > 0xFFFFFFFFull) return -1;
  const int64_t row_words = (cols + 63) / 64;
  const uint64_t base = sm(seed ^ tag);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    const uint64_t rowkey = sm(base ^ (uint64_t)(row0 + r));
    uint64_t* out = dst + (size_t)r * (size_t)ld;
    for (int64_t w = 0; w < nwords; ++w) {
      const int64_t gw = w0 + w;
      uint64_t v = 0;
      if (gw < row_words) {
        v = gen_word(rowkey, (uint64_t)gw, kind, param);
        const int64_t tail = cols - gw * 64;
        if (tail < 64) v &= (1ull << tail) - 1ull;
      }
      out[w] = v;
    }
  }
  return 0;
}
