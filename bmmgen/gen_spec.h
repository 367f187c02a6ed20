/* Seeded synthetic bit-matrix generator: the specification shared by the CPU
 * and GPU implementations in this module.
 *
 * This module only draws input bits.  It holds none of the matrix-product
 * arithmetic, so the oracle and the GPU library can both use it.
 *
 * Hash: sm(x) = splitmix64 finalizer applied to x + 0x9E3779B97F4A7C15
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014; Vigna's public-domain splitmix64.c).  sm(0) is the first
 * output of splitmix64 seeded with 0, 0xE220A8397B1DCDAF.
 *
 *   rowkey(seed, tag, r) = sm(sm(seed ^ tag) ^ r)
 *   word(seed, tag, r, w, t) = sm(rowkey ^ ((w << 8) | t))
 *
 * Bit j of row r is bit (j % 64) of packed word j / 64 (LSB first).
 * Distributions (kind, param):
 *   BMMGEN_HALF      Bernoulli(1/2): word(.., 0)
 *   BMMGEN_POW2      Bernoulli(2^-e), e = param in [1, 32]: AND of word(.., t), t < e
 *   BMMGEN_THRESH    Bernoulli(thr / 2^32), thr = param < 2^32: bit b is set iff
 *                    the 32-bit half (b even: low, b odd: high) of
 *                    word(.., 1 + b / 2) is below thr
 * Bits at columns >= cols, and words at index >= ceil(cols / 64) inside the
 * row pitch, are zero.
 */
#ifndef BMMGEN_SPEC_H
#define BMMGEN_SPEC_H

#include <stdint.h>

#define BMMGEN_HALF 0
#define BMMGEN_POW2 1
#define BMMGEN_THRESH 2

#define BMMGEN_GOLDEN 0x9E3779B97F4A7C15ull

#endif
