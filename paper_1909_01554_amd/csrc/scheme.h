// The 2x2 block schemes of the recursion, as register-level straight-line
// programs on one 64-bit word position of the four quadrants (index order
// 00, 01, 10, 11) or of the seven products (0..6).  XOR is addition over GF(2).
//
//   SELF_INVERSE (section 2.2, Theorem 1):
//     basis      eq. mb-fwdbasisrecurrence:  X11 <- X01 + X10 + X11
//     inverse    eq. mb-revbasisrecurrence:  X01 <- X01 + X11, X10 <- X10 + X11
//     alpha/beta eq. mb-tsrecurrence, gamma eq. mb-qrecurrence
//   CHAINING (section 2.3, Theorem 2):
//     basis      eq. ab-fwdbasisrecurrence:  X11 <- X01 + X11, X10 <- X01 + X10 + X11
//     inverse    eq. ab-revbasisrecurrence:  X10 <- X10 + X11, X11 <- X01 + X11
//     alpha/beta eq. ab-tsrecurrence, gamma eq. ab-qrecurrence
//   WINOGRAD (section 2.1, the standard basis):
//     no basis change; eqs. sw-input and sw-output
//
// The programs also run on the host: fed the masks 1, 2, 4, 8 for the four
// quadrants (1 << h for the seven products) they return, as bit masks, the
// coefficient sets of their outputs, which the out-of-core host levels use.
//
// The same forward change applies to both operands.  The right operand is
// kept transposed (its quadrant (j, k) stored at (k, j)), so on it the
// programs read the stored 01 quadrant as B10 and the stored 10 as B01.
#pragma once

#include <stdint.h>

#include "../../include/bmm.h"

namespace bmm {
namespace scheme {

// Forward basis change of one 2x2 block (in place).
template <int SCH>
__host__ __device__ __forceinline__ void fwd(uint64_t& x00, uint64_t& x01, uint64_t& x10,
                                             uint64_t& x11) {
  (void)x00;
  if constexpr (SCH == BMM_SCHEME_SELF_INVERSE) {
    x11 ^= x01 ^ x10;
  } else if constexpr (SCH == BMM_SCHEME_CHAINING) {
    x11 ^= x01;
    x10 ^= x11;
  }
}

// Inverse basis change of the result (in place).
template <int SCH>
__host__ __device__ __forceinline__ void inv(uint64_t& x00, uint64_t& x01, uint64_t& x10,
                                             uint64_t& x11) {
  (void)x00;
  if constexpr (SCH == BMM_SCHEME_SELF_INVERSE) {
    x01 ^= x11;
    x10 ^= x11;
  } else if constexpr (SCH == BMM_SCHEME_CHAINING) {
    x10 ^= x11;
    x11 ^= x01;
  }
}

// Quadrants a program writes (bit q = quadrant q in the order 00, 01, 10, 11),
// for operands stored as is (T = 0) or transposed (T = 1).  Words of the other
// quadrants keep their values and are not stored.
template <int SCH, int INV, int T>
constexpr int written() {
  if (SCH == BMM_SCHEME_SELF_INVERSE) return INV ? 0x6 : 0x8;  // 01+10 / 11
  // chaining: both directions write 10 and 11 (stored 01 and 11 when transposed)
  if (SCH == BMM_SCHEME_CHAINING) return T ? 0xA : 0xC;
  return 0;
}

// Left operand (alpha): seven children from A's quadrants.
template <int SCH>
__host__ __device__ __forceinline__ void alpha(uint64_t a00, uint64_t a01, uint64_t a10,
                                               uint64_t a11, uint64_t (&o)[7]) {
  if constexpr (SCH == BMM_SCHEME_SELF_INVERSE) {
    o[0] = a00;
    o[1] = a01;
    o[2] = a10;
    o[3] = a11;
    o[4] = a00 ^ a11;
    o[5] = a01 ^ a11;
    o[6] = a10 ^ a11;
  } else if constexpr (SCH == BMM_SCHEME_CHAINING) {
    o[0] = a00;
    o[1] = a01;
    o[2] = a10;
    o[3] = a11;
    o[4] = a00 ^ a10;
    o[5] = a01 ^ a10;
    o[6] = a10 ^ a11;
  } else {
    // T2 = A01 + A11 feeds T3 = A10 + T2, which feeds T4 = A00 + T3
    const uint64_t t2 = a01 ^ a11;
    const uint64_t t3 = a10 ^ t2;
    o[0] = a10 ^ a11;
    o[1] = a01;
    o[2] = t2;
    o[3] = t3;
    o[4] = a00 ^ t3;
    o[5] = a10;
    o[6] = a00;
  }
}

// Right operand (beta), from B's quadrants in the standard orientation.
template <int SCH>
__host__ __device__ __forceinline__ void beta(uint64_t b00, uint64_t b01, uint64_t b10,
                                              uint64_t b11, uint64_t (&o)[7]) {
  if constexpr (SCH == BMM_SCHEME_SELF_INVERSE) {
    o[0] = b00;
    o[1] = b10;
    o[2] = b00 ^ b11;
    o[3] = b11;
    o[4] = b01;
    o[5] = b01 ^ b11;
    o[6] = b10 ^ b11;
  } else if constexpr (SCH == BMM_SCHEME_CHAINING) {
    o[0] = b00;
    o[1] = b10 ^ b11;
    o[2] = b10;
    o[3] = b11;
    o[4] = b01;
    o[5] = b01 ^ b10;
    o[6] = b00 ^ b10;
  } else {
    // S2 = B01 + B11 feeds S3 = B10 + S2, which feeds S5 = B00 + S3
    const uint64_t s2 = b01 ^ b11;
    const uint64_t s3 = b10 ^ s2;
    o[0] = b10 ^ b11;
    o[1] = b10;
    o[2] = s2;
    o[3] = s3;
    o[4] = b01;
    o[5] = b00 ^ s3;
    o[6] = b00;
  }
}

// Expansion of a stored operand: SIDE 0 = left (alpha), 1 = right stored transposed (beta).
template <int SCH, int SIDE>
__host__ __device__ __forceinline__ void expand_one(uint64_t q00, uint64_t q01, uint64_t q10,
                                                    uint64_t q11, uint64_t (&o)[7]) {
  if constexpr (SIDE == 0)
    alpha<SCH>(q00, q01, q10, q11, o);
  else
    beta<SCH>(q00, q10, q01, q11, o);  // stored 01 is B10, stored 10 is B01
}

// Combination of the seven products into the four result quadrants (gamma / zeta).
template <int SCH>
__host__ __device__ __forceinline__ void compress_one(const uint64_t (&q)[7], uint64_t& c00,
                                                      uint64_t& c01, uint64_t& c10,
                                                      uint64_t& c11) {
  if constexpr (SCH == BMM_SCHEME_SELF_INVERSE) {
    c00 = q[0] ^ q[1];
    c01 = q[4] ^ q[6];
    c10 = q[2] ^ q[5];
    c11 = q[1] ^ q[3] ^ q[5] ^ q[6];
  } else if constexpr (SCH == BMM_SCHEME_CHAINING) {
    const uint64_t r = q[1] ^ q[2] ^ q[4];
    c00 = q[0] ^ q[1];
    c01 = r ^ q[5];
    c10 = r ^ q[6];
    c11 = q[3] ^ q[4];
  } else {
    const uint64_t u0 = q[1] ^ q[3];
    const uint64_t u1 = q[2] ^ u0;
    const uint64_t u2 = q[4] ^ u0;
    c00 = q[1] ^ q[6];
    c01 = q[0] ^ u2;
    c10 = q[5] ^ u1;
    c11 = q[0] ^ u1;
  }
}

}  // namespace scheme
}  // namespace bmm
