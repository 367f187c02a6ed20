"""Stage oracles for the alternative-basis recursion (sections 2.2, 2.6, 2.7, 3.4).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Blocks are 2-D numpy arrays whose elements support XOR: unpacked bits
(uint8, any even size) or packed uint64 words (the column split must fall on
a word boundary).  Quadrant (a, b) of X is rows a*h..(a+1)*h, columns
b*w..(b+1)*w, the paper's first-index-major block order 00, 01, 10, 11.

* ``basis(X, d, prog)`` applies a 2x2 basis change at every one of the top d
  levels, i.e. (phi x ... x phi x I_leaf) X, one level at a time (Yates's
  algorithm, section 2.6; levels may go in any order, ``bottom_up`` picks
  the other one).
* ``expand_left`` / ``expand_right`` form the seven operand blocks of one
  level (alpha / beta), ``compress`` combines seven product blocks (gamma).
* ``core`` is the recursion over the alternative basis: expand, recurse into
  the seven products, compress, down to a leaf product.
* ``product`` is the whole method: forward basis change of A and B, the core,
  inverse basis change of C.  It reaches AB exactly over GF(2), so its own
  oracle is the plain product ``oracle.mul``.
"""
import numpy as np

from . import algebra


def quadrants(X):
    r, c = X.shape
    if r % 2 or c % 2:
        raise ValueError("block dimensions must be even to split into quadrants")
    h, w = r // 2, c // 2
    return X[:h, :w], X[:h, w:], X[h:, :w], X[h:, w:]


def assemble(Q00, Q01, Q10, Q11):
    return np.block([[Q00, Q01], [Q10, Q11]])


def basis(X, d, prog, bottom_up=False):
    """Apply the 2x2 basis change `prog` at each of the top d levels of X."""
    if d == 0:
        return X.copy()
    if bottom_up:
        inner = assemble(*[basis(q, d - 1, prog, True) for q in quadrants(X)])
        return assemble(*prog(*[q.copy() for q in quadrants(inner)]))
    top = prog(*[q.copy() for q in quadrants(X)])
    return assemble(*[basis(q, d - 1, prog, False) for q in top])


def expand_left(X, dec=algebra.SELF_INVERSE):
    return [np.ascontiguousarray(t) for t in dec.alpha(*quadrants(X))]


def expand_right(X, dec=algebra.SELF_INVERSE):
    return [np.ascontiguousarray(t) for t in dec.beta(*quadrants(X))]


def compress(Q, dec=algebra.SELF_INVERSE):
    return assemble(*dec.gamma(*Q))


def core(Ah, Bh, d, leaf, dec=algebra.SELF_INVERSE):
    """Alternative-basis core (A-hat, B-hat) -> C-hat with d recursion levels."""
    if d == 0:
        return leaf(Ah, Bh)
    T = expand_left(Ah, dec)
    S = expand_right(Bh, dec)
    Q = [core(T[h], S[h], d - 1, leaf, dec) for h in range(7)]
    return compress(Q, dec)


def product(A, B, d, leaf, dec=algebra.SELF_INVERSE):
    """The full method: C = chi(core(phi A, psi B))."""
    Ah = basis(A, d, dec.fwd)
    Bh = basis(B, d, dec.fwd)
    return basis(core(Ah, Bh, d, leaf, dec), d, dec.inv)


def bits_leaf(A, B):
    """Leaf over unpacked bits: the GF(2) product by integer matmul mod 2."""
    return ((A.astype(np.int64) @ B.astype(np.int64)) & 1).astype(np.uint8)


def packed_leaf(k_bits, n_bits):
    """Leaf over packed words: calls the plain product with the leaf's shape."""
    from . import mul, GF2

    def leaf(A, B):
        return mul(A, B, A.shape[1] * 64, B.shape[1] * 64, GF2)
    return leaf
