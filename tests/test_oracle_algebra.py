"""Pins of the alternative-basis algebra and the recursion's stage oracles.

The straight-line programs in oracle.algebra were typed from the paper's
recurrences (sections 2.1-2.3); the golden files were typed from the printed
matrices (sections 2.5, 2.8).  Each transcription checks the other, and both are
checked against what the mathematics fixes: the triple product property, the
identities stated in section 2.8, the counts of Theorems 1-2 and section 1.1,
and the product AB itself.  CPU only.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
from oracle import algebra, brute, strassen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name + ".txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return np.array(rows, dtype=np.int64)


def gf2(M):
    return np.asarray(M, dtype=np.int64) & 1


def mm(*Ms):
    out = Ms[0]
    for M in Ms[1:]:
        out = gf2(out @ M)
    return out


DESIGNS = {
    "selfinv": algebra.SELF_INVERSE,
    "chain": algebra.CHAINING,
}


@pytest.mark.parametrize("prefix", ["selfinv", "chain"])
def test_programs_equal_printed_matrices(prefix):
    dec = DESIGNS[prefix]
    assert np.array_equal(algebra.matrix_of(dec.fwd, 4), golden(prefix + "_phi"))
    assert np.array_equal(algebra.matrix_of(dec.inv, 4), golden(prefix + "_chi"))
    assert np.array_equal(algebra.matrix_of(dec.alpha, 4), golden(prefix + "_alpha"))
    assert np.array_equal(algebra.matrix_of(dec.beta, 4), golden(prefix + "_beta"))
    assert np.array_equal(algebra.matrix_of(dec.gamma, 7), golden(prefix + "_gamma"))


def test_strassen_winograd_programs_equal_printed_matrices():
    assert np.array_equal(algebra.matrix_of(algebra.sw_xi, 4), golden("sw_xi"))
    assert np.array_equal(algebra.matrix_of(algebra.sw_eta, 4), golden("sw_eta"))
    assert np.array_equal(algebra.matrix_of(algebra.sw_zeta, 7), golden("sw_zeta"))


@pytest.mark.parametrize("prefix", ["selfinv", "chain"])
def test_triple_product_property_alt_basis(prefix):
    """(chi gamma | alpha phi, beta psi) has the triple product property <2,2,2>_7."""
    phi, chi = golden(prefix + "_phi"), golden(prefix + "_chi")
    al, be, ga = golden(prefix + "_alpha"), golden(prefix + "_beta"), golden(prefix + "_gamma")
    assert algebra.triple_product_ok(mm(chi, ga), mm(al, phi), mm(be, phi))


def test_triple_product_property_strassen_winograd():
    assert algebra.triple_product_ok(golden("sw_zeta"), golden("sw_xi"), golden("sw_eta"))


def test_triple_product_fails_on_planted_mistakes():
    """A dropped term, a flipped entry or a transposed operand breaks the property."""
    phi, chi = golden("selfinv_phi"), golden("selfinv_chi")
    al, be, ga = golden("selfinv_alpha"), golden("selfinv_beta"), golden("selfinv_gamma")
    for M, which in [(al, 0), (be, 1), (ga, 2)]:
        for (r, c) in itertools.product(range(M.shape[0]), range(M.shape[1])):
            X = M.copy()
            X[r, c] ^= 1
            args = [al, be, ga]
            args[which] = X
            assert not algebra.triple_product_ok(mm(chi, args[2]), mm(args[0], phi),
                                                 mm(args[1], phi))
    assert not algebra.triple_product_ok(mm(chi, ga), mm(be, phi), mm(al, phi))


def test_selfinverse_identities():
    """Section 2.8: phi = psi = chi^T, phi = phi^-1 and chi = chi^-1 over GF(2)."""
    phi, chi = golden("selfinv_phi"), golden("selfinv_chi")
    I = np.eye(4, dtype=np.int64)
    assert np.array_equal(mm(phi, phi), I)
    assert np.array_equal(mm(chi, chi), I)
    assert np.array_equal(chi, phi.T)
    # the design does not chain: chi is not phi^-1 (remark at the end of section 2.2)
    assert not np.array_equal(mm(chi, phi), I)


def test_chaining_identities():
    """Section 2.8: chi = phi^-1 = psi^-1 for the chaining design."""
    phi, chi = golden("chain_phi"), golden("chain_chi")
    assert np.array_equal(mm(chi, phi), np.eye(4, dtype=np.int64))
    assert np.array_equal(mm(phi, chi), np.eye(4, dtype=np.int64))


def test_weights_and_addition_counts():
    """Theorem 1 / Theorem 2 (section 1.2) and section 2.8."""
    for prefix in ("selfinv", "chain"):
        al, be = golden(prefix + "_alpha"), golden(prefix + "_beta")
        assert sorted(al.sum(axis=1)) == [1, 1, 1, 1, 2, 2, 2]
        assert sorted(be.sum(axis=1)) == [1, 1, 1, 1, 2, 2, 2]
    assert sorted(golden("selfinv_gamma").sum(axis=0)) == [1, 1, 1, 1, 2, 2, 2]
    assert sorted(golden("chain_gamma").sum(axis=0)) == [1, 1, 1, 1, 2, 3, 3]
    for dec in (algebra.SELF_INVERSE, algebra.CHAINING):
        assert algebra.slp_additions(dec.fwd, 4) == 2
        assert algebra.slp_additions(dec.inv, 4) == 2
        assert algebra.slp_additions(dec.alpha, 4) == 3
        assert algebra.slp_additions(dec.beta, 4) == 3
        assert algebra.slp_additions(dec.gamma, 7) == 6
    # Strassen-Winograd: 15 additions in total (section 2.1)
    sw = (algebra.slp_additions(algebra.sw_xi, 4) + algebra.slp_additions(algebra.sw_eta, 4)
          + algebra.slp_additions(algebra.sw_zeta, 7))
    assert sw == 15


@pytest.mark.parametrize("dec", [algebra.SELF_INVERSE, algebra.CHAINING,
                                 algebra.STRASSEN_WINOGRAD], ids=lambda d: d.name)
def test_exhaustive_one_level_2x2(dec):
    """All 256 pairs of 2x2 bit matrices: basis change, 7 products, inverse = AB."""
    for a, b in itertools.product(range(16), range(16)):
        A = np.array([[a & 1, (a >> 1) & 1], [(a >> 2) & 1, (a >> 3) & 1]], dtype=np.uint8)
        B = np.array([[b & 1, (b >> 1) & 1], [(b >> 2) & 1, (b >> 3) & 1]], dtype=np.uint8)
        C = strassen.product(A, B, 1, strassen.bits_leaf, dec)
        assert np.array_equal(C, brute.matmul(A, B)), (a, b)


def _count_core(e, dec):
    """Bit operations of the core recursion down to 1x1 leaves on 2^e x 2^e."""
    algebra.Counted.counter[0] = 0
    mults = [0]

    def rec(size, d):
        if d == 0:
            mults[0] += 1  # one bit multiplication (AND) at a 1x1 leaf
            return algebra.Counted(size)
        q = size // 4
        T = dec.alpha(*[algebra.Counted(q) for _ in range(4)])
        S = dec.beta(*[algebra.Counted(q) for _ in range(4)])
        Q = [rec(q, d - 1) for _ in range(7)]
        dec.gamma(*Q)
        return algebra.Counted(size)

    rec(4 ** e, e)
    return algebra.Counted.counter[0] + mults[0]


@pytest.mark.parametrize("e", range(0, 7))
def test_operation_counts_closed_form(e):
    """Section 1.1 and Theorem 1: 5 n^log2(7) - 4 n^2 bit operations in the
    alternative basis; 6 n^log2(7) - 5 n^2 for Strassen-Winograd."""
    n = 2 ** e
    assert _count_core(e, algebra.SELF_INVERSE) == 5 * 7 ** e - 4 * n * n
    assert _count_core(e, algebra.CHAINING) == 5 * 7 ** e - 4 * n * n
    assert _count_core(e, algebra.STRASSEN_WINOGRAD) == 6 * 7 ** e - 5 * n * n


@pytest.mark.parametrize("e", range(1, 8))
def test_basis_change_count(e):
    """Section 1.2: a basis change of an n x n matrix costs (1/2) n^2 log2 n."""
    n = 2 ** e
    for prog in (algebra.sinv_fwd, algebra.sinv_inv):
        algebra.Counted.counter[0] = 0

        def rec(size, d):
            if d == 0:
                return
            q = size // 4
            prog(*[algebra.Counted(q) for _ in range(4)])
            for _ in range(4):
                rec(q, d - 1)

        rec(n * n, e)
        assert algebra.Counted.counter[0] * 2 == n * n * e


def interleave_index(i, j, d):
    """Linear index of entry (i, j) of a 2^d x 2^d matrix in the interleaved
    layout i_1 j_1 i_2 j_2 ... (first-index-major, eq. a-interleaved)."""
    idx = 0
    for level in range(d):
        sh = d - 1 - level
        idx = idx * 4 + ((i >> sh) & 1) * 2 + ((j >> sh) & 1)
    return idx


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("name,prog", [("selfinv_phi", algebra.sinv_fwd),
                                       ("selfinv_chi", algebra.sinv_inv),
                                       ("chain_phi", algebra.chain_fwd),
                                       ("chain_chi", algebra.chain_inv)])
def test_recursive_basis_equals_kronecker(d, name, prog):
    """Section 2.6: per-level (Yates) application equals the Kronecker power,
    and the order of the levels does not matter."""
    M = golden(name)
    K = np.array([[1]], dtype=np.int64)
    for _ in range(d):
        K = np.kron(K, M)
    rng = np.random.default_rng(d)
    n = 2 ** d
    X = (rng.random((n, n)) < 0.5).astype(np.uint8)
    vec = np.zeros(n * n, dtype=np.int64)
    for i in range(n):
        for j in range(n):
            vec[interleave_index(i, j, d)] = X[i, j]
    want_vec = gf2(K @ vec)
    want = np.zeros_like(X)
    for i in range(n):
        for j in range(n):
            want[i, j] = want_vec[interleave_index(i, j, d)]
    assert np.array_equal(strassen.basis(X, d, prog), want)
    assert np.array_equal(strassen.basis(X, d, prog, bottom_up=True), want)


def test_self_inverse_basis_roundtrip_packed():
    rng = np.random.default_rng(12)
    X = rng.integers(0, 2 ** 63, size=(256, 8), dtype=np.int64).astype(np.uint64)
    for d in range(4):
        Y = strassen.basis(X, d, algebra.sinv_fwd)
        assert np.array_equal(strassen.basis(Y, d, algebra.sinv_fwd), X)
        Z = strassen.basis(X, d, algebra.sinv_inv)
        assert np.array_equal(strassen.basis(Z, d, algebra.sinv_inv), X)


@pytest.mark.parametrize("dec", [algebra.SELF_INVERSE, algebra.CHAINING,
                                 algebra.STRASSEN_WINOGRAD], ids=lambda d: d.name)
def test_recursion_rectangular_odd_leaves_bits(dec):
    """Multi-level recursion with rectangular blocks and odd leaf sizes reaches AB."""
    rng = np.random.default_rng(13)
    for d, (ml, kl, nl) in [(1, (3, 5, 7)), (2, (1, 3, 2)), (3, (3, 1, 5)), (4, (1, 1, 1))]:
        m, k, n = ml << d, kl << d, nl << d
        A = (rng.random((m, k)) < 0.5).astype(np.uint8)
        B = (rng.random((k, n)) < 0.5).astype(np.uint8)
        C = strassen.product(A, B, d, strassen.bits_leaf, dec)
        assert np.array_equal(C, brute.matmul(A, B)), (d, m, k, n)


def test_recursion_packed_matches_plain_product():
    """The stage oracles on packed words (quadrant splits on word boundaries)."""
    rng = np.random.default_rng(14)
    for d, m, k, n in [(1, 256, 128, 256), (2, 512, 256, 256), (3, 512, 512, 1024)]:
        A = rng.integers(0, 2 ** 63, size=(m, k // 64), dtype=np.int64).astype(np.uint64)
        B = rng.integers(0, 2 ** 63, size=(k, n // 64), dtype=np.int64).astype(np.uint64)
        A ^= rng.integers(0, 2, size=A.shape, dtype=np.int64).astype(np.uint64) << np.uint64(63)
        want = oracle.mul(A, B, k, n, oracle.GF2)
        got = strassen.product(A, B, d, strassen.packed_leaf(k, n))
        assert np.array_equal(got, want), (d, m, k, n)


def test_stage_oracles_single_level_formulas():
    """One expansion/compression level on packed blocks equals the recurrences
    entry by entry (eqs. mb-tsrecurrence, mb-qrecurrence)."""
    rng = np.random.default_rng(15)
    X = rng.integers(0, 2 ** 62, size=(128, 4), dtype=np.int64).astype(np.uint64)
    q = strassen.quadrants(X)
    T = strassen.expand_left(X)
    S = strassen.expand_right(X)
    assert np.array_equal(T[4], q[0] ^ q[3]) and np.array_equal(T[6], q[2] ^ q[3])
    assert np.array_equal(S[1], q[2]) and np.array_equal(S[2], q[0] ^ q[3])
    Q = [rng.integers(0, 2 ** 62, size=(64, 2), dtype=np.int64).astype(np.uint64)
         for _ in range(7)]
    C = strassen.compress(Q)
    cq = strassen.quadrants(C)
    assert np.array_equal(cq[3], Q[1] ^ Q[3] ^ Q[5] ^ Q[6])
    assert np.array_equal(cq[1], Q[4] ^ Q[6])


def test_strassen_beats_cubic_bit_ops_from_512():
    """Section 1.1: Strassen-Winograd needs n >= 512 to use fewer bit operations
    than the elementary algorithm (2 n^3 - n^2)."""
    def sw(n):
        return 6 * n ** math.log2(7) - 5 * n * n

    def cubic(n):
        return 2 * n ** 3 - n * n
    assert sw(256) > cubic(256)
    assert sw(512) < cubic(512)
