"""Pins of the plain-definition oracle (packed triple loop) against brute force,
invariants and closed forms.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import brute

SIZES = [1, 2, 3, 63, 64, 65, 127, 128, 129, 200]
SEMIRINGS = [(oracle.GF2, False), (oracle.BOOLEAN, True)]


def rand_bits(rng, r, c, p=0.5):
    return (rng.random((r, c)) < p).astype(np.uint8)


def omul(A_bits, B_bits, sr):
    k = A_bits.shape[1]
    n = B_bits.shape[1]
    C = oracle.mul(brute.pack(A_bits), brute.pack(B_bits), k, n, sr)
    return brute.unpack(C, n)


def test_pack_roundtrip():
    rng = np.random.default_rng(0)
    for c in [1, 63, 64, 65, 130]:
        X = rand_bits(rng, 5, c)
        P = brute.pack(X)
        assert P.shape == (5, (c + 63) // 64)
        assert np.array_equal(brute.unpack(P, c), X)
        # LSB-first: column j is bit j % 64 of word j // 64
        for j in range(c):
            assert ((int(P[0, j // 64]) >> (j % 64)) & 1) == X[0, j]


def test_tiny_loops_match_matmul():
    rng = np.random.default_rng(1)
    for m, k, n in [(1, 1, 1), (2, 3, 4), (5, 7, 3), (8, 9, 10)]:
        A = rand_bits(rng, m, k)
        B = rand_bits(rng, k, n)
        for _, boolean in SEMIRINGS:
            assert np.array_equal(brute.loops(A, B, boolean), brute.matmul(A, B, boolean))


@pytest.mark.parametrize("sr,boolean", SEMIRINGS)
def test_oracle_vs_brute_sizes(sr, boolean):
    rng = np.random.default_rng(2)
    for m in SIZES:
        for k in SIZES[::3]:
            for n in SIZES[1::3]:
                p = 0.5 if not boolean else min(0.5, 1.0 / np.sqrt(k) + 0.05)
                A = rand_bits(rng, m, k, p)
                B = rand_bits(rng, k, n, p)
                assert np.array_equal(omul(A, B, sr), brute.matmul(A, B, boolean)), (m, k, n)


@pytest.mark.parametrize("sr,boolean", SEMIRINGS)
def test_oracle_vs_triple_loop(sr, boolean):
    rng = np.random.default_rng(3)
    for m, k, n in [(3, 70, 5), (9, 64, 66), (4, 129, 2)]:
        A = rand_bits(rng, m, k)
        B = rand_bits(rng, k, n)
        assert np.array_equal(omul(A, B, sr), brute.loops(A, B, boolean))


@pytest.mark.parametrize("sr,boolean", SEMIRINGS)
def test_identity_zero_permutation(sr, boolean):
    rng = np.random.default_rng(4)
    m, k, n = 70, 130, 90
    A = rand_bits(rng, m, k)
    B = rand_bits(rng, k, n)
    assert np.array_equal(omul(A, np.eye(k, dtype=np.uint8), sr), A)
    assert np.array_equal(omul(np.eye(k, dtype=np.uint8), B, sr), B)
    assert not omul(np.zeros((m, k), np.uint8), B, sr).any()
    assert not omul(A, np.zeros((k, n), np.uint8), sr).any()
    pr = rng.permutation(m)
    Pm = np.eye(m, dtype=np.uint8)[pr]
    assert np.array_equal(omul(Pm, A, sr), A[pr])
    pc = rng.permutation(k)
    Pk = np.eye(k, dtype=np.uint8)[:, pc]
    assert np.array_equal(omul(A, Pk, sr), A[:, pc])


@pytest.mark.parametrize("sr,boolean", SEMIRINGS)
def test_associativity(sr, boolean):
    rng = np.random.default_rng(5)
    A = rand_bits(rng, 40, 70, 0.2)
    B = rand_bits(rng, 70, 65, 0.2)
    C = rand_bits(rng, 65, 130, 0.2)
    assert np.array_equal(omul(omul(A, B, sr), C, sr), omul(A, omul(B, C, sr), sr))


def test_gf2_bilinearity_and_transpose():
    rng = np.random.default_rng(6)
    A = rand_bits(rng, 50, 77)
    A2 = rand_bits(rng, 50, 77)
    B = rand_bits(rng, 77, 66)
    B2 = rand_bits(rng, 77, 66)
    g = oracle.GF2
    assert np.array_equal(omul(A, B ^ B2, g), omul(A, B, g) ^ omul(A, B2, g))
    assert np.array_equal(omul(A ^ A2, B, g), omul(A, B, g) ^ omul(A2, B, g))
    for sr in (oracle.GF2, oracle.BOOLEAN):
        assert np.array_equal(omul(A, B, sr).T, omul(B.T.copy(), A.T.copy(), sr))


def test_boolean_dominates_gf2():
    rng = np.random.default_rng(7)
    A = rand_bits(rng, 64, 200)
    B = rand_bits(rng, 200, 100)
    cg = omul(A, B, oracle.GF2)
    cb = omul(A, B, oracle.BOOLEAN)
    assert not (cg & (1 - cb)).any()


def test_closed_forms_all_ones_and_single_bit():
    rng = np.random.default_rng(8)
    A = rand_bits(rng, 33, 150, 0.05)
    A[3] = 0
    ones = np.ones((150, 70), dtype=np.uint8)
    cb = omul(A, ones, oracle.BOOLEAN)
    cg = omul(A, ones, oracle.GF2)
    nz = (A.sum(axis=1) > 0).astype(np.uint8)
    par = (A.sum(axis=1) & 1).astype(np.uint8)
    assert np.array_equal(cb, np.repeat(nz[:, None], 70, axis=1))
    assert np.array_equal(cg, np.repeat(par[:, None], 70, axis=1))
    B = rand_bits(rng, 150, 70)
    E = np.zeros((1, 150), dtype=np.uint8)
    E[0, 97] = 1
    for sr in (oracle.GF2, oracle.BOOLEAN):
        assert np.array_equal(omul(E, B, sr)[0], B[97])


def test_rows_matches_full_and_padding():
    rng = np.random.default_rng(9)
    m, k, n = 100, 300, 190
    A = brute.pack(rand_bits(rng, m, k))
    B = brute.pack(rand_bits(rng, k, n))
    for sr in (oracle.GF2, oracle.BOOLEAN):
        full = oracle.mul(A, B, k, n, sr)
        sel = [0, 17, 99]
        part = oracle.rows(A[sel], B, k, n, sr)
        assert np.array_equal(part, full[sel])
        # padding bits of the last word stay zero
        assert not (full[:, -1] >> np.uint64(n % 64)).any()


def test_freivalds_accepts_right_and_catches_planted_error():
    rng = np.random.default_rng(10)
    m, k, n = 130, 200, 150
    A = brute.pack(rand_bits(rng, m, k))
    B = brute.pack(rand_bits(rng, k, n))
    C = oracle.mul(A, B, k, n, oracle.GF2)
    xs = [brute.pack(rand_bits(rng, 1, m))[0] for _ in range(24)]
    assert all(oracle.freivalds(A, B, C, m, k, n, xs))
    bad = C.copy()
    bad[77, 1] ^= np.uint64(1 << 5)  # one wrong bit
    res = oracle.freivalds(A, B, bad, m, k, n, xs)
    assert not all(res)
    # a vector catches the error exactly when it selects row 77
    for x, ok in zip(xs, res):
        assert ok == (((int(x[1]) >> (77 - 64)) & 1) == 0)


def test_vecmat_matches_product_row():
    rng = np.random.default_rng(11)
    M = rand_bits(rng, 90, 140)
    x = rand_bits(rng, 1, 90)
    y = oracle.vecmat(brute.pack(x)[0], brute.pack(M), 90, 140)
    assert np.array_equal(brute.unpack(y[None, :], 140)[0], brute.matmul(x, M)[0])
