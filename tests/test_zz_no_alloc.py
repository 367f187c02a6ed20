"""The cubic product entry point that allocates nothing (bmm_cubic_noalloc),
through the C ABI, against the allocating entry points (bmm_gf2, bmm_boolean)
and the oracle, bit for bit: two calls in a row on one device, the second with
a smaller input (the fixed scratch array keeps the first call's contents)."""
import numpy as np
import pytest

import bmmgen
import oracle
from gpu_util import announce, empty_dev, from_dev, to_dev, words

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bmm():
    import paper_1909_01554_amd as bmm
    return bmm


def operands(m, k, n, seed, sr):
    dist = bmmgen.Dist.half() if sr == oracle.GF2 else bmmgen.Dist.inv_sqrt(k)
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, dist)
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, dist)
    return A, B


def both(bmm, sr, A, B, m, k, n, **kw):
    """(no-allocation result, allocating entry point's result) on the same operands."""
    Ad, Bd = to_dev(A), to_dev(B)
    C1 = empty_dev(m, words(n), fill=-1)
    C2 = empty_dev(m, words(n), fill=-1)
    announce("noalloc", sr, (m, k, n), kw)
    bmm.bmm_cubic_noalloc(sr, Ad, Bd, C1, m, k, n, **kw)
    ref = bmm.bmm_gf2 if sr == oracle.GF2 else bmm.bmm_boolean
    ref(Ad, Bd, C2, m, k, n, **kw)
    return from_dev(C1), from_dev(C2)


@pytest.mark.parametrize("sr", [oracle.GF2, oracle.BOOLEAN])
def test_two_calls_second_smaller(bmm, sr):
    for i, (m, k, n) in enumerate([(300, 5000, 700), (70, 1000, 130)]):
        A, B = operands(m, k, n, 31 + i, sr)
        got, ref = both(bmm, sr, A, B, m, k, n)
        want = oracle.mul(A, B, k, n, sr)
        assert np.array_equal(got, ref), (m, k, n)
        assert np.array_equal(got, want), (m, k, n)


@pytest.mark.parametrize("sr", [oracle.GF2, oracle.BOOLEAN])
def test_leaf_kinds_and_accumulate(bmm, sr):
    m, k, n = 200, 3000, 260
    A, B = operands(m, k, n, 7, sr)
    want = oracle.mul(A, B, k, n, sr)
    for leaf in (1, 2, 3):
        got, ref = both(bmm, sr, A, B, m, k, n, options=bmm.Options(leaf=leaf))
        assert np.array_equal(got, ref) and np.array_equal(got, want), leaf
    C0 = bmmgen.fill_cpu(m, n, 7, 0xC0, bmmgen.Dist.half())
    Cd = to_dev(C0)
    bmm.bmm_cubic_noalloc(sr, to_dev(A), to_dev(B), Cd, m, k, n, accumulate=True)
    assert np.array_equal(from_dev(Cd), (want ^ C0) if sr == oracle.GF2 else (want | C0))
    # B given transposed: no scratch at all
    BT = bmmgen.fill_cpu(n, k, 8, 0xB7, bmmgen.Dist.half())
    Cd = empty_dev(m, words(n), fill=-1)
    bmm.bmm_cubic_noalloc(sr, to_dev(A), to_dev(BT), Cd, m, k, n, b_transposed=True)
    Cr = empty_dev(m, words(n), fill=-1)
    (bmm.bmm_gf2 if sr == oracle.GF2 else bmm.bmm_boolean)(to_dev(A), to_dev(BT), Cr, m, k, n,
                                                           b_transposed=True)
    assert np.array_equal(from_dev(Cd), from_dev(Cr))


def test_largest_scratch_then_smaller(bmm):
    """B^T exactly fills the array (n * words(k) * 8 = 32 MiB), then a ragged
    smaller product; one byte more is refused before any device work."""
    sr = oracle.GF2
    m, k, n = 128, 32768, 8192
    assert n * words(k) * 8 == bmm.NOALLOC_SCRATCH_BYTES
    A, B = operands(m, k, n, 3, sr)
    got, ref = both(bmm, sr, A, B, m, k, n)
    assert np.array_equal(got, ref)
    rows = [0, 57, 127]
    assert np.array_equal(got[rows], oracle.rows(A[rows], B, k, n, sr))
    m2, k2, n2 = 65, 4097, 333
    A2, B2 = operands(m2, k2, n2, 4, oracle.BOOLEAN)
    got2, ref2 = both(bmm, oracle.BOOLEAN, A2, B2, m2, k2, n2)
    assert np.array_equal(got2, ref2)
    assert np.array_equal(got2, oracle.mul(A2, B2, k2, n2, oracle.BOOLEAN))
    Ad, Bd = to_dev(A[:, :words(k)]), to_dev(np.zeros((k, words(n + 1)), np.uint64))
    Cd = empty_dev(m, words(n + 1))
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_cubic_noalloc(sr, Ad, Bd, Cd, m, k, n + 64)
    assert e.value.status == -2
