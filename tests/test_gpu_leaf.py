"""GPU parity of the cubic leaves (VALU bitop3 and int8 MFMA) against the
oracle's plain product, bit-exact, through the C ABI."""
import numpy as np
import pytest

import bmmgen
import oracle
from gpu_util import announce, empty_dev, from_dev, to_dev, words

pytestmark = pytest.mark.gpu

SEMIRINGS = [("gf2", oracle.GF2), ("bool", oracle.BOOLEAN)]
LEAVES = [("valu", 1, 1), ("mfma128x64", 2, 1), ("mfma64x64", 2, 2), ("mfma64x128", 2, 3),
          ("mfma64x32", 2, 4), ("mfma_lds256", 2, 5), ("mfma_deep128x64", 2, 6),
          ("mfma_chunk64x128", 2, 7), ("mfma_lds4_256x128", 2, 8),
          ("f4_128x64", 3, 1), ("f4_64x64", 3, 2), ("f4_64x128", 3, 3), ("f4_64x32", 3, 4),
          ("f4_lds256", 3, 5), ("f4_deep128x64", 3, 6), ("f4_chunk64x128", 3, 7),
          ("f4_lds4_256x128", 3, 8),
          ("valu_outer", 1, 2)]  # VALU outer-product form: B row-major


@pytest.fixture(scope="module")
def bmm():
    import paper_1909_01554_amd as bmm
    return bmm


def gen(rows, cols, seed, tag, p=None):
    dist = bmmgen.Dist.half() if p is None else p
    return bmmgen.fill_cpu(rows, cols, seed, tag, dist)


def run(bmm, sr, leaf, tile, A, B, m, k, n, b_t=False, acc_init=None, pad=0, k_panel=0):
    opts = bmm.Options(leaf=leaf, tile=tile, k_panel=k_panel)
    Ad = to_dev(A, A.shape[1] + pad)
    if b_t:
        BT = oracle_transpose(B, k, n)
        Bd = to_dev(BT, BT.shape[1] + pad)
    else:
        Bd = to_dev(B, B.shape[1] + pad)
    if acc_init is None:
        Cd = empty_dev(m, words(n) + pad, fill=-1)
    else:
        Cd = to_dev(acc_init, words(n) + pad)
    fn = bmm.bmm_gf2 if sr == oracle.GF2 else bmm.bmm_boolean
    fn(Ad, Bd, Cd, m, k, n, options=opts, b_transposed=b_t, accumulate=acc_init is not None)
    return from_dev(Cd, words(n))


def oracle_transpose(B, k, n):
    from oracle import brute
    return brute.pack(brute.unpack(B, n).T.copy())


@pytest.mark.parametrize("sname,sr", SEMIRINGS)
@pytest.mark.parametrize("lname,leaf,tile", LEAVES)
def test_config1_2048_full(bmm, sname, sr, lname, leaf, tile):
    """2048 x 2048 x 2048, Bernoulli(1/2), full C compared bit for bit."""
    n = 2048
    seed = bmmgen.config_seed(0)
    A = gen(n, n, seed, bmmgen.TAG_A)
    B = gen(n, n, seed, bmmgen.TAG_B)
    announce("config1", sname, lname)
    got = run(bmm, sr, leaf, tile, A, B, n, n, n)
    want = oracle.mul(A, B, n, n, sr)
    assert np.array_equal(got, want)


RAGGED = [(1, 1, 1), (1, 64, 1), (3, 65, 2), (33, 70, 65), (100, 300, 129), (257, 1000, 200),
          (128, 4096, 64), (130, 129, 33), (64, 8192, 96), (300, 64, 300), (192, 6080, 160),
          (70, 3840, 130),
          # k = 2048 with unpadded pitches (entries 12 and 15): the recursion's leaf length,
          # with an odd number of 64-column wave tiles
          (130, 2048, 130), (64, 4096, 200), (200, 2048, 70), (250, 2048, 260)]


@pytest.mark.parametrize("sname,sr", SEMIRINGS)
@pytest.mark.parametrize("lname,leaf,tile", LEAVES)
def test_ragged_shapes(bmm, sname, sr, lname, leaf, tile):
    for i, (m, k, n) in enumerate(RAGGED):
        p = None if sr == oracle.GF2 else bmmgen.Dist.inv_sqrt(k)
        A = gen(m, k, 11 + i, bmmgen.TAG_A, p)
        B = gen(k, n, 11 + i, bmmgen.TAG_B, p)
        announce("ragged", sname, lname, (m, k, n))
        got = run(bmm, sr, leaf, tile, A, B, m, k, n, pad=i % 3)
        assert np.array_equal(got, oracle.mul(A, B, k, n, sr)), (m, k, n)


@pytest.mark.parametrize("sname,sr", SEMIRINGS)
@pytest.mark.parametrize("lname,leaf,tile", LEAVES)
def test_transposed_b_and_accumulate(bmm, sname, sr, lname, leaf, tile):
    """B passed transposed, and C accumulated into, with odd and even C pitches (5 and 6
    words: the 128-column tiles store 16-byte pieces only where a row starts 16-byte
    aligned, and the last tile's single word alone)."""
    m, k, n = 200, 777, 300
    A = gen(m, k, 5, bmmgen.TAG_A)
    B = gen(k, n, 5, bmmgen.TAG_B)
    C0 = gen(m, n, 5, 0xC0)
    want = oracle.mul(A, B, k, n, sr)
    announce("b_t", sname, lname)
    assert np.array_equal(run(bmm, sr, leaf, tile, A, B, m, k, n, b_t=True), want)
    for pad in (0, 1):
        announce("accumulate", sname, lname, pad)
        got = run(bmm, sr, leaf, tile, A, B, m, k, n, acc_init=C0, pad=pad)
        assert np.array_equal(got, (want ^ C0) if sr == oracle.GF2 else (want | C0))


# (m, k, n, panel bits): one-word panels, odd-word panels (8-byte loads after the
# first), the recursion's 2048-bit panels, a panel rounded up to whole words (3000 ->
# 3008), and a ragged last panel
KPANEL = [(64, 300, 130, 64), (100, 1000, 70, 128), (130, 4096, 200, 2048),
          (70, 777, 300, 192), (33, 8192, 65, 3000), (200, 5000, 128, 4096)]


@pytest.mark.parametrize("sname,sr", SEMIRINGS)
@pytest.mark.parametrize("lname,leaf,tile", [LEAVES[0], LEAVES[1], LEAVES[7], LEAVES[9],
                                             LEAVES[8], LEAVES[6], LEAVES[17]])
def test_k_panels(bmm, sname, sr, lname, leaf, tile):
    """C as the sum of panel products over k (each panel's product XORed / ORed into C
    after the first), fresh and accumulated, against the oracle's plain product."""
    for i, (m, k, n, kp) in enumerate(KPANEL):
        p = None if sr == oracle.GF2 else bmmgen.Dist.inv_sqrt(k)
        A = gen(m, k, 31 + i, bmmgen.TAG_A, p)
        B = gen(k, n, 31 + i, bmmgen.TAG_B, p)
        want = oracle.mul(A, B, k, n, sr)
        announce("k panels", sname, lname, (m, k, n, kp))
        assert np.array_equal(run(bmm, sr, leaf, tile, A, B, m, k, n, k_panel=kp,
                                  b_t=i % 2 == 1), want), (m, k, n, kp)
        C0 = gen(m, n, 31 + i, 0xC0)
        got = run(bmm, sr, leaf, tile, A, B, m, k, n, acc_init=C0, k_panel=kp)
        assert np.array_equal(got, (want ^ C0) if sr == oracle.GF2 else (want | C0)), kp


@pytest.mark.parametrize("sname,sr", SEMIRINGS)
def test_valu_outer_wide_shapes(bmm, sname, sr):
    """The VALU leaf's outer-product form on shapes that span whole 512 x 1024 tiles and
    ragged last ones, and k within one 64-row stage of B, over several, odd, and ending one
    row into a stage; B given row-major (read where it lies) and transposed (transposed
    back into scratch), fresh and accumulated."""
    for i, (m, k, n) in enumerate([(600, 777, 1100), (1025, 2048, 2048), (64, 64, 1024),
                                   (2100, 100, 2100), (40, 3000, 1088), (300, 1, 70),
                                   (130, 129, 3000), (2048, 63, 64)]):
        p = None if sr == oracle.GF2 else bmmgen.Dist.inv_sqrt(k)
        A = gen(m, k, 51 + i, bmmgen.TAG_A, p)
        B = gen(k, n, 51 + i, bmmgen.TAG_B, p)
        want = oracle.mul(A, B, k, n, sr)
        announce("valu outer", sname, (m, k, n))
        assert np.array_equal(run(bmm, sr, 1, 2, A, B, m, k, n, pad=i % 2), want), (m, k, n)
        assert np.array_equal(run(bmm, sr, 1, 2, A, B, m, k, n, b_t=True), want), (m, k, n)
        C0 = gen(m, n, 51 + i, 0xC0)
        got = run(bmm, sr, 1, 2, A, B, m, k, n, acc_init=C0, pad=1)
        assert np.array_equal(got, (want ^ C0) if sr == oracle.GF2 else (want | C0)), (m, k, n)


def test_k_zero_and_empty(bmm):
    Cd = empty_dev(5, 2, fill=-1)
    Ad = empty_dev(5, 1)
    Bd = empty_dev(1, 2)
    announce("k=0")
    bmm.bmm_gf2(Ad, Bd, Cd, 5, 0, 100)
    assert not from_dev(Cd).any()
    bmm.bmm_boolean(Ad, Bd, Cd, 0, 10, 100)  # m = 0: nothing to do
    bmm.bmm_boolean(Ad, Bd, Cd, 5, 10, 0)


def test_padding_bits_written_zero(bmm):
    m, k, n = 70, 100, 33
    A = gen(m, k, 9, bmmgen.TAG_A)
    B = gen(k, n, 9, bmmgen.TAG_B)
    for leaf, tile in [(1, 1), (1, 2), (2, 1), (2, 4)]:
        announce("padding", leaf, tile)
        got = run(bmm, oracle.BOOLEAN, leaf, tile, A, B, m, k, n)
        assert not (got[:, 0] >> np.uint64(33)).any()


def test_errors(bmm):
    import ctypes
    A = empty_dev(8, 2)
    B = empty_dev(128, 2)
    C = empty_dev(8, 2)
    # the binding refuses a tensor smaller than the sizes claim before the ABI call
    with pytest.raises(ValueError):
        bmm.bmm_gf2(A, B, C, 8, 200, 128)
    # the C side refuses the pitch on its own (raw ABI call: lda 2 < 4 words)
    o = bmm.Options()
    vp = ctypes.c_void_p
    rc = bmm._c_gf2(vp(A.data_ptr()), 2, vp(B.data_ptr()), 2, vp(C.data_ptr()), 2, 8, 200, 128,
                    ctypes.byref(o), None)
    assert rc == -1
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_gf2(A, B, A, 8, 128, 128)  # C overlaps A
    assert e.value.status == -1
    with pytest.raises(ValueError):
        bmm.bmm_gf2(A, B, C, -1, 128, 128)


def test_generator_gpu_matches_cpu():
    import torch
    for dist in [bmmgen.Dist.half(), bmmgen.Dist.pow2(3), bmmgen.Dist.inv_sqrt(500)]:
        t = torch.zeros((37, 6), dtype=torch.int64, device="cuda")
        announce("generator", dist)
        bmmgen.fill_tensor(t, 37, 300, 123, 0xB, dist, row0=5)
        got = from_dev(t)
        want = bmmgen.fill_cpu(37, 300, 123, 0xB, dist, row0=5, nwords=6, ld=6)
        assert np.array_equal(got, want)
