"""GPU parity of the alternative-basis recursion: every stage kernel against
the oracle's stage function, and the whole product against the plain product."""
import numpy as np
import pytest

import bmmgen
import oracle
from oracle import algebra, strassen
from gpu_util import announce, empty_dev, from_dev, to_dev, words

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bmm():
    import paper_1909_01554_amd as bmm
    return bmm


def rand_words(rows, nwords, seed):
    return bmmgen.fill_cpu(rows, nwords * 64, seed, 0x77, bmmgen.Dist.half())


@pytest.mark.parametrize("rows,cols", [(1, 1), (64, 64), (65, 130), (200, 1000), (128, 4096),
                                       (1000, 70)])
def test_transpose(bmm, rows, cols):
    from oracle import brute
    X = bmmgen.fill_cpu(rows, cols, rows + cols, 0x11, bmmgen.Dist.half())
    Xd = to_dev(X)
    Td = empty_dev(cols, words(rows) + 1, fill=-1)
    announce("transpose", rows, cols)
    bmm.bmm_transpose(Xd, Td, rows, cols)
    got = from_dev(Td, words(rows))
    want = brute.pack(brute.unpack(X, cols).T.copy())
    assert np.array_equal(got, want)


DECS = [algebra.SELF_INVERSE, algebra.CHAINING, algebra.STRASSEN_WINOGRAD]


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 5, 6, 7])
@pytest.mark.parametrize("inverse", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_basis_change(bmm, depth, inverse, scheme):
    rows, nw = 3 << depth, 2 << depth  # odd leaf rows, two-word leaf rows
    X = rand_words(rows, nw, depth)
    Xd = to_dev(X, nw + 3)
    announce("basis", depth, inverse, scheme)
    bmm.bmm_basis_change(Xd, rows, nw, depth, inverse=bool(inverse), scheme=scheme)
    got = from_dev(Xd, nw)
    dec = DECS[scheme]
    prog = dec.inv if inverse else dec.fwd
    assert np.array_equal(got, strassen.basis(X, depth, prog))


@pytest.mark.parametrize("depth", [1, 3, 6])
@pytest.mark.parametrize("inverse", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1])
def test_basis_change_transposed(bmm, depth, inverse, scheme):
    """On a matrix stored transposed, the forward (and the inverse) change equals the
    transpose of the change applied to the matrix itself.  The chaining programs are
    not symmetric in the 01 and 10 quadrants, so this checks the transposed
    instantiation of each direction."""
    from oracle import brute
    rows, nw = 3 << depth, 2 << depth
    cols = 64 * nw
    Xs = rand_words(rows, nw, 70 + depth + 10 * inverse)  # stored: X^T, rows x cols bits
    Xd = to_dev(Xs)
    announce("basis transposed", depth, inverse, scheme)
    bmm.bmm_basis_change(Xd, rows, nw, depth, inverse=bool(inverse), scheme=scheme,
                         transposed=True)
    B = brute.unpack(Xs, cols).T.copy()  # cols x rows bits
    prog = DECS[scheme].inv if inverse else DECS[scheme].fwd
    want = brute.pack(strassen.basis(B, depth, prog).T.copy())
    assert np.array_equal(from_dev(Xd), want)


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_expand(bmm, side, levels, scheme):
    rows, nw, parents = 24, 8, 3
    X = rand_words(rows * parents, nw, 40 + side + levels)
    Xd = to_dev(X, nw + 2)  # pitch nw + 2, parents stacked with stride rows * pitch
    ch = 7 ** levels
    sub_r, sub_w = rows >> levels, nw >> levels
    Dd = empty_dev(parents * ch * sub_r, sub_w, fill=-1)
    announce("expand", side, levels, scheme)
    bmm.bmm_expand(side, levels, Xd, nw + 2, rows * (nw + 2), Dd, rows, nw, parents,
                   scheme=scheme)
    got = from_dev(Dd).reshape(parents, ch, sub_r, sub_w)
    for p in range(parents):
        par = X[p * rows:(p + 1) * rows]
        if side == 1:
            # stored transposed: expand the real B (transpose of the stored words'
            # quadrant grid) and compare quadrant-transposed children
            want = expand_transposed(par, levels, DECS[scheme])
        else:
            want = expand_plain(par, levels, DECS[scheme])
        for h in range(ch):
            assert np.array_equal(got[p, h], want[h]), (p, h)


def expand_plain(X, levels, dec):
    kids = strassen.expand_left(X, dec)
    if levels == 1:
        return kids
    return [g for c in kids for g in strassen.expand_left(c, dec)]


def swap_quadrants(X):
    q = strassen.quadrants(X)
    return strassen.assemble(q[0], q[2], q[1], q[3])


def expand_transposed(X, levels, dec):
    """Right-operand expansion on transposed storage at the level of quadrant
    blocks: the stored block (a, b) is B's block (b, a) transposed; children
    of the stored matrix are the stored forms of beta's children."""
    def one(Y):
        # view stored quadrants as B's quadrants: B00=Y00, B01=Y10, B10=Y01, B11=Y11
        q = strassen.quadrants(Y)
        return [np.ascontiguousarray(t) for t in dec.beta(q[0], q[2], q[1], q[3])]
    kids = one(X)
    if levels == 1:
        return kids
    return [g for c in kids for g in one(c)]


@pytest.mark.parametrize("levels", [1, 2])
@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_compress(bmm, levels, scheme):
    rows, nw, parents = 16, 8, 2
    ch = 7 ** levels
    sub_r, sub_w = rows >> levels, nw >> levels
    Q = rand_words(parents * ch * sub_r, sub_w, 90 + levels)
    Qd = to_dev(Q)
    Pd = empty_dev(parents * rows, nw + 1, fill=-1)
    announce("compress", levels, scheme)
    bmm.bmm_compress(levels, Qd, Pd, nw + 1, rows * (nw + 1), rows, nw, parents, scheme=scheme)
    dec = DECS[scheme]
    got = from_dev(Pd, nw).reshape(parents, rows, nw)
    Qs = Q.reshape(parents, ch, sub_r, sub_w)
    for p in range(parents):
        if levels == 1:
            want = strassen.compress([Qs[p, h] for h in range(7)], dec)
        else:
            mids = [strassen.compress([Qs[p, 7 * h1 + h2] for h2 in range(7)], dec)
                    for h1 in range(7)]
            want = strassen.compress(mids, dec)
        assert np.array_equal(got[p], want)


CASES = [  # m, k, n, depth, depth_serial
    (512, 512, 512, 1, 0), (512, 512, 512, 3, 0), (1024, 1024, 1024, 4, 1),
    (2048, 2048, 2048, 3, 1), (2048, 2048, 2048, 5, 2), (1024, 2048, 512, 2, 1),
    (768, 1536, 1024, 1, 1), (4096, 4096, 4096, 6, 2), (2048, 2048, 2048, 0, 0),
]


@pytest.mark.parametrize("m,k,n,depth,ds", CASES)
@pytest.mark.parametrize("leaf", [1, 2])
def test_strassen_product(bmm, m, k, n, depth, ds, leaf):
    seed = bmmgen.config_seed(2) + m + depth
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    opts = bmm.Options(leaf=leaf, depth_serial=ds, depth_parallel=depth - ds)
    nbytes, s_, p_ = bmm.bmm_gf2_strassen_workspace(m, k, n, depth, opts)
    assert (s_, p_) == (ds, depth - ds)
    import torch
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Ad, Bd = to_dev(A), to_dev(B)
    Cd = empty_dev(m, words(n) + 1, fill=-1)
    announce("strassen", m, k, n, depth, ds, leaf)
    bmm.bmm_gf2_strassen(Ad, Bd, Cd, m, k, n, ws, depth=depth, options=opts)
    got = from_dev(Cd, words(n))
    assert np.array_equal(got, oracle.mul(A, B, k, n, oracle.GF2))
    # inputs untouched
    assert np.array_equal(from_dev(Ad), A) and np.array_equal(from_dev(Bd), B)


SHIFT_CASES = [  # m, k, n, depth, depth_serial: leaves of k = 2048 or 4096 bits
    (4096, 4096, 4096, 1, 0),     # the parent is the whole (staged) operand, Q is C
    (8192, 8192, 8192, 2, 0),     # one expanded level above the shifted one
    (8192, 8192, 8192, 2, 1),     # parents are the serial level's children
    (4000, 4096, 2048, 1, 0),     # child rows 2000: a ragged last row tile
    (4096, 8192, 2048, 1, 0),     # leaves of k = 4096
    (8192, 16384, 4096, 3, 1),    # rectangular, serial + merged parallel levels
]


@pytest.mark.parametrize("m,k,n,depth,ds", SHIFT_CASES)
@pytest.mark.parametrize("shift", [1, 2])
@pytest.mark.parametrize("scheme", [0, 1])
def test_strassen_shifted_leaf(bmm, m, k, n, depth, ds, shift, scheme):
    """The last parallel level inside the int8 leaf (section 3.15): every parent's
    seven products formed from its quadrants in registers and combined in LDS reach
    AB exactly, with 16-byte (shift 1) and 8-byte (shift 2) operand loads."""
    import torch
    seed = 300 + m + k + depth + 7 * shift + scheme
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    opts = bmm.Options(leaf=2, depth_serial=ds, depth_parallel=depth - ds, scheme=scheme,
                       shift=shift)
    plain = bmm.Options(leaf=2, depth_serial=ds, depth_parallel=depth - ds, scheme=scheme,
                        shift=0)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, depth, opts)
    assert nbytes < bmm.bmm_gf2_strassen_workspace(m, k, n, depth, plain)[0]
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Cd = empty_dev(m, words(n) + 1, fill=-1)
    announce("strassen shifted leaf", m, k, n, depth, ds, shift, scheme)
    bmm.bmm_gf2_strassen(to_dev(A), to_dev(B), Cd, m, k, n, ws, depth=depth, options=opts)
    got = from_dev(Cd, words(n))
    if m * k * n <= 8192 ** 3:
        assert np.array_equal(got, oracle.mul(A, B, k, n, oracle.GF2))
    else:
        rows = bmmgen.stratified_rows(m, 256, seed)
        assert np.array_equal(got[rows], oracle.rows(A[rows], B, k, n, oracle.GF2))
        X = bmmgen.freivalds_vectors(m, 4, seed)
        assert all(oracle.freivalds(A, B, got, m, k, n, X))


@pytest.mark.parametrize("scheme", [0, 1, 2])
@pytest.mark.parametrize("alt", [False, True])
def test_strassen_shifted_leaf_accumulate_inplace(bmm, scheme, alt):
    """The shifted leaf accumulating into C (standard and alternative basis), on
    operands changed in place with odd pitches (8-byte loads).  Winograd has no
    shifted leaf: the option falls back to the plain one."""
    import torch
    from oracle import brute
    m, k, n, d = 4096, 8192, 4096, 1  # one level: the parent is the caller's operand
    seed = 41 + scheme + (9 if alt else 0)
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    C0 = bmmgen.fill_cpu(m, n, seed, 0xC, bmmgen.Dist.half())
    dec = DECS[scheme]
    if alt:
        A = strassen.basis(A, d, dec.fwd)
        B = strassen.basis(B, d, dec.fwd)
        prod = strassen.core(A, B, d, strassen.packed_leaf(k >> d, n >> d), dec)
    else:
        prod = oracle.mul(A, B, k, n, oracle.GF2)
    BT = brute.pack(brute.unpack(B, n).T.copy())
    opts = bmm.Options(leaf=2, depth_serial=0, depth_parallel=d, scheme=scheme, shift=1)
    kw = dict(b_transposed=True, alt_basis_io=alt, inplace_basis=not alt)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, d, opts, **kw)
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Ad, Bd, Cd = to_dev(A, words(k) + 1), to_dev(BT, words(k) + 1), to_dev(C0)
    announce("strassen shifted accumulate", scheme, alt)
    bmm.bmm_gf2_strassen(Ad, Bd, Cd, m, k, n, ws, depth=d, options=opts, accumulate=True, **kw)
    assert np.array_equal(from_dev(Cd), C0 ^ prod)
    assert np.array_equal(from_dev(Ad, words(k)), A)
    assert np.array_equal(from_dev(Bd, words(k)), BT)


@pytest.mark.parametrize("leaf", [2, 3])
@pytest.mark.parametrize("m,k,n,depth", [(8192, 8192, 8192, 2), (8192, 8192, 4096, 1),
                                         (8192, 4096, 2048, 1), (4096, 4096, 4096, 1)])
def test_strassen_deep_pipeline_leaf(bmm, leaf, m, k, n, depth):
    """Tile 6: int8 leaves with k = 2048 or 4096 bits run the fully unrolled 3-deep
    pipeline, fp4 leaves the 2-step loop; batched 2048^3 and 4096^3 leaves (7 and 49 per
    launch) with two waves per SIMD."""
    import torch
    seed = 901 + m + depth + leaf
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    opts = bmm.Options(leaf=leaf, tile=6, depth_serial=0, depth_parallel=depth)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, depth, opts)
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Cd = empty_dev(m, words(n), fill=-1)
    announce("strassen deep leaf", leaf, m, k, n, depth)
    bmm.bmm_gf2_strassen(to_dev(A), to_dev(B), Cd, m, k, n, ws, depth=depth, options=opts)
    rows = bmmgen.stratified_rows(m, 128, seed)
    assert np.array_equal(from_dev(Cd)[rows], oracle.rows(A[rows], B, k, n, oracle.GF2))


SCHEME_CASES = [  # m, k, n, depth, depth_serial
    (512, 512, 512, 1, 0), (1024, 1024, 1024, 4, 1), (2048, 2048, 2048, 5, 2),
    (1024, 2048, 512, 2, 1), (768, 1536, 1024, 1, 1), (2048, 2048, 2048, 3, 0),
]


@pytest.mark.parametrize("m,k,n,depth,ds", SCHEME_CASES)
@pytest.mark.parametrize("scheme", [1, 2])
def test_strassen_product_schemes(bmm, m, k, n, depth, ds, scheme):
    """The chaining alternative basis and standard-basis Strassen-Winograd reach
    AB exactly, like the self-inverse design."""
    import torch
    seed = bmmgen.config_seed(2) + 3 * m + depth + scheme
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    opts = bmm.Options(leaf=2, depth_serial=ds, depth_parallel=depth - ds, scheme=scheme)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, depth, opts)
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Cd = empty_dev(m, words(n), fill=-1)
    announce("strassen scheme", scheme, m, k, n, depth, ds)
    bmm.bmm_gf2_strassen(to_dev(A), to_dev(B), Cd, m, k, n, ws, depth=depth, options=opts)
    assert np.array_equal(from_dev(Cd), oracle.mul(A, B, k, n, oracle.GF2))


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("accumulate", [False, True])
def test_chained_products_in_alternative_basis(bmm, scheme, accumulate):
    """Theorem 2: with the chaining design the forward and inverse changes are
    mutual inverses, so (AB)C is computed as two alternative-basis products with
    no change back in between (trivially so for the standard basis)."""
    import torch
    n, d = 1024, 3
    mats = [bmmgen.fill_cpu(n, n, 91 + i, bmmgen.TAG_A, bmmgen.Dist.half()) for i in range(3)]
    dev = [to_dev(x) for x in mats]
    for x in dev:
        bmm.bmm_basis_change(x, n, n // 64, d, scheme=scheme)
    opts = bmm.Options(leaf=2, scheme=scheme)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(n, n, n, d, opts, alt_basis_io=True)
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    P = empty_dev(n, n // 64)
    Q = empty_dev(n, n // 64)
    announce("chained alt-basis products", scheme, accumulate)
    bmm.bmm_gf2_strassen(dev[0], dev[1], P, n, n, n, ws, depth=d, options=opts,
                         alt_basis_io=True)
    bmm.bmm_gf2_strassen(P, dev[2], Q, n, n, n, ws, depth=d, options=opts, alt_basis_io=True)
    if accumulate:  # Q-hat ^= P-hat C-hat: a second product into the same result
        bmm.bmm_gf2_strassen(P, dev[2], Q, n, n, n, ws, depth=d, options=opts,
                             alt_basis_io=True, accumulate=True)
    bmm.bmm_basis_change(Q, n, n // 64, d, inverse=True, scheme=scheme)
    ab = oracle.mul(mats[0], mats[1], n, n, oracle.GF2)
    want = oracle.mul(ab, mats[2], n, n, oracle.GF2)
    if accumulate:
        want = np.zeros_like(want)
    assert np.array_equal(from_dev(Q), want)


def test_strassen_alt_basis_io(bmm):
    """With A-hat, B-hat given, C-hat comes back (the core of eq. mb-mm-*)."""
    m = k = n = 1024
    d = 3
    A = bmmgen.fill_cpu(m, k, 3, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, 3, bmmgen.TAG_B, bmmgen.Dist.half())
    Ah = strassen.basis(A, d, algebra.sinv_fwd)
    Bh = strassen.basis(B, d, algebra.sinv_fwd)
    want_hat = strassen.core(Ah, Bh, d, strassen.packed_leaf(k >> d, n >> d))
    import torch
    opts = bmm.Options(leaf=2)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, d, opts, alt_basis_io=True)
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Cd = empty_dev(m, words(n))
    announce("alt_basis_io")
    bmm.bmm_gf2_strassen(to_dev(Ah), to_dev(Bh), Cd, m, k, n, ws, depth=d, options=opts,
                         alt_basis_io=True)
    assert np.array_equal(from_dev(Cd), want_hat)
    # and the inverse basis change of C-hat gives AB
    assert np.array_equal(strassen.basis(want_hat, d, algebra.sinv_inv),
                          oracle.mul(A, B, k, n, oracle.GF2))


@pytest.mark.parametrize("alt", [False, True])
@pytest.mark.parametrize("depth,ds", [(0, 0), (1, 1), (2, 0), (3, 1)])
@pytest.mark.parametrize("scheme", [0, 1, 2])
def test_strassen_accumulate(bmm, alt, depth, ds, scheme):
    """C ^= AB: in the standard basis through the inverse change's own inverse,
    and C-hat ^= core(A-hat, B-hat) in the alternative basis."""
    import torch
    m, k, n = 1024, 1536, 512
    A = bmmgen.fill_cpu(m, k, 61 + depth, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, 61 + depth, bmmgen.TAG_B, bmmgen.Dist.half())
    C0 = bmmgen.fill_cpu(m, n, 61 + depth, 0xC, bmmgen.Dist.half())
    dec = DECS[scheme]
    if alt:
        A = strassen.basis(A, depth, dec.fwd)
        B = strassen.basis(B, depth, dec.fwd)
        prod = strassen.core(A, B, depth, strassen.packed_leaf(k >> depth, n >> depth), dec)
    else:
        prod = oracle.mul(A, B, k, n, oracle.GF2)
    opts = bmm.Options(leaf=2, depth_serial=ds, depth_parallel=depth - ds, scheme=scheme)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, depth, opts, alt_basis_io=alt)
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Cd = to_dev(C0, words(n) + 1)
    announce("strassen accumulate", alt, depth, ds, scheme)
    bmm.bmm_gf2_strassen(to_dev(A), to_dev(B), Cd, m, k, n, ws, depth=depth, options=opts,
                         alt_basis_io=alt, accumulate=True)
    assert np.array_equal(from_dev(Cd, words(n)), C0 ^ prod)


@pytest.mark.parametrize("scheme", [0, 1, 2])
@pytest.mark.parametrize("b_t", [False, True])
@pytest.mark.parametrize("depth,ds,accumulate", [(1, 0, False), (3, 1, True), (4, 2, False),
                                                 (2, 2, True)])
def test_strassen_inplace_basis(bmm, scheme, b_t, depth, ds, accumulate):
    """BMM_FLAG_INPLACE_BASIS: A (and B^T when passed transposed) change basis in
    place; C is AB (or C ^ AB) and both operands hold their original words again
    afterwards (the changes are invertible in place, sections 2.2, 2.3, 3.6).  The
    workspace shrinks by the operands that are no longer copied."""
    import torch
    from oracle import brute
    m, k, n = 512 << (depth // 2), 1024, 2048 if depth == 4 else 1536
    seed = 500 + 10 * depth + scheme + (5 if b_t else 0)
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    C0 = bmmgen.fill_cpu(m, n, seed, 0xC, bmmgen.Dist.half())
    Bin = brute.pack(brute.unpack(B, n).T.copy()) if b_t else B
    opts = bmm.Options(leaf=2, depth_serial=ds, depth_parallel=depth - ds, scheme=scheme)
    full, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, depth, opts, b_transposed=b_t)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, depth, opts, b_transposed=b_t,
                                                  inplace_basis=True)
    saved = m * words(k) * 8 + (n * words(k) * 8 if b_t else 0)
    assert full - nbytes == saved
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Ad = to_dev(A, words(k) + 1)
    Bd = to_dev(Bin, Bin.shape[1] + 2)
    Cd = to_dev(C0) if accumulate else empty_dev(m, words(n), fill=-1)
    announce("strassen inplace", scheme, b_t, depth, ds, accumulate)
    bmm.bmm_gf2_strassen(Ad, Bd, Cd, m, k, n, ws, depth=depth, options=opts, b_transposed=b_t,
                         accumulate=accumulate, inplace_basis=True)
    prod = oracle.mul(A, B, k, n, oracle.GF2)
    assert np.array_equal(from_dev(Cd), (C0 ^ prod) if accumulate else prod)
    assert np.array_equal(from_dev(Ad, words(k)), A)
    assert np.array_equal(from_dev(Bd, Bin.shape[1]), Bin)


def test_strassen_alt_io_transposed_b_in_place(bmm):
    """Alternative-basis input with B passed transposed is read where it lies (no
    copy in the workspace) and left unchanged."""
    import torch
    from oracle import brute
    m = k = n = 1024
    d = 2
    A = bmmgen.fill_cpu(m, k, 8, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, 8, bmmgen.TAG_B, bmmgen.Dist.half())
    Ah = strassen.basis(A, d, algebra.sinv_fwd)
    Bh = strassen.basis(B, d, algebra.sinv_fwd)
    want_hat = strassen.core(Ah, Bh, d, strassen.packed_leaf(k >> d, n >> d))
    BhT = brute.pack(brute.unpack(Bh, n).T.copy())
    opts = bmm.Options(leaf=2)
    with_copy, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, d, opts, alt_basis_io=True)
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, d, opts, alt_basis_io=True,
                                                  b_transposed=True)
    assert with_copy - nbytes == n * words(k) * 8
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Bd = to_dev(BhT, words(k) + 1)
    Cd = empty_dev(m, words(n))
    announce("alt_basis_io transposed B")
    bmm.bmm_gf2_strassen(to_dev(Ah), Bd, Cd, m, k, n, ws, depth=d, options=opts,
                         alt_basis_io=True, b_transposed=True)
    assert np.array_equal(from_dev(Cd), want_hat)
    assert np.array_equal(from_dev(Bd, words(k)), BhT)


def test_strassen_errors(bmm):
    import torch
    A = empty_dev(1024, 16)
    C = empty_dev(1024, 16)
    ws = torch.empty(16, dtype=torch.int64, device="cuda")
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_gf2_strassen(A, empty_dev(1024, 16), C, 1024, 1000, 1024, ws, depth=2)
    assert e.value.status == -2  # k not divisible by 64 * 2^d
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_gf2_strassen(A, empty_dev(1024, 16), C, 1024, 1024, 1024, ws, depth=2)
    assert e.value.status == -3  # workspace too small
    big = torch.empty(1 << 22, dtype=torch.int64, device="cuda")
    with pytest.raises(bmm.BmmError) as e:  # in place with B^T inside A's storage
        bmm.bmm_gf2_strassen(A, A[:, :], C, 1024, 1024, 1024, big, depth=2, b_transposed=True,
                             inplace_basis=True)
    assert e.value.status == -1


LEAN_CASES = [  # m, k, n, depth, depth_serial
    (1024, 1024, 1024, 2, 1), (2048, 2048, 2048, 3, 2), (2048, 4096, 1024, 4, 3),
    (4096, 4096, 4096, 5, 2), (768, 1536, 1024, 1, 1),
]


@pytest.mark.parametrize("m,k,n,depth,ds", LEAN_CASES)
@pytest.mark.parametrize("scheme", [0, 1, 2])
@pytest.mark.parametrize("accumulate", [False, True])
def test_strassen_lean_serial_levels(bmm, m, k, n, depth, ds, scheme, accumulate):
    """BMM_FLAG_LEAN_WORKSPACE: the depth-first levels form one child at a time from the
    parent's quadrants and add each product into the parent's result quadrants; the
    product is the same and the workspace's serial part is a seventh."""
    import torch
    seed = 700 + m + depth + 3 * scheme + (1 if accumulate else 0)
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    C0 = bmmgen.fill_cpu(m, n, seed, 0xC, bmmgen.Dist.half())
    opts = bmm.Options(leaf=2, depth_serial=ds, depth_parallel=depth - ds, scheme=scheme,
                       flags=bmm.FLAG_LEAN_WORKSPACE)
    full = bmm.bmm_gf2_strassen_workspace(
        m, k, n, depth, bmm.Options(leaf=2, depth_serial=ds, depth_parallel=depth - ds,
                                    scheme=scheme))[0]
    nbytes, _, _ = bmm.bmm_gf2_strassen_workspace(m, k, n, depth, opts)
    assert nbytes < full
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    Cd = to_dev(C0) if accumulate else empty_dev(m, words(n), fill=-1)
    announce("strassen lean", m, k, n, depth, ds, scheme, accumulate)
    bmm.bmm_gf2_strassen(to_dev(A), to_dev(B), Cd, m, k, n, ws, depth=depth, options=opts,
                         accumulate=accumulate)
    prod = oracle.mul(A, B, k, n, oracle.GF2)
    assert np.array_equal(from_dev(Cd), (C0 ^ prod) if accumulate else prod)
