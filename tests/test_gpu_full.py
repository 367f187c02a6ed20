"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (the package's autotune table loaded, the same seeds, tags and
bit distributions).  Outputs too large for the oracle to recompute whole are
checked on stratified sampled rows against its plain product, by Freivalds's
check over GF(2), and by the entrywise order Boolean >= GF(2) on the same
operands (a one in the GF(2) sum needs at least one nonzero term)."""
import os

import numpy as np
import pytest

import bmmgen
import oracle
from gpu_util import announce, words

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(os.path.dirname(HERE), "paper_1909_01554_amd", "tune_gfx950.txt")


@pytest.fixture(scope="module")
def bmm():
    import paper_1909_01554_amd as bmm
    bmm.bmm_autotune_load(TABLE)
    return bmm


@pytest.fixture(autouse=True)
def _release():
    yield
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def dev_matrix(rows, cols, seed, tag, dist):
    import torch
    t = torch.empty((rows, words(cols)), dtype=torch.int64, device="cuda")
    bmmgen.fill_tensor(t, rows, cols, seed, tag, dist)
    return t


def dev_rows(C, rows):
    import torch
    idx = torch.tensor(rows, device=C.device)
    return C.index_select(0, idx).cpu().numpy().view(np.uint64)


def leaf_ids(bmm):
    return [("valu", bmm.LEAF_VALU), ("int8", bmm.LEAF_MFMA_I8), ("fp4", bmm.LEAF_MFMA_F4)]


@pytest.mark.timeout(900)
def test_cubic_n65536_sampled_rows_freivalds_order(bmm):
    """Cubic products at n = 65536: GF(2) on Bernoulli(1/2) bits and Boolean on
    Bernoulli(2^-8) bits, every leaf kind; 1024 stratified rows of each against
    the oracle, 20 Freivalds vectors on the GF(2) product, and GF(2) <= Boolean
    entrywise on the GF(2) operands."""
    import torch
    n = 1 << 16
    seed = bmmgen.config_seed(1)
    half, sparse = bmmgen.Dist.half(), bmmgen.Dist.pow2(8)
    announce("full cubic n=65536: operands")
    A = dev_matrix(n, n, seed, bmmgen.TAG_A, half)
    B = dev_matrix(n, n, seed, bmmgen.TAG_B, half)
    Ab = dev_matrix(n, n, seed, 0x1A, sparse)
    Bb = dev_matrix(n, n, seed, 0x1B, sparse)
    C = torch.empty_like(A)
    Cor = torch.empty_like(A)

    rows = bmmgen.stratified_rows(n, 1024, seed)
    assert len(rows) >= 1024
    Bh = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_B, half)
    Ah = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_A, half)
    want_g = oracle.rows(Ah[rows], Bh, n, n, oracle.GF2)
    X = bmmgen.freivalds_vectors(n, 20, seed)
    lhs = [oracle.vecmat(oracle.vecmat(x, Ah, n, n), Bh, n, n) for x in X]
    del Ah, Bh
    Bbh = bmmgen.fill_cpu(n, n, seed, 0x1B, sparse)
    Abr = bmmgen.fill_rows_cpu(rows, n, seed, 0x1A, sparse)
    want_b = oracle.rows(Abr, Bbh, n, n, oracle.BOOLEAN)
    del Bbh
    # about 63% of the Boolean outputs are ones at p = 2^-8
    density = np.unpackbits(want_b.view(np.uint8)).mean()
    assert 0.55 < density < 0.70

    for name, leaf in leaf_ids(bmm):
        o = bmm.Options(leaf=leaf)
        announce("full cubic n=65536 GF(2)", name)
        C.fill_(-1)
        bmm.bmm_gf2(A, B, C, n, n, n, options=o)
        assert np.array_equal(dev_rows(C, rows), want_g), name
        Ch = C.cpu().numpy().view(np.uint64)
        ok = [np.array_equal(lhs[i], oracle.vecmat(x, Ch, n, n)) for i, x in enumerate(X)]
        assert all(ok), (name, ok)
        del Ch
        announce("full cubic n=65536 Boolean order", name)
        Cor.fill_(0)
        bmm.bmm_boolean(A, B, Cor, n, n, n, options=o)
        assert not bool(torch.any(C & ~Cor)), name
        announce("full cubic n=65536 Boolean", name)
        C.fill_(-1)
        bmm.bmm_boolean(Ab, Bb, C, n, n, n, options=o)
        assert np.array_equal(dev_rows(C, rows), want_b), name


@pytest.mark.timeout(900)
def test_strassen_n262144_sampled_rows_freivalds(bmm):
    """The GF(2) alternative-basis product at n = 2^18 (8 GiB per operand) with the
    tuned depth, every leaf kind: 1024 stratified rows against the oracle and 20
    Freivalds vectors."""
    import torch
    n = 1 << 18
    seed = bmmgen.config_seed(2)
    half = bmmgen.Dist.half()
    announce("full Strassen n=2^18: operands")
    A = dev_matrix(n, n, seed, bmmgen.TAG_A, half)
    B = dev_matrix(n, n, seed, bmmgen.TAG_B, half)
    C = torch.empty_like(A)
    nbytes = max(bmm.bmm_gf2_strassen_workspace(n, n, n, -1, bmm.Options(leaf=lf))[0]
                 for _, lf in leaf_ids(bmm))
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")

    announce("full Strassen n=2^18: oracle rows and Freivalds left sides")
    rows = bmmgen.stratified_rows(n, 1024, seed)
    Bh = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_B, half)
    Ar = bmmgen.fill_rows_cpu(rows, n, seed, bmmgen.TAG_A, half)
    want = oracle.rows(Ar, Bh, n, n, oracle.GF2)
    X = bmmgen.freivalds_vectors(n, 20, seed)
    Ah = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_A, half)
    xa = [oracle.vecmat(x, Ah, n, n) for x in X]
    del Ah
    lhs = [oracle.vecmat(v, Bh, n, n) for v in xa]
    del Bh

    for name, leaf in leaf_ids(bmm):
        announce("full Strassen n=2^18", name)
        C.fill_(-1)
        bmm.bmm_gf2_strassen(A, B, C, n, n, n, ws, depth=-1, options=bmm.Options(leaf=leaf))
        assert np.array_equal(dev_rows(C, rows), want), name
        Ch = C.cpu().numpy().view(np.uint64)
        ok = [np.array_equal(lhs[i], oracle.vecmat(x, Ch, n, n)) for i, x in enumerate(X)]
        del Ch
        assert all(ok), (name, ok)


@pytest.mark.timeout(900)
def test_boolean_n262144_sampled_rows(bmm):
    """The benchmark's Boolean cubic product at n = 2^18 (Bernoulli(2^-9) bits, B
    transposed once, then the leaf), every leaf kind, on 256 stratified rows."""
    import torch
    n = 1 << 18
    seed = bmmgen.config_seed(2)
    dist = bmmgen.Dist.pow2(9)
    announce("full Boolean n=2^18: operands")
    A = dev_matrix(n, n, seed, 0x1A, dist)
    B = dev_matrix(n, n, seed, 0x1B, dist)
    BT = torch.empty_like(B)
    bmm.bmm_transpose(B, BT, n, n)
    del B
    C = torch.empty_like(A)
    rows = bmmgen.stratified_rows(n, 256, seed)
    Bh = bmmgen.fill_cpu(n, n, seed, 0x1B, dist)
    want = oracle.rows(bmmgen.fill_rows_cpu(rows, n, seed, 0x1A, dist), Bh, n, n, oracle.BOOLEAN)
    del Bh
    for name, leaf in leaf_ids(bmm):
        announce("full Boolean n=2^18", name)
        C.fill_(-1)
        bmm.bmm_boolean(A, BT, C, n, n, n, options=bmm.Options(leaf=leaf), b_transposed=True)
        assert np.array_equal(dev_rows(C, rows), want), name


@pytest.mark.timeout(900)
def test_batched_4096_sampled(bmm):
    """4096 uneven products in one persistent launch replayed from a HIP graph:
    8 stratified rows of every product, 2 Freivalds vectors on every GF(2)
    product, and the whole output of every 64th product, against the oracle."""
    import torch
    seed = bmmgen.config_seed(3)
    shapes = bmmgen.batched_shapes(4096, seed)
    announce("full batched 4096: operands")
    na = sum(m * words(k) for _, m, k, n, _ in shapes)
    nb = sum(n * words(k) for _, m, k, n, _ in shapes)
    nc = sum(m * words(n) for _, m, k, n, _ in shapes)
    bufA = torch.empty(na, dtype=torch.int64, device="cuda")
    bufB = torch.empty(nb, dtype=torch.int64, device="cuda")
    bufC = torch.full((nc,), -1, dtype=torch.int64, device="cuda")
    probs, offs, oa, ob, oc = [], [], 0, 0, 0
    for p, (sr, m, k, n, dist) in enumerate(shapes):
        Ad = bufA[oa:oa + m * words(k)].view(m, words(k))
        BTd = bufB[ob:ob + n * words(k)].view(n, words(k))
        Cd = bufC[oc:oc + m * words(n)].view(m, words(n))
        offs.append(oc)
        oa, ob, oc = oa + Ad.numel(), ob + BTd.numel(), oc + Cd.numel()
        bmmgen.fill_tensor(Ad, m, k, seed, bmmgen.batched_tag(p, "A"), dist)
        Bd = dev_matrix(k, n, seed, bmmgen.batched_tag(p, "B"), dist)
        bmm.bmm_transpose(Bd, BTd, k, n)
        probs.append(dict(semiring=sr, m=m, k=k, n=n, A=Ad, B=BTd, C=Cd, b_transposed=True))
    torch.cuda.synchronize()
    plan = bmm.BatchedPlan(probs)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.launch(s.cuda_stream)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.launch(s.cuda_stream)
    bufC.fill_(-1)
    torch.cuda.synchronize()
    announce("full batched 4096: graph replay")
    g.replay()
    torch.cuda.synchronize()
    Call = bufC.cpu().numpy().view(np.uint64)
    plan.destroy()

    announce("full batched 4096: oracle")
    for p, (sr, m, k, n, dist) in enumerate(shapes):
        got = Call[offs[p]:offs[p] + m * words(n)].reshape(m, words(n))
        Bh = bmmgen.fill_cpu(k, n, seed, bmmgen.batched_tag(p, "B"), dist)
        if p % 64 == 0:
            Ah = bmmgen.fill_cpu(m, k, seed, bmmgen.batched_tag(p, "A"), dist)
            assert np.array_equal(got, oracle.mul(Ah, Bh, k, n, sr)), (p, sr, m, k, n)
            continue
        rows = bmmgen.stratified_rows(m, 8, seed + p)
        Ar = bmmgen.fill_rows_cpu(rows, k, seed, bmmgen.batched_tag(p, "A"), dist)
        assert np.array_equal(got[rows], oracle.rows(Ar, Bh, k, n, sr)), (p, sr, m, k, n)
        if sr == oracle.GF2:
            Ah = bmmgen.fill_cpu(m, k, seed, bmmgen.batched_tag(p, "A"), dist)
            X = bmmgen.freivalds_vectors(m, 2, seed + p)
            assert all(oracle.freivalds(Ah, Bh, got, m, k, n, X)), (p, m, k, n)


@pytest.mark.timeout(900)
def test_ooc_n262144_sampled_rows_freivalds(bmm):
    """The out-of-core products as the benchmark runs them: n = 2^18 with A, B and C
    in page-locked host memory (24 GiB) and blocks of 2^17 bits; GF(2) with one host
    level of the recursion and in the cubic block order (Bernoulli(1/2) bits), Boolean
    in the block order (Bernoulli(2^-9) bits), int8 leaves.  256 stratified rows of
    each product against the oracle, and 4 Freivalds vectors on each GF(2) product."""
    import torch
    n, blk = 1 << 18, 1 << 17
    nw = n // 64
    seed = bmmgen.config_seed(4)
    announce("full ooc n=2^18: pinned buffers")
    A = torch.empty((n, nw), dtype=torch.int64, pin_memory=True)
    B = torch.empty((n, nw), dtype=torch.int64, pin_memory=True)
    C = torch.empty((n, nw), dtype=torch.int64, pin_memory=True)
    slab = torch.empty((1 << 15, nw), dtype=torch.int64, device="cuda")
    rows = bmmgen.stratified_rows(n, 256, seed)
    runs = [("gf2_host_levels", oracle.GF2, bmmgen.Dist.half(), 0),
            ("gf2_block_order", oracle.GF2, bmmgen.Dist.half(), bmm.FLAG_OOC_BLOCK_ORDER),
            ("boolean_block_order", oracle.BOOLEAN, bmmgen.Dist.pow2(9), 0)]
    made, want, X, lhs = None, None, None, None
    for name, sr, dist, flags in runs:
        if made != (dist.kind, dist.param):
            announce("full ooc n=2^18: operands and oracle", name)
            for dst, tag in [(A, bmmgen.TAG_A), (B, bmmgen.TAG_B)]:
                for r0 in range(0, n, slab.shape[0]):
                    bmmgen.fill_tensor(slab, slab.shape[0], n, seed, tag, dist, row0=r0)
                    dst[r0:r0 + slab.shape[0]].copy_(slab)
            torch.cuda.synchronize()
            Bh = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_B, dist)
            Ar = bmmgen.fill_rows_cpu(rows, n, seed, bmmgen.TAG_A, dist)
            want = oracle.rows(Ar, Bh, n, n, sr)
            if sr == oracle.GF2:
                X = bmmgen.freivalds_vectors(n, 4, seed)
                Ah = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_A, dist)
                lhs = [oracle.vecmat(oracle.vecmat(x, Ah, n, n), Bh, n, n) for x in X]
                del Ah
            del Bh
            made = (dist.kind, dist.param)
        announce("full ooc n=2^18", name)
        C.fill_(-1)
        bmm.bmm_ooc(sr, A, B, C, n, n, n, block=blk,
                    options=bmm.Options(leaf=bmm.LEAF_MFMA_I8, flags=flags))
        Ch = C.numpy().view(np.uint64)
        assert np.array_equal(Ch[rows], want), name
        if sr == oracle.GF2:
            ok = [np.array_equal(lhs[i], oracle.vecmat(x, Ch, n, n)) for i, x in enumerate(X)]
            assert all(ok), (name, ok)
    del A, B, C, slab
