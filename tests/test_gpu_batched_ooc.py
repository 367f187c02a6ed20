"""GPU parity of the persistent batched launch (also replayed from a HIP graph)
and of the out-of-core pipeline, against the oracle's plain product."""
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


def transpose_packed(B, k, n):
    from oracle import brute
    return brute.pack(brute.unpack(B, n).T.copy())


def make_problems(count, seed, maxdim=600, transposed=True):
    rng = np.random.default_rng(seed)
    probs, host = [], []
    for p in range(count):
        m, k, n = (int(x) for x in rng.integers(1, maxdim, size=3))
        if p % 7 == 3:
            k = 0
        sr = oracle.GF2 if p % 2 == 0 else oracle.BOOLEAN
        dist = bmmgen.Dist.half() if sr == oracle.GF2 else bmmgen.Dist.inv_sqrt(max(k, 1))
        A = bmmgen.fill_cpu(m, max(k, 1), seed, bmmgen.batched_tag(p, "A"), dist)
        B = bmmgen.fill_cpu(max(k, 1), n, seed, bmmgen.batched_tag(p, "B"), dist)
        if k == 0:
            A[:] = 0
            B = B[:1]
        Bd = to_dev(transpose_packed(B, max(k, 1), n)) if transposed else to_dev(B)
        Cd = empty_dev(m, words(n), fill=-1)
        probs.append(dict(semiring=sr, m=m, k=k, n=n, A=to_dev(A), B=Bd, C=Cd,
                          b_transposed=transposed))
        host.append((sr, A, B, m, k, n))
    return probs, host


def check(probs, host):
    for pr, (sr, A, B, m, k, n) in zip(probs, host):
        want = oracle.mul(A, B, max(k, 1), n, sr) if k else np.zeros((m, words(n)), np.uint64)
        got = from_dev(pr["C"], words(n))
        assert np.array_equal(got, want), (sr, m, k, n)


@pytest.mark.parametrize("transposed", [True, False])
def test_batched_mixed(bmm, transposed):
    probs, host = make_problems(40, 7 + transposed, transposed=transposed)
    announce("batched", transposed)
    bmm.bmm_batched(probs)
    check(probs, host)


@pytest.mark.parametrize("leaf", [2, 3])
@pytest.mark.parametrize("tile", [1, 2, 3, 4])
def test_batched_leaf_and_tile(bmm, leaf, tile):
    """Every batched leaf kind (int8, fp4) and tile (128 x 64, 64 x 64, 64 x 128, and
    128 x 64 with LDS-shared operand rows)."""
    probs, host = make_problems(36, 50 + 3 * leaf + tile)
    announce("batched leaf/tile", leaf, tile)
    bmm.bmm_batched(probs, options=bmm.Options(leaf=leaf, tile=tile))
    check(probs, host)


@pytest.fixture(scope="module")
def large_batch():
    """Ten problems of 500-2100 rows and columns and 3000-6100 bits of k: every
    problem spans many work items, split over several queues, and most reach the
    chunked long-k loop; odd word counts of k take the 8-byte-load path."""
    rng = np.random.default_rng(2024)
    seed = 77
    items = []
    for p in range(10):
        m, n = (int(x) for x in rng.integers(500, 2100, size=2))
        k = int(rng.integers(3000, 6100))
        sr = oracle.GF2 if p % 2 == 0 else oracle.BOOLEAN
        dist = bmmgen.Dist.half() if sr == oracle.GF2 else bmmgen.Dist.inv_sqrt(k)
        A = bmmgen.fill_cpu(m, k, seed, bmmgen.batched_tag(p, "A"), dist)
        B = bmmgen.fill_cpu(k, n, seed, bmmgen.batched_tag(p, "B"), dist)
        items.append((sr, A, B, m, k, n, oracle.mul(A, B, k, n, sr)))
    return items


@pytest.mark.parametrize("leaf", [2, 3])
@pytest.mark.parametrize("tile", [1, 2, 3, 4])
def test_batched_large_items(bmm, large_batch, leaf, tile):
    probs = []
    for sr, A, B, m, k, n, _ in large_batch:
        probs.append(dict(semiring=sr, m=m, k=k, n=n, A=to_dev(A),
                          B=to_dev(transpose_packed(B, k, n)),
                          C=empty_dev(m, words(n), fill=-1), b_transposed=True))
    announce("batched large items", leaf, tile)
    bmm.bmm_batched(probs, options=bmm.Options(leaf=leaf, tile=tile))
    for pr, (sr, A, B, m, k, n, want) in zip(probs, large_batch):
        assert np.array_equal(from_dev(pr["C"], words(n)), want), (sr, m, k, n, leaf, tile)


def test_batched_autotune_and_auto_plan(bmm):
    probs, host = make_problems(24, 99)
    announce("batched autotune")
    leaf, tile, secs = bmm.bmm_autotune_batched(probs)
    assert leaf in (2, 3) and tile in (1, 2, 3, 4) and secs > 0
    check(probs, host)
    for pr in probs:
        pr["C"].fill_(-1)
    plan = bmm.BatchedPlan(probs)  # AUTO: takes the recorded choice
    plan.launch()
    check(probs, host)
    plan.destroy()
    for pr in probs:
        pr["C"].fill_(-1)
    announce("batched VALU leaf")
    bmm.bmm_batched(probs, options=bmm.Options(leaf=1))  # one VALU launch per problem
    check(probs, host)


def test_batched_plan_graph_replay(bmm):
    import torch
    probs, host = make_problems(30, 21)
    plan = bmm.BatchedPlan(probs)
    s = torch.cuda.Stream()
    announce("batched plan eager")
    with torch.cuda.stream(s):
        plan.launch(s.cuda_stream)
    s.synchronize()
    check(probs, host)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.launch(s.cuda_stream)
    for rep in range(3):
        for pr in probs:
            pr["C"].fill_(-1)
        torch.cuda.synchronize()
        announce("batched plan graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        check(probs, host)
    plan.destroy()


@pytest.mark.parametrize("sr", [oracle.GF2, oracle.BOOLEAN])
def test_ooc_small(bmm, sr):
    import torch
    m, k, n = 700, 1000, 900
    dist = bmmgen.Dist.half() if sr == oracle.GF2 else bmmgen.Dist.pow2(4)
    A = bmmgen.fill_cpu(m, k, 31, bmmgen.TAG_A, dist)
    B = bmmgen.fill_cpu(k, n, 31, bmmgen.TAG_B, dist)
    Ah = torch.from_numpy(A.view(np.int64)).pin_memory()
    Bh = torch.from_numpy(B.view(np.int64)).pin_memory()
    Ch = torch.full((m, words(n)), -1, dtype=torch.int64).pin_memory()
    announce("ooc", sr)
    secs = bmm.bmm_ooc(sr, Ah, Bh, Ch, m, k, n, block=256)
    assert secs > 0
    got = Ch.numpy().view(np.uint64)
    assert np.array_equal(got, oracle.mul(A, B, k, n, sr))
    # every C word crosses PCIe down once; each A block goes up once per column block
    # of C (4 of them) and each B block once per row block of C (3)
    hb, hs, db, ds = bmm.bmm_ooc_last_transfers()
    assert db == m * words(n) * 8 and ds > 0
    assert hb == 4 * A.nbytes + 3 * B.nbytes and hs > 0


@pytest.mark.parametrize("cubic_only", [False, True])
def test_ooc_gf2_alternative_basis_blocks(bmm, cubic_only):
    """GF(2) blocks of 8192 bits run one level of the alternative-basis recursion
    in HBM (the ragged last k block and the narrow last column block fall back to
    the cubic leaf); sampled rows and Freivalds's check against the oracle."""
    import torch
    m, k, n = 16384, 16384 + 640, 16384 + 128
    seed = 77
    dist = bmmgen.Dist.half()
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, dist)
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, dist)
    Ah = torch.from_numpy(A.view(np.int64)).pin_memory()
    Bh = torch.from_numpy(B.view(np.int64)).pin_memory()
    Ch = torch.full((m, words(n)), -1, dtype=torch.int64).pin_memory()
    opts = bmm.Options(leaf=bmm.LEAF_MFMA_I8, depth_serial=0 if cubic_only else -1,
                       depth_parallel=0 if cubic_only else -1)
    announce("ooc gf2 alternative-basis blocks", cubic_only)
    bmm.bmm_ooc(oracle.GF2, Ah, Bh, Ch, m, k, n, block=8192, options=opts)
    got = Ch.numpy().view(np.uint64)
    rows = bmmgen.stratified_rows(m, 64, seed)
    assert np.array_equal(got[rows], oracle.rows(A[rows], B, k, n, oracle.GF2))
    X = bmmgen.freivalds_vectors(m, 8, seed)
    assert all(oracle.freivalds(A, B, got, m, k, n, X))


@pytest.mark.parametrize("scheme", [0, 1, 2])
@pytest.mark.parametrize("dh", [1, 2])
@pytest.mark.parametrize("block_order", [False, True])
def test_ooc_gf2_host_levels(bmm, scheme, dh, block_order):
    """Square GF(2) operands of 2^dh blocks per side: dh host levels of the
    recursion (7^dh sub-instances formed on the GPU from uploaded blocks, one
    device level each), or the cubic block order; sampled rows and Freivalds's
    check against the oracle."""
    import torch
    blk = 8192
    n = blk << dh
    seed = 300 + 10 * scheme + dh
    dist = bmmgen.Dist.half()
    A = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_A, dist)
    B = bmmgen.fill_cpu(n, n, seed, bmmgen.TAG_B, dist)
    Ah = torch.from_numpy(A.view(np.int64)).pin_memory()
    Bh = torch.from_numpy(B.view(np.int64)).pin_memory()
    Ch = torch.full((n, words(n)), -1, dtype=torch.int64).pin_memory()
    opts = bmm.Options(leaf=bmm.LEAF_MFMA_I8, scheme=scheme,
                       flags=bmm.FLAG_OOC_BLOCK_ORDER if block_order else 0)
    announce("ooc gf2 host levels", scheme, dh, block_order)
    bmm.bmm_ooc(oracle.GF2, Ah, Bh, Ch, n, n, n, block=blk, options=opts)
    got = Ch.numpy().view(np.uint64)
    rows = bmmgen.stratified_rows(n, 64, seed)
    assert np.array_equal(got[rows], oracle.rows(A[rows], B, n, n, oracle.GF2))
    X = bmmgen.freivalds_vectors(n, 8, seed)
    assert all(oracle.freivalds(A, B, got, n, n, n, X))


def test_ooc_rejects_pageable(bmm):
    A = np.zeros((64, 1), np.uint64)
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_ooc(0, A, A.copy(), A.copy(), 64, 64, 64)
    assert e.value.status == -1


def test_batched_cached_plan_replays(bmm):
    """bmm_batched keeps a plan (and its graph) per problem table: a second call on
    the same buffers with new contents replays it and reads the new operands; calls
    on two streams with the same table are ordered by the library; inside a stream
    capture the call records its kernels into the caller's graph."""
    import torch
    probs, host = make_problems(20, 303, transposed=False)
    announce("batched cache first call")
    bmm.bmm_batched(probs)
    check(probs, host)
    # new operand contents in the same buffers: the cached table points at them
    host2 = []
    for p, (pr, (sr, A, B, m, k, n)) in enumerate(zip(probs, host)):
        dist = bmmgen.Dist.half() if sr == oracle.GF2 else bmmgen.Dist.inv_sqrt(max(k, 1))
        A2 = bmmgen.fill_cpu(m, max(k, 1), 404, bmmgen.batched_tag(p, "A"), dist)
        if k == 0:
            A2[:] = 0
        pr["A"].copy_(to_dev(A2))
        pr["C"].fill_(-1)
        host2.append((sr, A2, B, m, k, n))
    torch.cuda.synchronize()
    announce("batched cache replay, new contents")
    bmm.bmm_batched(probs)
    check(probs, host2)
    # two streams back to back with no host synchronization in between
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for pr in probs:
        pr["C"].fill_(-1)
    torch.cuda.synchronize()
    announce("batched cache, two streams")
    bmm.bmm_batched(probs, stream=s1.cuda_stream)
    bmm.bmm_batched(probs, stream=s2.cuda_stream)
    torch.cuda.synchronize()
    check(probs, host2)
    # captured into a torch graph (the plan exists already), replayed three times
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s1):
        bmm.bmm_batched(probs, stream=s1.cuda_stream)
    for rep in range(3):
        for pr in probs:
            pr["C"].fill_(-1)
        torch.cuda.synchronize()
        announce("batched cache captured replay", rep)
        g.replay()
        torch.cuda.synchronize()
        check(probs, host2)


def test_batched_cache_eviction_and_capture_refusal(bmm):
    import torch
    tables = [make_problems(3, 600 + i, maxdim=200) for i in range(10)]
    for i, (probs, host) in enumerate(tables):  # more tables than the cache holds
        announce("batched cache table", i)
        bmm.bmm_batched(probs)
        check(probs, host)
    probs, host = tables[0]  # evicted by now: rebuilt on this call
    for pr in probs:
        pr["C"].fill_(-1)
    announce("batched cache rebuilt table")
    bmm.bmm_batched(probs)
    check(probs, host)
    fresh, _ = make_problems(3, 700, maxdim=200)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    announce("batched first call inside capture")
    with torch.cuda.graph(g, stream=s):
        with pytest.raises(bmm.BmmError) as e:
            bmm.bmm_batched(fresh, stream=s.cuda_stream)
        fresh[0]["C"].fill_(0)  # keep the captured graph non-empty
    assert e.value.status == -2


@pytest.mark.parametrize("which", ["gf2", "boolean", "strassen"])
def test_host_operands_through_product_calls(bmm, which):
    """BMM_FLAG_HOST_OPERANDS on bmm_gf2, bmm_boolean and bmm_gf2_strassen runs the
    out-of-core pipeline on page-locked host tensors (cubic block order for the
    cubic calls, host-level recursion levels for the Strassen call)."""
    import torch
    m = k = n = 2048 if which == "strassen" else 1000
    sr = oracle.BOOLEAN if which == "boolean" else oracle.GF2
    dist = bmmgen.Dist.half() if sr == oracle.GF2 else bmmgen.Dist.pow2(5)
    A = bmmgen.fill_cpu(m, k, 44, bmmgen.TAG_A, dist)
    B = bmmgen.fill_cpu(k, n, 44, bmmgen.TAG_B, dist)
    Ah = torch.from_numpy(A.view(np.int64)).pin_memory()
    Bh = torch.from_numpy(B.view(np.int64)).pin_memory()
    Ch = torch.full((m, words(n)), -1, dtype=torch.int64).pin_memory()
    opts = bmm.Options(block=1024 if which == "strassen" else 384)
    announce("host operands", which)
    if which == "strassen":
        bmm.bmm_gf2_strassen(Ah, Bh, Ch, m, k, n, None, options=opts, host_operands=True)
    else:
        fn = bmm.bmm_gf2 if sr == oracle.GF2 else bmm.bmm_boolean
        fn(Ah, Bh, Ch, m, k, n, options=opts, host_operands=True)
    assert np.array_equal(Ch.numpy().view(np.uint64), oracle.mul(A, B, k, n, sr))
    with pytest.raises(bmm.BmmError) as e:  # no accumulation out of core
        bmm.bmm_gf2(Ah, Bh, Ch, m, k, n, accumulate=True, host_operands=True)
    assert e.value.status == -2


def test_batched_plan_mixes_leaves_per_class(bmm, tmp_path):
    """A plan whose problems take different leaf kinds and tiles by size class of k
    (records loaded from a table): VALU launches for the short ones, an int8 and an fp4
    persistent group for the others, all exact."""
    probs, host = make_problems(30, 515, maxdim=6000)
    ops = float(sum(2 * p["m"] * p["k"] * p["n"] for p in probs))
    b = 0
    while ops >= 2.0 and b < 200:
        ops *= 0.5
        b += 1
    kcls = [0 if p["k"] < 1024 else (1 if p["k"] < 4096 else 2) for p in probs]
    assert len(set(kcls)) == 3
    table = tmp_path / "mix.txt"
    table.write_text(f"batched {len(probs)} {b} 2 4 2\n"
                     f"batched_class {len(probs)} {b} 0 1 1\n"
                     f"batched_class {len(probs)} {b} 1 2 4\n"
                     f"batched_class {len(probs)} {b} 2 3 1\n")
    bmm.bmm_autotune_load(str(table))
    try:
        plan = bmm.BatchedPlan(probs)
        announce("batched per-class mix")
        plan.launch()
        check(probs, host)
        plan.destroy()
        for pr in probs:
            pr["C"].fill_(-1)
        bmm.bmm_batched(probs)  # the cached, graph-replayed form of the same plan
        check(probs, host)
    finally:
        bmm.bmm_finalize()  # drop the loaded records
