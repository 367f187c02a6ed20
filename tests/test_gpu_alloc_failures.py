"""Allocation failures inside the library (forced with bmm_debug_fail_allocations)
come back as BMM_E_NOMEM from every allocating entry point, and the next call,
with the hook spent, computes the right product."""
import numpy as np
import pytest

import bmmgen
import oracle
from gpu_util import announce, empty_dev, from_dev, to_dev, words

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bmm():
    import paper_1909_01554_amd as bmm
    yield bmm
    bmm.bmm_debug_fail_allocations(0)


def operands(m, k, n, seed):
    A = bmmgen.fill_cpu(m, k, seed, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, seed, bmmgen.TAG_B, bmmgen.Dist.half())
    return A, B


def test_cubic_scratch_allocation_failure(bmm):
    m, k, n = 300, 5000, 700
    A, B = operands(m, k, n, 71)
    Ad, Bd = to_dev(A), to_dev(B)
    Cd = empty_dev(m, words(n), fill=-1)
    bmm.bmm_finalize()  # drop the cached B^T scratch, so the next call allocates
    bmm.bmm_debug_fail_allocations(1)
    announce("forced allocation failure: cubic scratch")
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_gf2(Ad, Bd, Cd, m, k, n)
    assert e.value.status == -4
    bmm.bmm_gf2(Ad, Bd, Cd, m, k, n)  # the hook is spent
    assert np.array_equal(from_dev(Cd), oracle.mul(A, B, k, n, oracle.GF2))


@pytest.mark.parametrize("failing", [1, 2, 3])
def test_batched_plan_allocation_failures(bmm, failing):
    """Any of the plan's three device allocations (problem table, queue segments,
    counters) failing leaves the call with BMM_E_NOMEM and nothing half-built."""
    probs = []
    host = []
    for i in range(5):
        m, k, n = 100 + 37 * i, 300 + 64 * i, 90 + 11 * i
        A, B = operands(m, k, n, 80 + i)
        from oracle import brute
        BT = brute.pack(brute.unpack(B, n).T.copy())
        probs.append(dict(semiring=i % 2, m=m, k=k, n=n, A=to_dev(A), B=to_dev(BT),
                          C=empty_dev(m, words(n), fill=-1), b_transposed=True))
        host.append((i % 2, A, B, m, k, n))
    bmm.bmm_debug_fail_allocations(failing)
    announce("forced allocation failure: batched plan", failing)
    with pytest.raises(bmm.BmmError) as e:
        bmm.BatchedPlan(probs)
    assert e.value.status == -4
    bmm.bmm_debug_fail_allocations(0)
    plan = bmm.BatchedPlan(probs)
    plan.launch()
    for pr, (sr, A, B, m, k, n) in zip(probs, host):
        assert np.array_equal(from_dev(pr["C"], words(n)), oracle.mul(A, B, k, n, sr))
    plan.destroy()


def test_out_of_core_allocation_failure(bmm):
    import torch
    m, k, n = 500, 700, 600
    A, B = operands(m, k, n, 91)
    Ah = torch.from_numpy(A.view(np.int64)).pin_memory()
    Bh = torch.from_numpy(B.view(np.int64)).pin_memory()
    Ch = torch.full((m, words(n)), -1, dtype=torch.int64).pin_memory()
    bmm.bmm_debug_fail_allocations(3)
    announce("forced allocation failure: out of core")
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_ooc(oracle.BOOLEAN, Ah, Bh, Ch, m, k, n, block=256)
    assert e.value.status == -4
    bmm.bmm_debug_fail_allocations(0)
    bmm.bmm_ooc(oracle.BOOLEAN, Ah, Bh, Ch, m, k, n, block=256)
    assert np.array_equal(Ch.numpy().view(np.uint64), oracle.mul(A, B, k, n, oracle.BOOLEAN))
