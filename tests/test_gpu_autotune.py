"""GPU checks of the autotuners: they pick valid kernels, the products that use
their choices stay bit-exact, and the tables survive a save/load round trip."""
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


@pytest.mark.parametrize("sr", [oracle.GF2, oracle.BOOLEAN])
def test_autotuned_cubic_leaf_is_exact(bmm, sr):
    m, k, n = 384, 1536, 320
    announce("autotune leaf", sr)
    leaf, tile, secs = bmm.bmm_autotune_cubic(sr, m, k, n)
    assert leaf in (1, 2, 3) and tile >= 1 and secs > 0
    leaf4, tile4, _ = bmm.bmm_autotune_leaf(sr, m, k, n, 8)
    assert leaf4 in (1, 2, 3) and tile4 >= 1
    A = bmmgen.fill_cpu(m, k, 3, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, 3, bmmgen.TAG_B, bmmgen.Dist.half())
    Cd = empty_dev(m, words(n), fill=-1)
    fn = bmm.bmm_gf2 if sr == oracle.GF2 else bmm.bmm_boolean
    fn(to_dev(A), to_dev(B), Cd, m, k, n)  # LEAF_AUTO: the tuned choice
    assert np.array_equal(from_dev(Cd), oracle.mul(A, B, k, n, sr))


@pytest.mark.parametrize("sr", [oracle.GF2, oracle.BOOLEAN])
def test_k_panel_tuner(bmm, sr, tmp_path):
    """The k-panel tuner picks one of the candidates, leaves the product in C, records
    its choice for k_panel = 0 (the product that uses it stays exact) and refuses
    accumulation."""
    m, k, n = 256, 16384, 320
    A = bmmgen.fill_cpu(m, k, 9, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(k, n, 9, bmmgen.TAG_B, bmmgen.Dist.half())
    want = oracle.mul(A, B, k, n, sr)
    Ad, Bd = to_dev(A), to_dev(B)
    Cd = empty_dev(m, words(n), fill=-1)
    announce("k-panel tuner", sr)
    bits, secs = bmm.bmm_autotune_k_panel(sr, Ad, Bd, Cd, m, k, n, candidates=[k, 4096, 1000])
    assert bits in (k, 4096, 1024) and secs > 0
    assert np.array_equal(from_dev(Cd), want)
    p = tmp_path / "t.txt"
    bmm.bmm_autotune_save(str(p))
    assert f"kpanel {sr} {m} {k} {n} {bits}" in p.read_text()
    Cd = empty_dev(m, words(n), fill=-1)
    fn = bmm.bmm_gf2 if sr == oracle.GF2 else bmm.bmm_boolean
    fn(Ad, Bd, Cd, m, k, n)
    assert np.array_equal(from_dev(Cd), want)
    with pytest.raises(bmm.BmmError):
        bmm.bmm_autotune_k_panel(sr, Ad, Bd, Cd, m, k, n,
                                 options=bmm.Options(flags=bmm.FLAG_ACCUMULATE))


def test_autotuned_strassen_depth_is_exact(bmm, tmp_path):
    import torch
    n = 4096
    A = bmmgen.fill_cpu(n, n, 5, bmmgen.TAG_A, bmmgen.Dist.half())
    B = bmmgen.fill_cpu(n, n, 5, bmmgen.TAG_B, bmmgen.Dist.half())
    Ad, Bd = to_dev(A), to_dev(B)
    Cd = empty_dev(n, n // 64)
    nbytes = max(bmm.bmm_gf2_strassen_workspace(n, n, n, d, bmm.Options(depth_serial=0))[0]
                 for d in range(0, 3))
    ws = torch.empty(nbytes // 8 + 1, dtype=torch.int64, device="cuda")
    announce("autotune strassen")
    d, ds, shift, secs = bmm.bmm_autotune_strassen(Ad, Bd, Cd, n, n, n, ws)
    assert 0 <= ds <= d <= 2 and secs > 0
    Cd.fill_(-1)
    bmm.bmm_gf2_strassen(Ad, Bd, Cd, n, n, n, ws, depth=-1)
    assert np.array_equal(from_dev(Cd), oracle.mul(A, B, n, n, oracle.GF2))
    path = tmp_path / "tune.txt"
    bmm.bmm_autotune_save(str(path))
    text = path.read_text()
    assert f"depth {n} {n} {n} {d} {ds}" in text
    bmm.bmm_autotune_load(str(path))
