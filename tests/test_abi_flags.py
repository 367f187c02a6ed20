"""CPU-side checks of the flags that change what the Strassen product stages in
its workspace (no device work: the workspace query only plans)."""
import pytest


@pytest.fixture(scope="module")
def bmm():
    import paper_1909_01554_amd as bmm
    return bmm


@pytest.mark.parametrize("m,k,n,d", [(1024, 1024, 1024, 2), (2048, 4096, 1024, 3),
                                     (1 << 18, 1 << 18, 1 << 18, 7)])
def test_workspace_by_flags(bmm, m, k, n, d):
    a_bytes = m * (k // 64) * 8
    b_bytes = n * (k // 64) * 8

    def ws(**kw):
        return bmm.bmm_gf2_strassen_workspace(m, k, n, d, **kw)[0]

    full = ws()
    assert full == ws(b_transposed=True)  # B^T is copied so it can change basis
    assert full - ws(inplace_basis=True) == a_bytes  # A changes in place
    assert full - ws(inplace_basis=True, b_transposed=True) == a_bytes + b_bytes
    assert full - ws(alt_basis_io=True) == a_bytes
    assert full - ws(alt_basis_io=True, b_transposed=True) == a_bytes + b_bytes
    # the alternative-basis input is never changed, so in place adds nothing to it
    assert ws(alt_basis_io=True, inplace_basis=True) == ws(alt_basis_io=True)


def test_headline_workspace_drops(bmm):
    """n = 2^18, depth 7 (3 serial + 4 parallel levels): in-place changes with B
    passed transposed save both 8 GiB operand copies."""
    n = 1 << 18
    o = bmm.Options(depth_serial=3, depth_parallel=4)
    full = bmm.bmm_gf2_strassen_workspace(n, n, n, 7, o)[0]
    lean = bmm.bmm_gf2_strassen_workspace(n, n, n, 7, o, inplace_basis=True,
                                          b_transposed=True)[0]
    assert full - lean == 16 << 30


def test_shifted_leaf_plan(bmm):
    """The shifted leaf level drops the last level's expanded operands and products
    from the workspace; it needs a parallel level, the int8 leaf and a scheme with
    weight-2 combinations (Winograd keeps the plain plan)."""
    n = 1 << 18
    base = dict(depth_serial=3, depth_parallel=4, leaf=2)
    plain = bmm.bmm_gf2_strassen_workspace(n, n, n, 7, bmm.Options(shift=0, **base))[0]
    shifted = bmm.bmm_gf2_strassen_workspace(n, n, n, 7, bmm.Options(shift=1, **base))[0]
    # 7^4 leaves of 2048^2 bits: T, S and Q at the last level (the 7^3 level they come
    # from is expanded one level at a time instead of two, and stays)
    last = 3 * 7 ** 4 * (2048 * 2048 // 8)
    level6 = 3 * 7 ** 3 * (4096 * 4096 // 8)
    assert plain - shifted == last - level6
    for o in [bmm.Options(shift=1, scheme=2, **base),            # Winograd
              bmm.Options(shift=1, leaf=1, depth_serial=3, depth_parallel=4),  # VALU leaf
              bmm.Options(shift=1, leaf=2, depth_serial=7, depth_parallel=0)]:  # no parallel
        ref = bmm.Options(**{f: getattr(o, f) for f, _ in bmm.Options._fields_})
        ref.shift = 0
        assert (bmm.bmm_gf2_strassen_workspace(n, n, n, 7, o)[0]
                == bmm.bmm_gf2_strassen_workspace(n, n, n, 7, ref)[0])
    with pytest.raises(bmm.BmmError):
        bmm.bmm_gf2_strassen_workspace(n, n, n, 7, bmm.Options(shift=3))


def test_lean_workspace_plan(bmm):
    """The lean depth-first levels hold one child of T, S and Q instead of seven: at
    n = 2^18, depth 7 (3 + 4) the serial levels drop from 7 * 3 * (2 + 0.5 + 0.125) GiB to
    a seventh of that."""
    n = 1 << 18
    base = dict(depth_serial=3, depth_parallel=4, leaf=2)
    full = bmm.bmm_gf2_strassen_workspace(n, n, n, 7, bmm.Options(**base))[0]
    lean = bmm.bmm_gf2_strassen_workspace(
        n, n, n, 7, bmm.Options(flags=bmm.FLAG_LEAN_WORKSPACE, **base))[0]
    serial = sum(3 * ((n >> l) ** 2 // 8) for l in (1, 2, 3))
    assert full - lean == 6 * serial
