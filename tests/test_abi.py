"""CPU-side checks of the C ABI: the library loads, exports every function that
include/bmm.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bmm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|const char\*)\s*\**\s*(bmm_\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_1909_01554_amd as bmm
    return ctypes.CDLL(bmm.library_path())


def test_header_parses():
    names = declared_functions()
    for n in ["bmm_gf2", "bmm_boolean", "bmm_gf2_strassen", "bmm_batched", "bmm_ooc",
              "bmm_gf2_strassen_workspace", "bmm_batched_plan_create", "bmm_last_error"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_argument_errors_without_gpu():
    """The C side rejects bad sizes, pitches and overlaps before any device work
    (called through ctypes with pointers that are never dereferenced)."""
    import paper_1909_01554_amd as bmm
    vp = ctypes.c_void_p
    o = bmm.Options()

    def gf2(a, lda, b, ldb, c, ldc, m, k, n, fn=None):
        return (fn or bmm._c_gf2)(vp(a), lda, vp(b), ldb, vp(c), ldc, m, k, n,
                                  ctypes.byref(o), None)

    assert gf2(0x10000, 1, 0x20000, 1, 0x30000, 1, 8, 128, 64) == -1  # lda 1 < 2 words
    assert gf2(0x10000, 1, 0x20000, 1, 0x30000, 1, -3, 64, 64, bmm._c_boolean) == -1
    assert gf2(0x10000, 1, 0x20000, 1, 0x10000, 1, 8, 64, 64) == -1  # C overlaps A
    assert gf2(0x10004, 1, 0x20000, 1, 0x30000, 1, 8, 64, 64) == -1  # misaligned A
    assert "aligned" in bmm._c_last_error().decode()
    # Strassen size rules are checked before any device work
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_gf2_strassen_workspace(1002, 1024, 1024, 3)
    assert e.value.status == -2
    nbytes, ds, dp = bmm.bmm_gf2_strassen_workspace(4096, 4096, 4096, 4)
    assert nbytes > 0 and ds + dp == 4


def test_python_binding_checks_tensors():
    """The binding checks dtype, layout and shape against m, k, n (and the device)
    before a pointer crosses the ABI, so a caller's mistake is a ValueError and not an
    out-of-bounds access on the GPU."""
    import torch

    import paper_1909_01554_amd as bmm
    m, k, n = 8, 128, 64
    A = torch.zeros((m, 2), dtype=torch.int64)
    B = torch.zeros((k, 1), dtype=torch.int64)
    C = torch.zeros((m, 1), dtype=torch.int64)
    bad = [
        (A.to(torch.int32), B, C, "A"),                        # 4-byte words
        (A, B.to(torch.float64), C, "B"),                      # floating point
        (A[:, :1], B, C, "A"),                                 # k needs 2 words per row
        (A, B[:64], C, "B"),                                   # B needs k rows
        (A, B, C[:4], "C"),                                    # C needs m rows
        (A.t(), B, C, "A"),                                    # rows not contiguous
        (A, B, C, "GPU"),                                      # right shapes, host memory
    ]
    for a, b, c, what in bad:
        with pytest.raises(ValueError, match=what):
            bmm.bmm_gf2(a, b, c, m, k, n)
        with pytest.raises(ValueError, match=what):
            bmm.bmm_boolean(a, b, c, m, k, n)
    with pytest.raises(ValueError, match="negative"):
        bmm.bmm_gf2(A, B, C, -1, k, n)
    with pytest.raises(TypeError):
        bmm.bmm_gf2(A.numpy(), B, C, m, k, n)
    # B passed transposed must be n x k
    with pytest.raises(ValueError, match="transposed"):
        bmm.bmm_gf2(A, torch.zeros((n - 1, 2), dtype=torch.int64), C, m, k, n,
                    b_transposed=True)
    # Strassen: operands as above, and the workspace must be a GPU tensor
    with pytest.raises(ValueError, match="A"):
        bmm.bmm_gf2_strassen(A[:, :1], B, C, m, k, n, torch.zeros(8, dtype=torch.int64))
    with pytest.raises(ValueError, match="GPU"):
        bmm.bmm_gf2_strassen(A, B, C, m, k, n, torch.zeros(8, dtype=torch.int64))
    # batched problems name the problem
    prob = dict(semiring=bmm.GF2, m=m, k=k, n=n, A=A, B=B[:10], C=C)
    with pytest.raises(ValueError, match="problem 0"):
        bmm.bmm_batched([prob])
    with pytest.raises(ValueError, match="problem 0"):
        bmm.BatchedPlan([prob])
    # stage entry points
    with pytest.raises(ValueError, match="dst"):
        bmm.bmm_transpose(torch.zeros((64, 1), dtype=torch.int64),
                          torch.zeros((63, 1), dtype=torch.int64), 64, 64)
    with pytest.raises(ValueError, match="X"):
        bmm.bmm_basis_change(torch.zeros((64, 1), dtype=torch.int64), 64, 2, 1)
    with pytest.raises(ValueError, match="src"):
        bmm.bmm_expand(0, 1, torch.zeros(10, dtype=torch.int64), 2, 0,
                       torch.zeros(100, dtype=torch.int64), 4, 2, 1)
    with pytest.raises(ValueError, match="dst"):
        bmm.bmm_compress(1, torch.zeros(100, dtype=torch.int64),
                         torch.zeros(5, dtype=torch.int64), 2, 0, 4, 2, 1)
    # out of core: host operands of the right shapes
    import numpy as np
    with pytest.raises(ValueError, match="B"):
        bmm.bmm_ooc(bmm.GF2, np.zeros((m, 2), np.uint64), np.zeros((k - 1, 1), np.uint64),
                    np.zeros((m, 1), np.uint64), m, k, n)


def test_workspace_formula():
    """Workspace = B-hat^T (+ A-hat) + 3 buffers per stored level."""
    import paper_1909_01554_amd as bmm
    n = 1 << 14
    op = bmm.Options(depth_serial=1, depth_parallel=2)
    nbytes, ds, dp = bmm.bmm_gf2_strassen_workspace(n, n, n, 3, op)
    mat = n * n // 8
    want = 2 * mat + 3 * 7 * mat // 4 + 3 * 49 * mat // 16 // 4
    assert (ds, dp) == (1, 2)
    assert nbytes == want
    alt, _, _ = bmm.bmm_gf2_strassen_workspace(n, n, n, 3, op, alt_basis_io=True)
    assert nbytes - alt == mat


def test_leaf_tiles_and_status_strings():
    import paper_1909_01554_amd as bmm
    assert bmm.bmm_leaf_tiles(bmm.LEAF_VALU) == 2
    assert bmm.bmm_leaf_tiles(bmm.LEAF_MFMA_I8) == 8
    assert bmm.bmm_leaf_tiles(bmm.LEAF_MFMA_F4) == 8
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_I8, 5) == (256, 256)
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_I8, 1) == (128, 64)
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_F4, 3) == (64, 128)
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_I8, 6) == (128, 64)  # 3-deep pipeline
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_I8, 8) == (256, 128)  # LDS-shared 2 x 2 waves
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_VALU, 1) == (128, 128)
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_VALU, 2) == (512, 1024)  # outer-product form
    assert "gfx950" in bmm.bmm_version()


def test_options_layout_matches_header(tmp_path):
    """The binding's Options mirrors bmm_options field for field (a C program built
    against include/bmm.h prints the size and offsets)."""
    import paper_1909_01554_amd as bmm
    names = [f for f, _ in bmm.Options._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "bmm.h"\n'
                   'int main(void) {\n  printf("%zu", sizeof(bmm_options));\n' +
                   "".join(f'  printf(" %zu", offsetof(bmm_options, {f}));\n' for f in names) +
                   '  printf("\\n");\n  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(bmm.Options)] + [getattr(bmm.Options, f).offset for f in names]
    assert got == want


def test_k_panel_table_roundtrip(tmp_path):
    """k-panel records load, save and reject malformed lines (panel not a whole number of
    words, unknown semiring)."""
    import paper_1909_01554_amd as bmm
    p = tmp_path / "kp.txt"
    p.write_text("kpanel 1 4096 65536 4096 16384\n")
    bmm.bmm_autotune_load(str(p))
    q = tmp_path / "out.txt"
    bmm.bmm_autotune_save(str(q))
    assert "kpanel 1 4096 65536 4096 16384" in q.read_text()
    for bad in ["kpanel 1 4096 65536 4096 1000\n", "kpanel 5 64 64 64 64\n",
                "kpanel 0 64 0 64 64\n"]:
        p.write_text(bad)
        with pytest.raises(bmm.BmmError):
            bmm.bmm_autotune_load(str(p))
    assert bmm.Options().k_panel == 0


def test_autotune_table_roundtrip(tmp_path):
    import paper_1909_01554_amd as bmm
    bmm.bmm_autotune_set(bmm.GF2, 100, 200, 300, bmm.LEAF_VALU, 1)
    p = tmp_path / "tune.txt"
    bmm.bmm_autotune_save(str(p))
    assert "leaf 0 100 200 300 1 1 1 0 0" in p.read_text()
    bmm.bmm_autotune_load(str(p))
    with pytest.raises(bmm.BmmError):
        bmm.bmm_autotune_set(bmm.GF2, 1, 1, 1, bmm.LEAF_MFMA_I8, 9)


def test_leaf_choice_follows_the_table(tmp_path):
    """bmm_leaf_choice is host-only: explicit options win, then the table, then the
    default rule (64 x 64 tiles when the launch has fewer than 4096 waves of 128 x 64;
    else for k >= 8192 int8 tile 7, for k >= 4096 fp4 tile 5; else 128 x 64)."""
    import paper_1909_01554_amd as bmm
    p = tmp_path / "t.txt"
    p.write_text("leaf 1 4096 8192 4096 1 3 1 4 5\n")
    bmm.bmm_autotune_load(str(p))
    assert bmm.bmm_leaf_choice(bmm.BOOLEAN, 4096, 8192, 4096) == (3, 5)
    assert bmm.bmm_leaf_choice(bmm.BOOLEAN, 4096, 8192, 4096, options=bmm.Options(leaf=2)) == (2, 4)
    assert bmm.bmm_leaf_choice(bmm.BOOLEAN, 4096, 8192, 4096,
                               options=bmm.Options(leaf=2, tile=3)) == (2, 3)
    assert bmm.bmm_leaf_choice(bmm.GF2, 1 << 16, 1 << 16, 1 << 16) == (2, 7)
    assert bmm.bmm_leaf_choice(bmm.GF2, 1 << 16, 1 << 16, 1 << 16,
                               options=bmm.Options(leaf=3)) == (3, 5)
    assert bmm.bmm_leaf_choice(bmm.GF2, 1 << 16, 4096, 1 << 16) == (2, 1)
    assert bmm.bmm_leaf_choice(bmm.GF2, 1 << 16, 2048, 1 << 16,
                               options=bmm.Options(leaf=3)) == (3, 1)
    assert bmm.bmm_leaf_choice(bmm.GF2, 256, 256, 256) == (2, 2)
    with pytest.raises(bmm.BmmError):
        bmm.bmm_leaf_choice(7, 1, 1, 1)


def test_launch_grid_bound():
    """A launch whose grid would reach 2^32 work-items is refused on the host with
    BMM_E_UNSUPPORTED (never launched truncated): m = n = 2^19 with the VALU leaf
    (128 x 128 per 256-thread workgroup) and the int8 64 x 64 tile (128 x 128 per
    workgroup) both need 2^24 workgroups.  Pointers are never dereferenced."""
    import paper_1909_01554_amd as bmm
    vp = ctypes.c_void_p
    m = n = 1 << 19
    k = 64
    A, B, C = 1 << 32, 2 << 32, 16 << 32
    for leaf, tile in [(bmm.LEAF_VALU, 1), (bmm.LEAF_MFMA_I8, 2)]:
        o = bmm.Options(leaf=leaf, tile=tile, flags=bmm.FLAG_B_TRANSPOSED)
        rc = bmm._c_gf2(vp(A), 1, vp(B), 1, vp(C), n // 64, m, k, n, ctypes.byref(o), None)
        assert rc == -2, (leaf, tile, rc)
        assert "2^32" in bmm._c_last_error().decode()


def test_allocation_failure_hook_arms_and_disarms():
    """The testing hook is exported and takes any count; a negative count disarms."""
    import paper_1909_01554_amd as bmm
    bmm.bmm_debug_fail_allocations(3)
    bmm.bmm_debug_fail_allocations(-1)
    bmm.bmm_debug_fail_allocations(0)
