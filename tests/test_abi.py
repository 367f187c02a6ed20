"""CPU-side checks of the C ABI: the library loads, exports every function that
include/bmm.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

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
    import paper_1909_01554_amd as bmm

    class Fake:
        """A stand-in with a data pointer and a row stride; never dereferenced."""
        def __init__(self, ptr, rows, ld):
            self._p, self._r, self._ld = ptr, rows, ld

        def data_ptr(self):
            return self._p

        def dim(self):
            return 2

        def stride(self, i):
            return (self._ld, 1)[i]

    A = Fake(0x10000, 8, 1)
    B = Fake(0x20000, 64, 1)
    C = Fake(0x30000, 8, 1)
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_gf2(A, B, C, 8, 128, 64, stream=0)  # lda 1 < 2 words
    assert e.value.status == -1
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_boolean(A, B, C, -3, 64, 64, stream=0)
    assert e.value.status == -1
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_gf2(A, B, A, 8, 64, 64, stream=0)  # C overlaps A
    assert e.value.status == -1
    # Strassen size rules are checked before any device work
    with pytest.raises(bmm.BmmError) as e:
        bmm.bmm_gf2_strassen_workspace(1002, 1024, 1024, 3)
    assert e.value.status == -2
    nbytes, ds, dp = bmm.bmm_gf2_strassen_workspace(4096, 4096, 4096, 4)
    assert nbytes > 0 and ds + dp == 4


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
    assert bmm.bmm_leaf_tiles(bmm.LEAF_VALU) == 1
    assert bmm.bmm_leaf_tiles(bmm.LEAF_MFMA_I8) == 7
    assert bmm.bmm_leaf_tiles(bmm.LEAF_MFMA_F4) == 7
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_I8, 5) == (256, 256)
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_I8, 1) == (128, 64)
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_F4, 3) == (64, 128)
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_MFMA_I8, 6) == (128, 64)  # 3-deep pipeline
    assert bmm.bmm_leaf_tile_shape(bmm.LEAF_VALU, 1) == (128, 128)
    assert "gfx950" in bmm.bmm_version()


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
