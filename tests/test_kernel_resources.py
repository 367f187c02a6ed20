"""Register and scratch budgets of the hot kernels, read from their gfx950 code objects.

The leaves' speed rests on occupancy choices: two waves per SIMD (at most 256 registers,
architected plus accumulation) for the matrix-core leaves, four for the VALU outer-product
leaf (at most 128), and no per-lane scratch in their loops.  A change that makes one of
them spill or drop a wave per SIMD stays exact, so the parity tests would not notice; these
checks compile the kernels to assembly with the library's own flags (hipcc cross-compiles
without a GPU) and read each kernel's descriptor."""
import importlib.util
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_01554_amd", "csrc")


def _build_module():
    spec = importlib.util.spec_from_file_location(
        "_bmm_build_flags", os.path.join(ROOT, "paper_1909_01554_amd", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _descriptors(source):
    """{kernel symbol: (next free VGPR incl. accumulation registers, scratch bytes)}."""
    b = _build_module()
    if not shutil.which(b.HIPCC) and not os.path.exists(b.HIPCC):
        pytest.skip("hipcc not available")
    flags = [f for f in b.FLAGS if f not in ("-fPIC", "-Wall")]
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "k.s")
        r = subprocess.run([b.HIPCC] + flags + ["-S", "--cuda-device-only",
                                                os.path.join(CSRC, source), "-o", out],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        asm = open(out).read()
    res = {}
    for m in re.finditer(r"\.amdhsa_kernel (\S+)(.*?)\.end_amdhsa_kernel", asm, re.S):
        body = m.group(2)
        vgpr = int(re.search(r"\.amdhsa_next_free_vgpr\s+(\d+)", body).group(1))
        priv = int(re.search(r"\.amdhsa_private_segment_fixed_size\s+(\d+)", body).group(1))
        res[m.group(1)] = (vgpr, priv)
    return res


@pytest.fixture(scope="module")
def leaf_mfma():
    return _descriptors("leaf_mfma.hip")


def _pick(desc, *parts):
    hits = {k: v for k, v in desc.items() if all(p in k for p in parts)}
    assert hits, f"no kernel matching {parts}"
    return hits


@pytest.mark.slow
@pytest.mark.parametrize("steps", ["Li8E", "Li16E"])
def test_recursion_leaf_fits_two_waves_without_scratch(leaf_mfma, steps):
    """The unrolled 128 x 64 int8 leaf of the recursion (k = 2048: 8 steps, k = 4096: 16
    steps; two buffers, both operand sides expanded by 64-bit shifts)."""
    for name, (vgpr, priv) in _pick(leaf_mfma, "leaf_mfma_kernel", "ELi4ELi2ELi2ELi0ELi2E" + steps,
                                    "Lb1ELb0ELb1E").items():
        assert vgpr <= 256 and priv == 0, (name, vgpr, priv)


@pytest.mark.slow
def test_long_k_leaf_register_budget(leaf_mfma):
    """The chunked 64 x 128 int8 leaf of the cubic products: 256 registers, and only the
    few bytes of scratch its fallback path keeps outside the main loop."""
    for name, (vgpr, priv) in _pick(leaf_mfma, "leaf_mfma_kernel", "ELi2ELi4ELi2ELi0ELi2ELin12E").items():
        assert vgpr <= 256 and priv <= 32, (name, vgpr, priv)


@pytest.mark.slow
def test_batched_lds_items_without_scratch():
    desc = _descriptors("batched.hip")
    for name, (vgpr, priv) in _pick(desc, "batched_lds_kernel").items():
        assert vgpr <= 256 and priv == 0, (name, vgpr, priv)


@pytest.mark.slow
def test_valu_leaves_occupancy():
    """The VALU outer-product leaf needs four waves per SIMD to pair its instructions
    (at most 128 registers); the dot-product leaf runs without scratch."""
    desc = _descriptors("leaf_valu.hip")
    for name, (vgpr, priv) in _pick(desc, "leaf_valu_outer_kernel").items():
        assert vgpr <= 128, (name, vgpr)
    for name, (vgpr, priv) in _pick(desc, "leaf_valu_kernel").items():
        assert priv == 0, (name, vgpr, priv)
