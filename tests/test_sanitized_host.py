"""The host logic under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
tests of the C ABI (argument checks, Strassen plans and workspace sizes, batched
queue segmentation up to the device query, autotune tables) and of the oracle's C
code run against host-only sanitized builds, in a child interpreter with the
sanitizer runtime preloaded.  No GPU is involved."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CPU_TESTS = ["tests/test_abi.py", "tests/test_abi_flags.py", "tests/test_oracle_product.py",
             "tests/test_oracle_algebra.py"]


def test_host_code_under_asan_and_ubsan():
    if not os.path.exists("/opt/rocm/llvm/bin/clang"):
        pytest.skip("no clang with sanitizer runtimes")
    sys.path.insert(0, ROOT)
    from paper_1909_01554_amd import build_sanitized
    from oracle import build as oracle_build
    lib = build_sanitized.build()
    olib = oracle_build.build_sanitized()
    env = dict(os.environ)
    env.update(LD_PRELOAD=build_sanitized.runtime(), BMM_LIBRARY=lib, ORACLE_LIBRARY=olib,
               ASAN_OPTIONS="detect_leaks=0:detect_odr_violation=0:alloc_dealloc_mismatch=0:"
                            "halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               CUDA_VISIBLE_DEVICES="", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider"] + CPU_TESTS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr
