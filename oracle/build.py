"""Compile the oracle's C library (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", SO,
           os.path.join(HERE, "bmm_oracle.c")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build_sanitized():
    """The same library with AddressSanitizer and UndefinedBehaviorSanitizer (clang, to
    share the sanitizer runtime of the library's host-only sanitized build); returns
    its path.  For CPU tests run with that runtime preloaded and ORACLE_LIBRARY set."""
    out = os.path.join(HERE, "_build")
    os.makedirs(out, exist_ok=True)
    so = os.path.join(out, "liboracle_san.so")
    clang = os.environ.get("SAN_CLANG", "/opt/rocm/llvm/bin/clang")
    subprocess.run([clang, "-O1", "-g", "-fopenmp=libgomp", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-shared-libsan", "-o", so, os.path.join(HERE, "bmm_oracle.c")],
                   check=True, capture_output=True)
    return so


if __name__ == "__main__":
    build(verbose=True)
