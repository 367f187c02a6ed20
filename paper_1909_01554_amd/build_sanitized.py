"""A build of the library whose host logic carries AddressSanitizer and
UndefinedBehaviorSanitizer, for CPU tests (argument checks, Strassen plans, batched
queue segmentation, out-of-core schedules, autotune tables): the pure host sources
(api.cpp, batched_api.cpp, ooc.cpp) are compiled host-only with the sanitizers and
linked with the product build's objects of the kernel sources (their device code and
thin launchers, unsanitized), which the product build leaves in _build/.

    python -m paper_1909_01554_amd.build_sanitized   # prints the library path

Run tests against it with the sanitizer runtime preloaded (see runtime()) and
BMM_LIBRARY naming the built library."""
import concurrent.futures
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "_build", "san")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = os.environ.get("SAN_CLANG", "/opt/rocm/llvm/bin/clang")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


HOST_SOURCES = ["api.cpp", "batched_api.cpp", "ooc.cpp"]


def _kernel_objects():
    """The product build's objects of the kernel sources (built first if missing)."""
    from . import build as _b
    srcs = [s for s in _b.SOURCES if s not in HOST_SOURCES]
    objs = [os.path.join(_b.BUILD, s + ".o") for s in srcs]
    if not all(os.path.exists(o) for o in objs):
        _b.build()
    return objs


def _compile(src):
    out = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = [HIPCC, "--cuda-host-only", "-x", "hip", "-fPIC", "-std=c++17", "-I",
           os.path.join(ROOT, "include")] + SAN + ["-c", os.path.join(HERE, "csrc", src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"sanitized compile failed: {src}\n{r.stderr}")
    return out


def runtime():
    """Path of the sanitizer runtime to preload (LD_PRELOAD) into the interpreter."""
    return subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                          capture_output=True, text=True, check=True).stdout.strip()


def build(jobs=8):
    os.makedirs(OUT, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, HOST_SOURCES))
    objs += _kernel_objects()
    lib = os.path.join(OUT, "libbmm.so")
    subprocess.run([HIPCC, "-shared", "-fPIC"] + SAN + ["-shared-libsan", "-o", lib] + objs,
                   check=True, capture_output=True)
    return lib


if __name__ == "__main__":
    print(build())
