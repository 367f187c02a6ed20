"""Compile the generator's CPU (gcc) and GPU (hipcc, gfx950) shared libraries in place."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CPU_SO = os.path.join(HERE, "libbmmgen_cpu.so")
GPU_SO = os.path.join(HERE, "libbmmgen_gpu.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed-FP32 instruction selection is disabled for every HIP build here.
HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False):
    src_c = os.path.join(HERE, "gen_cpu.c")
    _run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", CPU_SO, src_c], verbose)
    src_h = os.path.join(HERE, "gen_gpu.hip")
    _run([HIPCC] + HIP_FLAGS + ["-o", GPU_SO, src_h], verbose)


if __name__ == "__main__":
    build(verbose=True)
