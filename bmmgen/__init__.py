"""Seeded synthetic bit-matrix inputs, shared by the oracle side and the GPU side.

The specification lives in ``gen_spec.h``.  This module draws input bits only:
it holds no part of the matrix-product arithmetic.  The CPU (C, OpenMP) and
GPU (HIP) implementations must agree bit for bit; the tests check that.

Matrices are packed row-major uint64 with bit j of a row at bit j % 64 of word
j // 64 (LSB first).
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

HALF, POW2, THRESH = 0, 1, 2
GOLDEN = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1

TAG_A = 0xA
TAG_B = 0xB
TAG_SAMPLER = 0x5A
BASE_SEED = 1909015540


def config_seed(c):
    """Seed of workload number c (0-based list of the five workloads)."""
    return BASE_SEED + c


def batched_tag(p, which):
    """Tag of operand `which` ('A' or 'B') of batched problem p."""
    return (p << 8) | (TAG_A if which == "A" else TAG_B)


def freivalds_tag(v):
    return 0xF0000 + v


def hash64(x):
    """Reference splitmix64 finalizer of x + golden gamma, in Python integers."""
    z = (x + GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def thresh_for_inv_sqrt(k):
    """32-bit threshold thr = min(isqrt(floor(2^64 / k)), 2^32 - 1): P(bit) = thr / 2^32 ~ 1/sqrt(k)."""
    return min(math.isqrt((1 << 64) // int(k)), 0xFFFFFFFF)


class Dist:
    """A bit distribution: kind HALF, POW2 (param = e) or THRESH (param = thr)."""

    def __init__(self, kind, param=0):
        self.kind = int(kind)
        self.param = int(param)

    @staticmethod
    def half():
        return Dist(HALF, 0)

    @staticmethod
    def pow2(e):
        return Dist(POW2, e)

    @staticmethod
    def inv_sqrt(k):
        return Dist(THRESH, thresh_for_inv_sqrt(k))

    @property
    def p(self):
        if self.kind == HALF:
            return 0.5
        if self.kind == POW2:
            return 2.0 ** (-self.param)
        return self.param / 2.0 ** 32

    def __repr__(self):
        return f"Dist(kind={self.kind}, param={self.param})"


_cpu = None
_gpu = None


def _load_cpu():
    global _cpu
    if _cpu is None:
        if not os.path.exists(_build.CPU_SO):
            _build.build()
        lib = ctypes.CDLL(_build.CPU_SO)
        lib.bmmgen_fill_cpu.restype = ctypes.c_int
        lib.bmmgen_fill_cpu.argtypes = [ctypes.c_void_p] + [ctypes.c_int64] * 6 + [
            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64]
        lib.bmmgen_hash.restype = ctypes.c_uint64
        lib.bmmgen_hash.argtypes = [ctypes.c_uint64]
        _cpu = lib
    return _cpu


def _load_gpu():
    global _gpu
    if _gpu is None:
        if not os.path.exists(_build.GPU_SO):
            raise RuntimeError("libbmmgen_gpu.so is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_build.GPU_SO)
        lib.bmmgen_fill_gpu.restype = ctypes.c_int
        lib.bmmgen_fill_gpu.argtypes = [ctypes.c_void_p] + [ctypes.c_int64] * 6 + [
            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p]
        _gpu = lib
    return _gpu


def c_hash64(x):
    return int(_load_cpu().bmmgen_hash(x))


def words(cols):
    return (int(cols) + 63) // 64


def fill_cpu(rows, cols, seed, tag, dist, row0=0, w0=0, nwords=None, ld=None):
    """Rows [row0, row0+rows) and words [w0, w0+nwords) of the seeded matrix, as numpy uint64."""
    if nwords is None:
        nwords = words(cols) - w0
    if ld is None:
        ld = nwords
    out = np.zeros((rows, ld), dtype=np.uint64)
    if rows and nwords:
        rc = _load_cpu().bmmgen_fill_cpu(out.ctypes.data, rows, nwords, ld, row0, w0, cols,
                                         seed & MASK64, tag & MASK64, dist.kind, dist.param)
        if rc != 0:
            raise ValueError(f"bmmgen_fill_cpu rejected its arguments (rc={rc})")
    return out


def fill_rows_cpu(row_ids, cols, seed, tag, dist):
    """The listed rows of the seeded matrix, one per output row."""
    row_ids = [int(r) for r in row_ids]
    out = np.zeros((len(row_ids), words(cols)), dtype=np.uint64)
    for i, r in enumerate(row_ids):
        out[i:i + 1] = fill_cpu(1, cols, seed, tag, dist, row0=r)
    return out


def fill_gpu(ptr, rows, cols, ld, seed, tag, dist, row0=0, w0=0, nwords=None, stream=0):
    """Write the seeded matrix into device memory at `ptr` (row pitch ld words)."""
    if nwords is None:
        nwords = words(cols) - w0
    rc = _load_gpu().bmmgen_fill_gpu(ctypes.c_void_p(ptr), rows, nwords, ld, row0, w0, cols,
                                     seed & MASK64, tag & MASK64, dist.kind, dist.param,
                                     ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"bmmgen_fill_gpu failed (rc={rc})")


def fill_tensor(t, rows, cols, seed, tag, dist, row0=0):
    """Fill a contiguous 2-D torch int64 CUDA tensor (rows x ld) on its device's current stream."""
    import torch
    assert t.is_cuda and t.dtype == torch.int64 and t.dim() == 2 and t.is_contiguous()
    stream = torch.cuda.current_stream(t.device).cuda_stream
    fill_gpu(t.data_ptr(), rows, cols, t.shape[1], seed, tag, dist, row0=row0, stream=stream)


def stratified_rows(m, count, seed):
    """`count` row indices, one per stratum of ceil(m / count) rows; the first
    stratum yields row 0 and the last yields row m - 1."""
    count = max(1, min(int(count), int(m)))
    size = -(-m // count)
    rows = []
    for s in range(count):
        lo = s * size
        hi = min(m, lo + size)
        if lo >= hi:
            break
        if s == 0:
            rows.append(0)
        elif hi == m:
            rows.append(m - 1)
        else:
            rows.append(lo + hash64((seed ^ TAG_SAMPLER) * 1000003 + s) % (hi - lo))
    if rows[-1] != m - 1:
        rows.append(m - 1)
    return sorted(set(rows))


def freivalds_vectors(length, count, seed):
    """`count` seeded Bernoulli(1/2) bit vectors of `length` bits (one packed row
    each), vector v drawn under the tag 0xF0000 + v."""
    out = np.zeros((count, words(length)), dtype=np.uint64)
    for v in range(count):
        out[v:v + 1] = fill_cpu(1, length, seed, freivalds_tag(v), Dist.half())
    return out


def batched_shapes(count, seed, lo=256, hi=8192, step=64):
    """Shapes (m, k, n) of a batch of `count` independent products: each size
    drawn log-uniform on [lo, hi] from numpy's PCG64 seeded with `seed`, floored
    to a multiple of `step` and clamped to [lo, hi].  Problem p is over GF(2)
    with Bernoulli(1/2) bits when p is even and Boolean with Bernoulli(1/sqrt(k))
    bits when p is odd (semiring codes 0 and 1)."""
    rng = np.random.default_rng(seed)
    shapes = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(count, 3)))
    shapes = np.clip((shapes // step).astype(np.int64) * step, lo, hi)
    out = []
    for p, (m, k, n) in enumerate(shapes):
        sr = 0 if p % 2 == 0 else 1
        dist = Dist.half() if sr == 0 else Dist.inv_sqrt(int(k))
        out.append((sr, int(m), int(k), int(n), dist))
    return out
