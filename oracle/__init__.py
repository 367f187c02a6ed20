"""Oracle for packed bit-matrix products: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_1909_01554_amd``) and never imports it.

Contents
--------
* ``mul`` / ``rows`` / ``vecmat``: the plain definition of the product,
  C[i][k] = SUM_j A[i][j] B[j][k] over GF(2) (XOR) or the Boolean algebra (OR),
  as a packed-word triple loop in C (``bmm_oracle.c``).
* ``freivalds``: Freivalds's randomized check over GF(2), built on ``vecmat``.
* ``algebra``: the paper's straight-line programs (section 2) for the
  self-inverse and the chaining alternative-basis algorithms and for
  Strassen-Winograd.
* ``strassen``: stage oracles (basis changes, expansion, compression and the
  recursion) written from the paper's equations, for kernel-by-kernel tests.
* ``brute``: unpacked brute force for tiny inputs.

Packed layout: row-major uint64, bit j of a row at bit j % 64 of word j // 64.
Parity status: every function here is pinned by a ``-m "not gpu"`` test; see
the test files named ``test_oracle_*``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

GF2, BOOLEAN = 0, 1
_lib = None


def _load():
    global _lib
    if _lib is None:
        # ORACLE_LIBRARY: a sanitized build of the same C file (host-logic CPU tests)
        so = os.environ.get("ORACLE_LIBRARY") or _build.SO
        if not os.path.exists(so):
            _build.build()
        lib = ctypes.CDLL(so)
        i64 = ctypes.c_int64
        vp = ctypes.c_void_p
        lib.oracle_rows.argtypes = [ctypes.c_int, vp, i64, i64, vp, i64, vp, i64, i64, i64]
        lib.oracle_mul.argtypes = [ctypes.c_int, vp, i64, vp, i64, vp, i64, i64, i64, i64]
        lib.oracle_vecmat.argtypes = [vp, vp, i64, i64, i64, vp]
        for f in (lib.oracle_rows, lib.oracle_mul, lib.oracle_vecmat):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def words(bits):
    return (int(bits) + 63) // 64


def _as_packed(x, name):
    if x.dtype != np.uint64:
        x = x.view(np.uint64) if x.dtype == np.int64 else x.astype(np.uint64)
    x = np.ascontiguousarray(x)
    if x.ndim != 2:
        raise ValueError(f"{name} must be 2-D packed uint64")
    return x


def mul(A, B, k, n, semiring=GF2):
    """C = AB for packed A (m x ceil(k/64)) and B (k x ceil(n/64)); returns packed C."""
    A = _as_packed(A, "A")
    B = _as_packed(B, "B")
    m = A.shape[0]
    if B.shape[0] < k or A.shape[1] < words(k) or B.shape[1] < words(n):
        raise ValueError("operand shapes do not match k, n")
    C = np.zeros((m, words(n)), dtype=np.uint64)
    rc = _load().oracle_mul(semiring, A.ctypes.data, A.shape[1], B.ctypes.data, B.shape[1],
                            C.ctypes.data, C.shape[1], m, k, n)
    if rc:
        raise ValueError("oracle_mul rejected its arguments")
    return C


def rows(A_rows, B, k, n, semiring=GF2):
    """Rows of C = AB for the given rows of A (streams B once)."""
    A_rows = _as_packed(A_rows, "A_rows")
    B = _as_packed(B, "B")
    R = A_rows.shape[0]
    C = np.zeros((R, words(n)), dtype=np.uint64)
    rc = _load().oracle_rows(semiring, A_rows.ctypes.data, A_rows.shape[1], R, B.ctypes.data,
                             B.shape[1], C.ctypes.data, C.shape[1], k, n)
    if rc:
        raise ValueError("oracle_rows rejected its arguments")
    return C


def vecmat(x, M, rows_, cols):
    """x^T M over GF(2): XOR of the rows of M selected by the bits of x."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint64).reshape(-1))
    M = _as_packed(M, "M")
    y = np.zeros(words(cols), dtype=np.uint64)
    rc = _load().oracle_vecmat(x.ctypes.data, M.ctypes.data, M.shape[1], rows_, cols,
                               y.ctypes.data)
    if rc:
        raise ValueError("oracle_vecmat rejected its arguments")
    return y


def freivalds(A, B, C, m, k, n, xs):
    """Freivalds's check over GF(2): for each bit vector x in xs (length m),
    test (x^T A) B == x^T C.  A wrong C passes one vector with probability at
    most 1/2.  Returns the list of per-vector outcomes."""
    out = []
    for x in xs:
        xa = vecmat(x, A, m, k)
        lhs = vecmat(xa, B, k, n)
        rhs = vecmat(x, C, m, n)
        out.append(bool(np.array_equal(lhs, rhs)))
    return out
