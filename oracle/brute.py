"""Unpacked brute force and bit packing for tiny inputs.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Bit j of a packed row is bit
j % 64 of word j // 64 (LSB first).
"""
import numpy as np


def pack(bits):
    """(r x c) 0/1 array -> (r x ceil(c/64)) packed uint64."""
    bits = np.asarray(bits, dtype=np.uint8)
    r, c = bits.shape
    nw = (c + 63) // 64
    padded = np.zeros((r, nw * 64), dtype=np.uint8)
    padded[:, :c] = bits
    by = np.packbits(padded, axis=1, bitorder="little")
    return np.ascontiguousarray(by).view("<u8").astype(np.uint64).reshape(r, nw)


def unpack(words, c):
    """(r x nw) packed uint64 -> (r x c) 0/1 uint8 array."""
    w = np.ascontiguousarray(np.asarray(words, dtype=np.uint64)).astype("<u8")
    by = w.view(np.uint8).reshape(w.shape[0], -1)
    return np.unpackbits(by, axis=1, bitorder="little")[:, :c]


def loops(A, B, boolean=False):
    """Triple loop over unpacked bits, one bit product at a time."""
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), dtype=np.uint8)
    for i in range(m):
        for kk in range(n):
            acc = 0
            for j in range(k):
                prod = int(A[i, j]) & int(B[j, kk])
                acc = (acc | prod) if boolean else (acc ^ prod)
            C[i, kk] = acc
    return C


def matmul(A, B, boolean=False):
    """Integer matmul of unpacked bits, then > 0 (Boolean) or & 1 (GF(2))."""
    P = A.astype(np.int64) @ B.astype(np.int64)
    return (P > 0).astype(np.uint8) if boolean else (P & 1).astype(np.uint8)
