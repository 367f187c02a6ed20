"""Helpers for the GPU parity tests: move packed numpy matrices to and from
torch device tensors.  No product arithmetic here."""
import sys

import numpy as np


def announce(*what):
    """Name the case before a GPU step, so a fault report says which one ran."""
    print("[gpu-case]", *what, flush=True)
    sys.stdout.flush()


def to_dev(x, ld=None):
    import torch
    x = np.ascontiguousarray(x, dtype=np.uint64)
    if ld is not None and ld != x.shape[1]:
        y = np.zeros((x.shape[0], ld), dtype=np.uint64)
        y[:, :x.shape[1]] = x
        x = y
    return torch.from_numpy(x.view(np.int64).copy()).cuda()


def from_dev(t, cols_words=None):
    import torch
    torch.cuda.synchronize()
    a = t.cpu().numpy().view(np.uint64)
    if cols_words is not None:
        a = a[:, :cols_words]
    return np.ascontiguousarray(a)


def empty_dev(rows, ld, fill=0):
    import torch
    t = torch.empty((rows, ld), dtype=torch.int64, device="cuda")
    t.fill_(fill)
    return t


def words(bits):
    return (int(bits) + 63) // 64
