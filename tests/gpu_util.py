"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import os
import sys
import tempfile

import numpy as np

import workloads


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    """|a - b|_F / |b|_F."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def export_read(comp):
    """Structure of a library compression, read back by the oracle's reader."""
    from oracle import cfile
    fd, path = tempfile.mkstemp(suffix=".gofmm")
    os.close(fd)
    try:
        comp.export(path)
        return cfile.read(path)
    finally:
        os.unlink(path)


def cuda_rhs(n, r, seed, ld=None):
    """(n, r) FP32 Gaussian right-hand sides on cuda:0 (row stride ld >= r)."""
    import torch
    W64 = workloads.rhs(n, r, seed)
    if ld is None or ld == r:
        Wd = torch.from_numpy(W64.astype(np.float32)).cuda()
    else:
        big = torch.zeros((n, ld), dtype=torch.float32)
        big[:, :r] = torch.from_numpy(W64.astype(np.float32))
        Wd = big.cuda()[:, :r]
    return W64, Wd
