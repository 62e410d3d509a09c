"""Interpolative decompositions on the device (params.device_id; Alg.
Skeletonize, eqs. 7-8: pivoted QR in FP64 stopped at the adaptive rank, then
R11^{-1} R12), every node of a tree level in one batch, through the C ABI.

The device follows the host factorization step by step with the same
rounding, so the whole compression must be the host's bit for bit:
skeletons, P, row samples, lists.  Cases: ragged trees with FMM lists, both
distances, ranks stopped by the tolerance and by the cap, full rank
(tol = 0), zero sampled blocks (a diagonal matrix: every node keeps one
column), the N=65536 and N=262144 workloads (host and device timed).  The
host factorization itself is pinned against LAPACK's pivoted QR on the CPU
(tests/test_host_library.py).
"""
import time

import numpy as np
import pytest

import workloads
from gpu_util import export_read, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    import paper_1707_00164_amd as lib
    lib.lib()
    return lib


def _same(a, b):
    assert np.array_equal(a.perm, b.perm)
    for x, y in zip(a.skel, b.skel):
        assert np.array_equal(x, y)
    for x, y in zip(a.samp, b.samp):
        assert np.array_equal(x, y)
    for h, (x, y) in enumerate(zip(a.proj, b.proj)):
        if x is None or y is None:
            assert x is None and y is None
            continue
        assert x.shape == y.shape and np.array_equal(x, y), h
    for x, y in zip(a.far, b.far):
        assert np.array_equal(x, y)


def _pair(g, S, **kw):
    t0 = time.perf_counter()
    host = g.Compression.compress(S, device_id=0, **kw)
    t1 = time.perf_counter()
    dev = g.Compression.compress(S, device_id=1, **kw)
    t2 = time.perf_counter()
    return export_read(host), export_read(dev), t1 - t0, t2 - t1


@pytest.mark.parametrize("distance", [0, 1])
@pytest.mark.parametrize("max_rank,tol", [(64, 1e-6), (24, 1e-9), (400, 0.0)])
def test_ragged_tree_same_bits(g, distance, max_rank, tol):
    rng = np.random.default_rng(31)
    n = 3001
    pts = rng.random((n, 3))
    S = g.KernelSampler(pts, "imq", 0.3, 1e-2)
    log(f"case device ID n={n} distance={distance} s={max_rank} tol={tol}")
    host, dev, th, td = _pair(g, S, leaf_size=100, max_rank=max_rank, tol=tol, kappa=16, budget=0.1,
                              distance=distance, seed=4)
    ranks = [len(x) for x in host.skel[1:]]
    log(f"  ranks {min(ranks)}..{max(ranks)}; host {th:.2f} s, device {td:.2f} s")
    _same(host, dev)


def test_zero_blocks_keep_one_column(g):
    n = 700
    S = g.PySampler(lambda I, J: 2.0 * (I[:, None] == J[None, :]), n)
    host, dev, _, _ = _pair(g, S, leaf_size=64, max_rank=32, tol=1e-6, kappa=8, budget=0.0, seed=1, exact_knn=1)
    assert all(len(x) == 1 for x in host.skel[1:])
    _same(host, dev)


def test_clustered_gaussian_n65536_same_bits(g):
    w = workloads.clustered_gaussian()
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    log(f"case device ID {w.name}")
    host, dev, th, td = _pair(g, S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol, kappa=w.kappa,
                              budget=w.budget, seed=w.seed)
    log(f"  compress: host IDs {th:.2f} s, device IDs {td:.2f} s")
    _same(host, dev)


def test_large_imq_n262144_same_bits(g):
    w = workloads.large_imq()
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    log(f"case device ID {w.name}")
    kw = dict(leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol, kappa=w.kappa, budget=w.budget, seed=w.seed)
    out = []
    for dev_id in (0, 1):
        t0 = time.perf_counter()
        c = g.Compression.compress(S, device_id=dev_id, **kw)
        t = time.perf_counter() - t0
        out.append(export_read(c))
        c.free()
        log(f"  compress with {'device' if dev_id else 'host'} IDs: {t:.1f} s")
    _same(out[0], out[1])
