"""Neighbour lists merged on the device (params.device_knn; the ANN task of
Sec. 2.2 and Table 2) against the oracle and the host path, through the C ABI.

* Brute force (exact_knn): every index's kappa nearest by (distance, index)
  must equal the oracle's exact_knn bit for bit.  Both sides read the same
  FP64 entries (the library samples the oracle's own kernel through a Python
  sampler) and decide in FP64 with the same formula, so any difference is a
  mistake, not rounding.  Gram-l2 and angle distances.
* Randomized trees (the default search): the device merges must give the
  same lists as the host merges of the same trees and blocks, and so the same
  compression; ragged leaves (N = 3001) and the N=65536 clustered workload.
"""
import numpy as np
import pytest

import workloads
from gpu_util import export_read, log
from oracle import compress as ocompress, kernels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    import paper_1707_00164_amd as lib
    lib.lib()
    return lib


@pytest.mark.parametrize("distance", [0, 1])
def test_exact_lists_equal_the_oracle(g, distance):
    w = workloads.small_gaussian()
    pts = workloads.points(w)
    K = kernels.KernelMatrix(pts, w.kernel, w.h, w.shift)
    log(f"case exact device knn n={w.n} distance={distance}")
    S = g.PySampler(K, w.n)
    comp = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=32, tol=1e-3, kappa=w.kappa,
                                  budget=0.0, distance=distance, seed=3, exact_knn=1, device_knn=1)
    got = export_read(comp).knn
    want = ocompress.exact_knn(K, K.diag(), w.n, w.kappa, distance)
    assert got.shape == want.shape
    bad = np.argwhere(got != want)
    assert bad.size == 0, (bad[:5].tolist(), got[bad[0][0]].tolist(), want[bad[0][0]].tolist())


@pytest.mark.parametrize("distance", [0, 1])
def test_tree_search_device_equals_host_ragged(g, distance):
    rng = np.random.default_rng(12)
    n = 3001
    pts = rng.random((n, 3))
    S = g.KernelSampler(pts, "gaussian", 0.3, 1e-3)
    log(f"case tree search n={n} distance={distance}")
    kw = dict(leaf_size=100, max_rank=48, tol=1e-6, kappa=16, budget=0.1, distance=distance, seed=5,
              ann_max_iters=4, ann_target_recall=1.0)
    host = export_read(g.Compression.compress(S, device_knn=0, **kw))
    dev = export_read(g.Compression.compress(S, device_knn=1, **kw))
    assert np.array_equal(dev.knn, host.knn)
    assert np.array_equal(dev.perm, host.perm)
    for a, b in zip(dev.skel, host.skel):
        assert np.array_equal(a, b)


def test_tree_search_device_equals_host_clustered_n65536(g):
    import time
    w = workloads.clustered_gaussian()
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    log(f"case tree search {w.name}")
    kw = dict(leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol, kappa=w.kappa, budget=w.budget, seed=w.seed)
    t0 = time.perf_counter()
    host = export_read(g.Compression.compress(S, device_knn=0, **kw))
    t1 = time.perf_counter()
    dev = export_read(g.Compression.compress(S, device_knn=1, **kw))
    t2 = time.perf_counter()
    log(f"  compress with host merges {t1 - t0:.2f} s, device merges {t2 - t1:.2f} s")
    assert np.array_equal(dev.knn, host.knn)
    assert np.array_equal(dev.perm, host.perm)
