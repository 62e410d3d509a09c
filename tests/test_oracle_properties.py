"""Invariants of the oracle's K~ over many random compressions.

Each property below is fixed by the method itself, not by the oracle's code:

* K~ W is linear in W (every step of Sec. 2.3 is a matrix product), so
  K~(aW1 + bW2) = a K~W1 + b K~W2 to rounding.
* K~ is symmetric once the far lists are refined (Sec. 2.2), so the probes
  x^T (K~ y) and y^T (K~ x) agree; this is checked at a size where assembling
  K~ is already costly, through two tree walks only.
* For random sizes, leaf sizes, ranks, budgets and kernels: the tree is a
  balanced partition of the indices (Alg. 1), every leaf is in its own near
  list and the near lists are symmetric with at most floor(budget N / m)
  others chosen per leaf (Alg. 2), the near and far lists together cover every
  pair of leaves exactly once (Sec. 2.2), skeletons are nested with ranks in
  [1, s] (Sec. 2.1), and the tree walk equals K~ assembled block by block.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import workloads
from oracle import cfile, compress, evaluate, kernels


def _points_kernel(n, d, kind, h, seed):
    rng = np.random.default_rng(seed)
    return kernels.KernelMatrix(rng.random((n, d)), kind, h, 1e-3)


def test_linearity_in_w():
    K = _points_kernel(2048, 3, "gaussian", 0.4, 21)
    c = compress.compress(K, 2048, leaf_size=128, max_rank=48, tol=1e-6, kappa=16, budget=0.05, seed=2)
    W1 = workloads.rhs(c.n, 3, 1)
    W2 = workloads.rhs(c.n, 3, 2)
    a, b = 0.75, -2.5
    lhs = evaluate.tree_walk(c, K, a * W1 + b * W2)
    rhs = a * evaluate.tree_walk(c, K, W1) + b * evaluate.tree_walk(c, K, W2)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)


@pytest.mark.parametrize("kind,h,budget", [("gaussian", 0.4, 0.03), ("imq", 0.3, 0.0)])
def test_probe_symmetry_at_n4096(kind, h, budget):
    K = _points_kernel(4096, 4, kind, h, 33)
    c = compress.compress(K, 4096, leaf_size=128, max_rank=64, tol=1e-5, kappa=16, budget=budget, seed=7)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((c.n, 1))
    y = rng.standard_normal((c.n, 1))
    xKy = float(x[:, 0] @ evaluate.tree_walk(c, K, y)[:, 0])
    yKx = float(y[:, 0] @ evaluate.tree_walk(c, K, x)[:, 0])
    scale = np.linalg.norm(x) * np.linalg.norm(y) * K(np.arange(1), np.arange(1))[0, 0]
    assert abs(xKy - yKx) <= 1e-12 * scale


def _check_invariants(c, K, n, m, s, budget):
    D = c.depth
    fl = cfile.first_leaf(D)
    L = 1 << D
    # Alg. 1: a balanced binary partition of 0..n-1
    assert np.array_equal(np.sort(c.perm), np.arange(n))
    sizes = c.node_size[fl:]
    assert sizes.max() - sizes.min() <= 1 and sizes.max() <= m
    for h in range(fl):
        assert c.node_size[h] == c.node_size[2 * h + 1] + c.node_size[2 * h + 2]
        assert c.node_start[2 * h + 1] == c.node_start[h]
        assert c.node_start[2 * h + 2] == c.node_start[h] + c.node_size[2 * h + 1]
    # Alg. 2: near lists (heap ids of leaves)
    cap = int(np.floor(budget * n / m + 1e-12))
    near = [set(int(a) - fl for a in c.near[b]) for b in range(L)]
    for b in range(L):
        assert b in near[b]
        for a in near[b]:
            assert b in near[a]
    assert sum(len(x) - 1 for x in near) <= 2 * cap * L     # each leaf chose at most cap others
    # Sec. 2.2: near and far cover each pair of leaves once
    cnt = np.zeros((L, L), dtype=int)
    for b in range(L):
        for a in near[b]:
            cnt[b, a] += 1
    for h in range(c.nn):
        for a in c.far[h]:
            assert not compress._contains(int(a), h) and not compress._contains(h, int(a))
            for bl in range(L):
                if compress._contains(h, fl + bl):
                    for al in range(L):
                        if compress._contains(int(a), fl + al):
                            cnt[bl, al] += 1
    assert np.all(cnt == 1)
    # Sec. 2.1: nested skeletons, ranks in [1, s]
    for h in range(1, c.nn):
        assert 1 <= c.rank(h) <= s
        if h < fl:
            assert set(c.skel[h]) <= set(c.skel[2 * h + 1]) | set(c.skel[2 * h + 2])
        else:
            assert set(c.skel[h]) <= set(c.indices(h))
    # K~ symmetric and the walk equals the assembly
    Kt = evaluate.assemble(c, K)
    assert np.linalg.norm(Kt - Kt.T) <= 1e-13 * max(1.0, np.linalg.norm(Kt))
    W = workloads.rhs(n, 2, 4)
    U = evaluate.tree_walk(c, K, W)
    assert np.linalg.norm(U - Kt @ W) <= 1e-12 * max(1.0, np.linalg.norm(U))


@settings(max_examples=40, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(n=st.integers(33, 520), m=st.sampled_from([8, 16, 32, 64]), s=st.integers(2, 40),
       budget=st.sampled_from([0.0, 0.02, 0.1, 0.5]), kind=st.sampled_from(["gaussian", "imq"]),
       kappa=st.integers(1, 24), seed=st.integers(0, 2 ** 16))
def test_random_compressions_keep_the_invariants(n, m, s, budget, kind, kappa, seed):
    kappa = min(kappa, n)
    K = _points_kernel(n, 3, kind, 0.35, seed)
    c = compress.compress(K, n, leaf_size=m, max_rank=s, tol=1e-7, kappa=kappa, budget=budget, seed=seed)
    _check_invariants(c, K, n, m, s, budget)
