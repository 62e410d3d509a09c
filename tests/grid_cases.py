"""Hand-made compressions on an integer grid (test inputs, CPU and GPU tests).

Every entry of P, K and W is a small integer, so every partial sum that an
evaluation forms is an integer far below 2^24: FP64 on the CPU and FP32 on
the device compute them exactly, in any order.  Any rounding left is the one
a storage form prescribes (BF16 of an operand), which both sides take on the
same exact value.  A device result must therefore equal the oracle's to the
last bit in every storage form, whatever the tile shape.

The structure (tree, Near, Far, skeletons, P) is chosen here so that ranks
and leaf sizes sit on the kernel's tile and slab edges: 1, 31-33, 63-65,
127-129, 255-257, 511-513.  Far lists come from the oracle's FindFar and
MergeFar (Alg. 3, 4) on the chosen Near lists, so every leaf pair is covered
once.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from oracle import cfile, compress

# (leaf sizes, leaf ranks, ranks of the internal levels from D - 1 up to 1)
CASES = {
    "edges_a": ([257, 256, 97, 33, 257, 128, 65, 129], [257, 256, 33, 31, 255, 1, 32, 64],
                [[513, 63, 129, 65], [512, 127]]),
    "edges_b": ([257, 257, 33, 33, 97, 96, 256, 255], [256, 255, 33, 32, 1, 96, 128, 127],
                [[511, 65, 97, 255], [513, 257]]),
}


def build(leaf_sizes: Sequence[int], leaf_ranks: Sequence[int], level_ranks: List[Sequence[int]],
          seed: int = 0):
    """Returns (compression, dense integer matrix A); K(I, J) = A[I, J]."""
    L = len(leaf_sizes)
    D = L.bit_length() - 1
    assert 1 << D == L and len(level_ranks) == max(D - 1, 0)
    rng = np.random.default_rng(seed)
    n = int(sum(leaf_sizes))
    nn = cfile.n_nodes(D)
    fl = cfile.first_leaf(D)
    perm = rng.permutation(n).astype(np.int64)
    node_start = np.zeros(nn, dtype=np.int64)
    node_size = np.zeros(nn, dtype=np.int64)
    pos = 0
    for b in range(L):
        node_start[fl + b], node_size[fl + b] = pos, leaf_sizes[b]
        pos += leaf_sizes[b]
    for h in range(fl - 1, -1, -1):
        node_start[h] = node_start[2 * h + 1]
        node_size[h] = node_size[2 * h + 1] + node_size[2 * h + 2]
    # Near: each leaf, its left and right neighbours in leaf order (symmetric)
    near = [sorted({b, (b + 1) % L, (b - 1) % L}) for b in range(L)]
    far = [set() for _ in range(nn)]
    for b in range(L):
        far[fl + b] = set(compress.find_far(D, {fl + a for a in near[b]}))
    compress.merge_far(D, far)
    rank = {fl + b: leaf_ranks[b] for b in range(L)}
    for lev, rs in zip(range(D - 1, 0, -1), level_ranks):
        for i, s in enumerate(rs):
            rank[(1 << lev) - 1 + i] = s
    skel = [np.zeros(0, dtype=np.int64) for _ in range(nn)]
    proj = [None] * nn
    for h in range(nn - 1, 0, -1):
        if h >= fl:
            cols = perm[node_start[h]:node_start[h] + node_size[h]]
        else:
            cols = np.concatenate([skel[2 * h + 1], skel[2 * h + 2]])
        s = rank[h]
        assert 1 <= s <= len(cols), (h, s, len(cols))
        piv = rng.choice(len(cols), size=s, replace=False)
        skel[h] = cols[piv]
        P = np.zeros((s, len(cols)))
        P[np.arange(s), piv] = 1.0                          # skeleton columns: identity
        others = np.setdiff1d(np.arange(len(cols)), piv)
        if len(others):
            for i in range(s):                              # two more +-1 entries per row
                j = rng.choice(others, size=min(2, len(others)), replace=False)
                P[i, j] = rng.choice([-1.0, 1.0], size=len(j))
        proj[h] = P
    c = cfile.Compression(
        n=n, depth=D, leaf_size=max(leaf_sizes), max_rank=max(rank.values()), tol=0.0, kappa=1,
        budget=0.0, distance=0, perm=perm, node_start=node_start, node_size=node_size,
        split_p=np.full(nn, -1, dtype=np.int64), split_q=np.full(nn, -1, dtype=np.int64),
        centroid=[np.zeros(0, dtype=np.int64) for _ in range(nn)], knn=None,
        near=[np.array([fl + a for a in near[b]], dtype=np.int64) for b in range(L)],
        far=[np.array(sorted(far[h]), dtype=np.int64) for h in range(nn)],
        skel=skel, samp=[np.zeros(0, dtype=np.int64) for _ in range(nn)], proj=proj)
    # symmetric integer matrix: off-diagonal entries in {-1, 0, 1}, diagonal 2
    up = rng.integers(-1, 2, size=(n, n)).astype(np.float64)
    A = np.triu(up, 1)
    A = A + A.T + 2.0 * np.eye(n)
    return c, A


def integer_rhs(n: int, r: int, seed: int) -> np.ndarray:
    """(n, r) right-hand sides with integer entries in [-8, 8]."""
    return np.random.default_rng(seed + 5).integers(-8, 9, size=(n, r)).astype(np.float64)
