"""Plain GOFMM compression in FP64 (oracle side, test infrastructure).

Steps, in the order of the paper's Compress algorithm (Alg. "Compress"):

  distances     Gram-l2 d_ij^2 = K_ii + K_jj - 2 K_ij (Sec. 2.1, eq. 3),
                clamped at 0; Gram angle d_ij = 1 - K_ij^2 / (K_ii K_jj)
                (eq. 4), clamped to [0, 1].
  neighbours    exact kappa-NN by brute force (the limit of the iterative
                randomized-tree search of Sec. 2.2; an index is its own
                nearest neighbour).
  tree          metricSplit (Alg. 1): centroid c of a sample of n_c = min(|a|,
                32) Gram vectors, p = argmax d(i, c), q = argmax d(i, p),
                median split of d_ip - d_iq; left child takes ceil(n/2).
                Depth D = smallest with ceil(N / 2^D) <= m.
  Near          LeafNear (Alg. 2) with the ballot of eq. (budget): every leaf
                keeps itself and at most floor(budget * N / m) other leaves,
                most votes first (ties by leaf id); then made symmetric by
                union.
  Far           FindFar (Alg. 3) per leaf from the root, MergeFar (Alg. 4) in
                postorder, then the common refinement of the far pairs with
                their transposes so that K~ is exactly symmetric.
  skeletons     nested ID (eqs. 7-8, Alg. 5) in postorder on every non-root
                node: rows I' = neighbours outside the node by votes (at most
                half), filled with uniform draws, |I'| = min(N - |a|, 2 ncols); QR with
                column pivoting (LAPACK GEQP3 through SciPy); rank s = smallest
                k >= 1 with |R_kk| < tau |R_00|, at most min(s_max, ncols,
                |I'|); P = [I, R11^-1 R12] Pi^T.

Readings where the paper is silent are listed in the repository's design
notes; each is marked "reading" below.

Parity: pinned by the worked FindFar/MergeFar example of the paper's Fig. 2,
the HSS closed form Far(a) = {sibling(a)}, brute-force Gram-vector distances,
and the closed forms of K~ (full rank, all-near, single leaf => K~ = K).
"""
from __future__ import annotations

from typing import Callable, Dict, List, Optional, Set, Tuple

import numpy as np
import scipy.linalg

from .cfile import Compression, first_leaf, level_of, n_nodes

GRAM_L2 = 0
ANGLE = 1


# ---------------------------------------------------------------- distances
def distance(K, diag: np.ndarray, I, J, kind: int) -> np.ndarray:
    """Matrix of d_ij for i in I, j in J (eq. 3 takes the square root)."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    kij = K(I, J)
    if kind == GRAM_L2:
        d2 = diag[I][:, None] + diag[J][None, :] - 2.0 * kij
        return np.sqrt(np.maximum(d2, 0.0))
    if kind == ANGLE:
        d = 1.0 - kij * kij / (diag[I][:, None] * diag[J][None, :])
        return np.clip(d, 0.0, 1.0)
    raise ValueError(kind)


def depth_for(n: int, m: int) -> int:
    d = 0
    while -(-n // (1 << d)) > m:
        d += 1
    return d


# ---------------------------------------------------------------- neighbours
def exact_knn(K, diag, n: int, kappa: int, kind: int) -> np.ndarray:
    """kappa nearest indices of every index, ordered by (distance, index)."""
    kappa = min(kappa, n)
    out = np.empty((n, kappa), dtype=np.int64)
    allj = np.arange(n)
    for a in range(0, n, 512):
        I = allj[a:a + 512]
        d = distance(K, diag, I, allj, kind)
        for t, i in enumerate(I):
            order = np.lexsort((allj, d[t]))
            out[i] = order[:kappa]
    return out


# ---------------------------------------------------------------- tree
def metric_split(idx: np.ndarray, K, diag, kind: int, rng) -> Tuple[np.ndarray, np.ndarray, int, int, np.ndarray]:
    """Alg. 1 on the (ascending) index set idx. Returns left, right, p, q, sample."""
    n = len(idx)
    nc = min(n, 32)
    C = np.sort(rng.choice(idx, size=nc, replace=False))
    kic = K(idx, C)
    kcc = K(C, C)
    if kind == GRAM_L2:
        # |phi_i - c|^2 up to the constant |c|^2, which argmax ignores
        dc = diag[idx] - 2.0 * kic.mean(axis=1)
    else:
        ip = kic.mean(axis=1)
        dc = 1.0 - ip * ip / (diag[idx] * kcc.mean())
    p = int(idx[int(np.argmax(dc))])            # first maximum = smallest index
    dp = distance(K, diag, idx, [p], kind)[:, 0]
    q = int(idx[int(np.argmax(dp))])
    dq = distance(K, diag, idx, [q], kind)[:, 0]
    order = np.lexsort((idx, dp - dq))           # by value, then index
    nl = (n + 1) // 2
    return np.sort(idx[order[:nl]]), np.sort(idx[order[nl:]]), p, q, C


# ---------------------------------------------------------------- lists
def leaf_near(knn: np.ndarray, leaf_of: np.ndarray, leaves: List[np.ndarray],
              budget: float, n: int, m: int) -> List[np.ndarray]:
    """Alg. 2 with the ballot; returns Near(b) as leaf numbers, then symmetric."""
    L = len(leaves)
    cap = int(np.floor(budget * n / m + 1e-12))
    near: List[Set[int]] = []
    for b in range(L):
        votes: Dict[int, int] = {}
        for i in leaves[b]:
            for j in knn[i]:
                a = int(leaf_of[j])
                votes[a] = votes.get(a, 0) + 1
        cands = sorted((a for a in votes if a != b), key=lambda a: (-votes[a], a))
        near.append({b, *cands[:cap]})
    for b in range(L):
        for a in list(near[b]):
            near[a].add(b)
    return [np.array(sorted(s), dtype=np.int64) for s in near]


def _contains(h: int, leaf_heap: int) -> bool:
    """Is leaf (heap id) in the subtree of node h?  Compare the ancestor of the
    leaf at h's level with h (the MortonID prefix test)."""
    up = level_of(leaf_heap) - level_of(h)
    if up < 0:
        return False
    x = leaf_heap
    for _ in range(up):
        x = (x - 1) // 2
    return x == h


def find_far(depth: int, near_heap: Set[int]) -> List[int]:
    """Alg. 3 for one leaf: descend while the subtree holds a Near leaf.

    A leaf reached by the descent is either in Near (a near pair, nothing is
    added) or not (it is added to Far)."""
    fl = first_leaf(depth)
    out: List[int] = []

    def rec(h: int):
        if h >= fl:
            if h not in near_heap:
                out.append(h)
            return
        if any(_contains(h, a) for a in near_heap):
            rec(2 * h + 1)
            rec(2 * h + 2)
        else:
            out.append(h)

    rec(0)
    return out


def merge_far(depth: int, far: List[Set[int]], at: int = 0):
    """Alg. 4 in postorder from node `at`: move Far(l) & Far(r) up to the parent."""
    fl = first_leaf(depth)

    def rec(h: int):
        if h >= fl:
            return
        l, r = 2 * h + 1, 2 * h + 2
        rec(l)
        rec(r)
        common = far[l] & far[r]
        far[h] = set(common)
        far[l] -= common
        far[r] -= common

    rec(at)


def symmetric_refinement(depth: int, far: List[Set[int]], near: List[np.ndarray]) -> List[Set[int]]:
    """Common refinement of the far pairs T and their transposes (reading).

    For every far ordered leaf pair (b, a), take the covering pair (B, A) in T
    and the covering pair (B', A') in T^T; the refined pair is (deeper of B,
    B'; deeper of A, A').  The result is symmetric and equals T when T is."""
    fl = first_leaf(depth)
    L = 1 << depth
    nn = n_nodes(depth)
    owner: Dict[Tuple[int, int], Tuple[int, int]] = {}
    anc = [[0] * (depth + 1) for _ in range(L)]
    for b in range(L):
        x = fl + b
        for lev in range(depth, -1, -1):
            anc[b][lev] = x
            x = (x - 1) // 2 if x > 0 else 0
    pair_set = {(bh, ah) for bh in range(nn) for ah in far[bh]}

    def cover(b: int, a: int) -> Tuple[int, int]:
        for lb in range(depth, -1, -1):
            B = anc[b][lb]
            for la in range(depth, -1, -1):
                A = anc[a][la]
                if (B, A) in pair_set:
                    return B, A
        raise AssertionError(f"leaf pair {(b, a)} not covered")

    new: List[Set[int]] = [set() for _ in range(nn)]
    nearset = [set(int(x) for x in near[b]) for b in range(L)]
    for b in range(L):
        for a in range(L):
            if a in nearset[b]:
                continue
            B, A = cover(b, a)
            A2, B2 = cover(a, b)            # (A2, B2) in T  =>  (B2, A2) in T^T
            Bn = B if level_of(B) >= level_of(B2) else B2
            An = A if level_of(A) >= level_of(A2) else A2
            new[Bn].add(An)
    return new


# ---------------------------------------------------------------- skeletons
def interp_decomp(A: np.ndarray, tol: float, smax: int) -> Tuple[np.ndarray, np.ndarray]:
    """ID of A (rows x cols): returns pivot columns J (length s) and P (s x cols)
    with A ~= A[:, J] P (eq. 7)."""
    nrow, ncol = A.shape
    _, R, piv = scipy.linalg.qr(A, mode="economic", pivoting=True)
    dg = np.abs(np.diag(R))
    kmax = max(1, min(smax, ncol, nrow))
    if dg[0] == 0.0:
        P = np.zeros((1, ncol))
        P[0, piv[0]] = 1.0
        return piv[:1].copy(), P
    s = 1
    while s < kmax and dg[s] >= tol * dg[0]:
        s += 1
    P = np.zeros((s, ncol))
    P[np.arange(s), piv[:s]] = 1.0
    if s < ncol:
        T = scipy.linalg.solve_triangular(R[:s, :s], R[:s, s:], lower=False)
        P[:, piv[s:]] = T
    return piv[:s].copy(), P


def sample_rows(members: np.ndarray, knn: np.ndarray, n: int, ncols: int, rng) -> np.ndarray:
    """I': neighbours of the node outside it, most votes first (ties by index),
    at most half of the rows, then uniform draws from the rest of the
    complement (reading: |I'| = min(N - |a|, 2 ncols))."""
    ns = min(n - len(members), 2 * ncols)
    inside = np.zeros(n, dtype=bool)
    inside[members] = True
    flat = knn[members].reshape(-1)
    flat = flat[~inside[flat]]
    if flat.size:
        ids, cnt = np.unique(flat, return_counts=True)
        order = np.lexsort((ids, -cnt))
        take = ids[order][:ns // 2]
    else:
        take = np.zeros(0, dtype=np.int64)
    if len(take) < ns:
        used = inside.copy()
        used[take] = True
        pool = np.flatnonzero(~used)
        extra = rng.choice(pool, size=ns - len(take), replace=False)
        take = np.concatenate([take, np.sort(extra)])
    return take.astype(np.int64)


# ---------------------------------------------------------------- top level
def compress(K, n: int, *, leaf_size: int, max_rank: int, tol: float, kappa: int,
             budget: float, distance_kind: int = GRAM_L2, seed: int = 0,
             knn: Optional[np.ndarray] = None, refine: bool = True) -> Compression:
    diag = np.asarray(K.diag(), dtype=np.float64)
    if not np.all(np.isfinite(diag)) or np.any(diag <= 0):
        raise ValueError("K is not SPD: non-positive or non-finite diagonal")
    rng = np.random.default_rng(seed)
    D = depth_for(n, leaf_size)
    nn = n_nodes(D)
    fl = first_leaf(D)
    L = 1 << D
    if knn is None:
        knn = exact_knn(K, diag, n, kappa, distance_kind)

    # tree (PRE): heap order visits parents before children
    members: List[Optional[np.ndarray]] = [None] * nn
    members[0] = np.arange(n, dtype=np.int64)
    split_p = np.full(nn, -1, dtype=np.int64)
    split_q = np.full(nn, -1, dtype=np.int64)
    centroid: List[np.ndarray] = [np.zeros(0, dtype=np.int64) for _ in range(nn)]
    for h in range(fl):
        l, r, p, q, C = metric_split(members[h], K, diag, distance_kind, rng)
        members[2 * h + 1], members[2 * h + 2] = l, r
        split_p[h], split_q[h], centroid[h] = p, q, C
    perm = np.concatenate([members[fl + b] for b in range(L)])
    node_start = np.zeros(nn, dtype=np.int64)
    node_size = np.zeros(nn, dtype=np.int64)
    pos = 0
    for b in range(L):
        node_start[fl + b] = pos
        node_size[fl + b] = len(members[fl + b])
        pos += len(members[fl + b])
    for h in range(fl - 1, -1, -1):
        node_start[h] = node_start[2 * h + 1]
        node_size[h] = node_size[2 * h + 1] + node_size[2 * h + 2]
    leaf_of = np.empty(n, dtype=np.int64)
    for b in range(L):
        leaf_of[members[fl + b]] = b
    leaves = [members[fl + b] for b in range(L)]

    # Near, Far
    near = leaf_near(knn, leaf_of, leaves, budget, n, leaf_size)
    far: List[Set[int]] = [set() for _ in range(nn)]
    for b in range(L):
        far[fl + b] = set(find_far(D, {fl + int(a) for a in near[b]}))
    merge_far(D, far)
    if far[0]:
        raise AssertionError("root received a far list")
    if refine:
        far = symmetric_refinement(D, far, near)

    # skeletons (POST): reverse heap order visits children before parents
    skel: List[np.ndarray] = [np.zeros(0, dtype=np.int64) for _ in range(nn)]
    samp: List[np.ndarray] = [np.zeros(0, dtype=np.int64) for _ in range(nn)]
    proj: List[Optional[np.ndarray]] = [None] * nn
    for h in range(nn - 1, 0, -1):
        if h >= fl:
            cols = perm[node_start[h]:node_start[h] + node_size[h]]
        else:
            cols = np.concatenate([skel[2 * h + 1], skel[2 * h + 2]])
        rows = sample_rows(members[h], knn, n, len(cols), rng)
        if len(rows) == 0:       # a node holding every index has nothing to skeletonize
            raise AssertionError("empty sample")
        piv, P = interp_decomp(K(rows, cols), tol, max_rank)
        skel[h] = cols[piv]
        samp[h] = rows
        proj[h] = P

    return Compression(
        n=n, depth=D, leaf_size=leaf_size, max_rank=max_rank, tol=tol, kappa=kappa,
        budget=budget, distance=distance_kind, perm=perm, node_start=node_start,
        node_size=node_size, split_p=split_p, split_q=split_q, centroid=centroid,
        knn=knn, near=[np.array([fl + int(a) for a in near[b]], dtype=np.int64) for b in range(L)],
        far=[np.array(sorted(far[h]), dtype=np.int64) for h in range(nn)],
        skel=skel, samp=samp, proj=proj)
