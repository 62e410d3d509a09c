"""K~ W for a given compression, in FP64 (oracle side, test infrastructure).

Two independent ways of computing the same product:

  tree_walk  the paper's Evaluate (Alg. 6), node by node:
               N2S (POST)  leaf:     w~_a = P_a W[a]
                           internal: w~_a = P_a [w~_l; w~_r]
               S2S (ANY)   u~_b = sum over a in Far(b) of K(b~, a~) w~_a
               S2N (PRE)   internal: [u~_l; u~_r] += P_b^T u~_b
                           leaf:     U[b] += P_b^T u~_b
               L2L (ANY)   U[b] += sum over a in Near(b) of K(b, a) W[a]
             (Table 2 and the Evaluation paragraph of Sec. 2.2).
  assemble   the dense matrix K~ = sum_near E_b K_ba E_a^T
                               + sum_far E_b Ph_b^T K(b~, a~) Ph_a E_a^T,
             where Ph_a is the telescoped interpolation matrix of eq.
             (telescope): Ph_leaf = P_leaf, Ph_a = P_a blockdiag(Ph_l, Ph_r).

Every kernel block is re-sampled from the kernel K(I, J) given by the caller,
so nothing computed by the library enters these products except the
structure (tree, skeletons, P, Near, Far) when a library compression is read.

`rows` restricts the output to a sampled row set (the full upward pass is
still needed for the far field).

Parity: tree_walk and assemble agree to 1e-12 (tested); both reduce to K in
the closed-form cases (full rank, all-near, single leaf).
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from .cfile import Compression, first_leaf


def upward(c: Compression, Wp: np.ndarray) -> List[Optional[np.ndarray]]:
    """N2S in postorder on the permuted right-hand sides Wp."""
    fl = first_leaf(c.depth)
    wt: List[Optional[np.ndarray]] = [None] * c.nn
    for h in range(c.nn - 1, 0, -1):
        if h >= fl:
            a = int(c.node_start[h])
            wt[h] = c.proj[h] @ Wp[a:a + int(c.node_size[h])]
        else:
            wt[h] = c.proj[h] @ np.vstack([wt[2 * h + 1], wt[2 * h + 2]])
    return wt


def tree_walk(c: Compression, K, W: np.ndarray, rows: Optional[np.ndarray] = None) -> np.ndarray:
    W = np.asarray(W, dtype=np.float64)
    r = W.shape[1]
    fl = first_leaf(c.depth)
    Wp = W[c.perm]
    wt = upward(c, Wp)
    # which nodes matter for the requested rows (all of them by default)
    pos_of = np.empty(c.n, dtype=np.int64)
    pos_of[c.perm] = np.arange(c.n)
    if rows is None:
        want_leaf = np.ones(1 << c.depth, dtype=bool)
    else:
        want_leaf = np.zeros(1 << c.depth, dtype=bool)
        starts = c.node_start[fl:]
        want_leaf[np.searchsorted(starts, pos_of[np.asarray(rows)], side="right") - 1] = True
    want = np.zeros(c.nn, dtype=bool)
    for b in np.flatnonzero(want_leaf):
        x = fl + int(b)
        while True:
            want[x] = True
            if x == 0:
                break
            x = (x - 1) // 2
    # S2S
    ut: List[Optional[np.ndarray]] = [None] * c.nn
    for h in range(1, c.nn):
        acc = np.zeros((c.rank(h), r))
        if want[h]:
            for a in c.far[h]:
                a = int(a)
                acc += K(c.skel[h], c.skel[a]) @ wt[a]
        ut[h] = acc
    # S2N (PRE: heap order is a valid preorder for this purpose)
    Up = np.zeros((c.n, r))
    for h in range(1, c.nn):
        if not want[h]:
            continue
        if h >= fl:
            a = int(c.node_start[h])
            Up[a:a + int(c.node_size[h])] += c.proj[h].T @ ut[h]
        else:
            d = c.proj[h].T @ ut[h]
            sl = c.rank(2 * h + 1)
            ut[2 * h + 1] = ut[2 * h + 1] + d[:sl]
            ut[2 * h + 2] = ut[2 * h + 2] + d[sl:]
    # L2L
    for b in range(1 << c.depth):
        if not want_leaf[b]:
            continue
        h = fl + b
        a0 = int(c.node_start[h])
        ib = c.indices(h)
        for a in c.near[b]:
            a = int(a)
            s0 = int(c.node_start[a])
            Up[a0:a0 + len(ib)] += K(ib, c.indices(a)) @ Wp[s0:s0 + int(c.node_size[a])]
    U = np.empty_like(Up)
    U[c.perm] = Up
    return U if rows is None else U[np.asarray(rows)]


def telescoped(c: Compression) -> List[Optional[np.ndarray]]:
    """Ph_a (s_a x |a|, columns in permuted order) for every non-root node."""
    fl = first_leaf(c.depth)
    ph: List[Optional[np.ndarray]] = [None] * c.nn
    for h in range(c.nn - 1, 0, -1):
        if h >= fl:
            ph[h] = c.proj[h]
        else:
            l, r = 2 * h + 1, 2 * h + 2
            sl, sr = c.rank(l), c.rank(r)
            blk = np.zeros((sl + sr, int(c.node_size[h])))
            nl = int(c.node_size[l])
            blk[:sl, :nl] = ph[l]
            blk[sl:, nl:] = ph[r]
            ph[h] = c.proj[h] @ blk
    return ph


def assemble(c: Compression, K) -> np.ndarray:
    """Dense K~ in the original ordering."""
    fl = first_leaf(c.depth)
    ph = telescoped(c)
    Kp = np.zeros((c.n, c.n))
    for b in range(1 << c.depth):
        h = fl + b
        rb = slice(int(c.node_start[h]), int(c.node_start[h] + c.node_size[h]))
        for a in c.near[b]:
            a = int(a)
            ra = slice(int(c.node_start[a]), int(c.node_start[a] + c.node_size[a]))
            Kp[rb, ra] += K(c.indices(h), c.indices(a))
    for h in range(1, c.nn):
        rb = slice(int(c.node_start[h]), int(c.node_start[h] + c.node_size[h]))
        for a in c.far[h]:
            a = int(a)
            ra = slice(int(c.node_start[a]), int(c.node_start[a] + c.node_size[a]))
            Kp[rb, ra] += ph[h].T @ K(c.skel[h], c.skel[a]) @ ph[a]
    out = np.empty_like(Kp)
    out[np.ix_(c.perm, c.perm)] = Kp
    return out


def algorithmic_flops(c: Compression, r: int) -> float:
    """Flops of one K~W from the built compression (Table 2, with the internal
    N2S/S2N counted as 2 s_a (s_l + s_r) r since P is s_a x (s_l + s_r))."""
    fl = first_leaf(c.depth)
    f = 0.0
    for h in range(1, c.nn):
        s = c.rank(h)
        if h >= fl:
            f += 2 * 2.0 * s * int(c.node_size[h]) * r       # N2S + S2N
        else:
            f += 2 * 2.0 * s * (c.rank(2 * h + 1) + c.rank(2 * h + 2)) * r
        for a in c.far[h]:
            f += 2.0 * s * c.rank(int(a)) * r
    for b in range(1 << c.depth):
        h = fl + b
        for a in c.near[b]:
            f += 2.0 * int(c.node_size[h]) * int(c.node_size[int(a)]) * r
    return f
