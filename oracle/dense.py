"""Exact reference products and the error metric (oracle side).

  kw(K, W, rows)   U* = K W in FP64, for all rows or a sampled row set.
  eps2(Ut, Ue)     the relative error of Sec. 3: |K~W - KW|_F / |KW|_F,
                   evaluated over the rows supplied (the paper samples 100).

Parity: kw is the textbook definition, pinned by `math.fsum` recomputation of
single entries and by the sampled-row result agreeing with the full product.
"""
from __future__ import annotations

import numpy as np


def kw(K, W: np.ndarray, rows=None, block: int = 2048) -> np.ndarray:
    """Rows `rows` (default all) of K @ W in FP64, built from K(I, J) blocks."""
    n = W.shape[0]
    W = np.asarray(W, dtype=np.float64)
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    out = np.zeros((len(rows), W.shape[1]))
    allj = np.arange(n)
    for a in range(0, len(rows), block):
        I = rows[a:a + block]
        for b in range(0, n, 8192):
            J = allj[b:b + 8192]
            out[a:a + block] += K(I, J) @ W[J]
    return out


def eps2(approx: np.ndarray, exact: np.ndarray) -> float:
    """|approx - exact|_F / |exact|_F (Sec. 3, epsilon_2)."""
    approx = np.asarray(approx, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))
