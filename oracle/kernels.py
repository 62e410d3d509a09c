"""FP64 entries K(I, J) of the synthetic SPD kernels (oracle side).

The method's only input is a routine returning K_IJ for index sets I, J
(Sec. 1, problem statement).  This module is that routine for the synthetic
point clouds of `workloads`, evaluated directly in FP64 NumPy:

  gaussian      exp(-|x_i - x_j|^2 / (2 h^2))
  imq           1 / sqrt(1 + |x_i - x_j|^2 / h^2)
  laplace_like  1 / (|x_i - x_j| + 0.05)

plus shift * [i == j] on the original indices.  Squared distances are summed
coordinate by coordinate as (x_i - x_j)^2, which is exactly symmetric in i, j.

Parity: pinned by tests that recompute single entries with `math` scalar
functions (pure Python) and check symmetry and positive definiteness.
"""
from __future__ import annotations

import numpy as np


class KernelMatrix:
    """Callable K(I, J) -> (|I|, |J|) FP64 block over a hidden point cloud."""

    def __init__(self, pts: np.ndarray, kind: str, h: float, shift: float):
        self.x = np.ascontiguousarray(pts, dtype=np.float64)
        self.n = self.x.shape[0]
        self.kind = kind
        self.h = float(h)
        self.shift = float(shift)

    def _sq(self, I, J):
        xi = self.x[I]
        xj = self.x[J]
        d2 = np.zeros((len(I), len(J)))
        for c in range(self.x.shape[1]):
            diff = xi[:, c][:, None] - xj[:, c][None, :]
            d2 += diff * diff
        return d2

    def __call__(self, I, J) -> np.ndarray:
        I = np.asarray(I, dtype=np.int64).reshape(-1)
        J = np.asarray(J, dtype=np.int64).reshape(-1)
        out = np.empty((len(I), len(J)))
        step = max(1, (1 << 22) // max(1, len(J)))
        for a in range(0, len(I), step):
            Ia = I[a:a + step]
            d2 = self._sq(Ia, J)
            if self.kind == "gaussian":
                k = np.exp(-d2 / (2.0 * self.h * self.h))
            elif self.kind == "imq":
                k = 1.0 / np.sqrt(1.0 + d2 / (self.h * self.h))
            elif self.kind == "laplace_like":
                k = 1.0 / (np.sqrt(d2) + 0.05)
            else:
                raise ValueError(self.kind)
            if self.shift != 0.0:
                k = k + self.shift * (Ia[:, None] == J[None, :])
            out[a:a + step] = k
        return out

    def diag(self) -> np.ndarray:
        i = np.arange(self.n)
        base = {"gaussian": 1.0, "imq": 1.0, "laplace_like": 1.0 / 0.05}[self.kind]
        return np.full(self.n, base) + self.shift * np.ones_like(i, dtype=np.float64)


class DenseMatrix:
    """Callable K(I, J) over an explicit dense SPD matrix (small pins)."""

    def __init__(self, a: np.ndarray):
        self.a = np.asarray(a, dtype=np.float64)
        self.n = self.a.shape[0]

    def __call__(self, I, J) -> np.ndarray:
        I = np.asarray(I, dtype=np.int64).reshape(-1)
        J = np.asarray(J, dtype=np.int64).reshape(-1)
        return self.a[np.ix_(I, J)]

    def diag(self) -> np.ndarray:
        return np.diag(self.a).copy()


def for_workload(w, pts=None) -> KernelMatrix:
    import workloads
    if pts is None:
        pts = workloads.points(w)
    return KernelMatrix(pts, w.kernel, w.h, w.shift)
