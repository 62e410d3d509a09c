"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module only draws numbers: point clouds, right-hand sides, sampled row
sets and the parameter sets of the synthetic workloads.  It contains none of
the method's arithmetic (no distances, trees, skeletons or products), so both
the FP64 oracle and the HIP library can consume the same inputs without
sharing any computation.

The paper's own matrices (K02-K18, G01-G05, COVTYPE, HIGGS, MNIST; Sec. 3,
"Matrices") are not available, so these radial-kernel point clouds stand in
for them.  The kernel of each workload is named here (kind, bandwidth,
diagonal shift) but evaluated separately by each side: the oracle in NumPy,
the library in C.

Kernel kinds (all SPD; the shift adds a strict margin):
  gaussian      K_ij = exp(-|x_i - x_j|^2 / (2 h^2)) + shift * [i == j]
  imq           K_ij = 1 / sqrt(1 + |x_i - x_j|^2 / h^2) + shift * [i == j]
  laplace_like  K_ij = 1 / (|x_i - x_j| + 0.05) + shift * [i == j]
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 1707_00164

KERNEL_IDS = {"gaussian": 0, "imq": 1, "laplace_like": 2}


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    dim: int
    kernel: str            # one of KERNEL_IDS
    h: float               # bandwidth (unused by laplace_like)
    shift: float           # diagonal shift
    leaf_size: int         # m
    max_rank: int          # s
    tol: float             # tau
    kappa: int
    budget: float
    r: int
    points_kind: str       # "uniform" | "clusters"
    seed: int
    n_clusters: int = 8
    cluster_sigma: float = 0.1


def _cfg_seed(cfg_index: int, instance: int = 0) -> int:
    return SEED_BASE + 1000 * cfg_index + instance


def small_gaussian() -> Workload:
    """N=4096 Gaussian kernel (h=0.5, shift 1e-3) on 3-D uniform points, HSS."""
    return Workload("gauss3d_n4096_hss", 4096, 3, "gaussian", 0.5, 1e-3,
                    128, 128, 1e-5, 32, 0.0, 16, "uniform", _cfg_seed(1))


def clustered_gaussian() -> Workload:
    """N=65536 Gaussian (h=0.8, shift 1e-2) on 8 Gaussian clusters in 6-D."""
    return Workload("gauss6d_n65536_fmm3", 65536, 6, "gaussian", 0.8, 1e-2,
                    256, 256, 1e-5, 32, 0.03, 512, "clusters", _cfg_seed(2))


def large_imq(r: int = 2048) -> Workload:
    """N=262144 inverse multiquadric (h=0.3, shift 1e-2) on 4-D uniform points."""
    return Workload("imq4d_n262144_fmm3", 262144, 4, "imq", 0.3, 1e-2,
                    512, 512, 1e-6, 32, 0.03, r, "uniform", _cfg_seed(3))


def batched_instances(count: int = 48) -> List[Workload]:
    """Instances of uneven N, log-uniform in [8192, 131072], d in 3..8.

    Each is a Gaussian (h=0.8) or a 1/(|x-y|+0.05) kernel with shift 1e-2;
    m=256, s=256, tau=1e-5, kappa=32, budget 3%; r drawn from {32,64,128,256}.
    """
    rng = np.random.default_rng(_cfg_seed(4))
    out = []
    for k in range(count):
        n = int(math.floor(math.exp(rng.uniform(math.log(8192), math.log(131072)))))
        d = int(rng.integers(3, 9))
        kind = "gaussian" if rng.random() < 0.5 else "laplace_like"
        r = int(rng.choice([32, 64, 128, 256]))
        out.append(Workload(f"batch{k:02d}_{kind}_{d}d_n{n}", n, d, kind, 0.8, 1e-2,
                            256, 256, 1e-5, 32, 0.03, r, "uniform", _cfg_seed(4, k + 1)))
    return out


def _serving_budget(n: int, m: int) -> float:
    """3%, or enough for 4 other near leaves per leaf where that is more."""
    return max(0.03, 4.5 * m / n)


def serving_instances(count: int = 16, n_lo: int = 16384, n_hi: int = 262144) -> List[Workload]:
    """Resident compressions for the serving loop: N log-spaced in [n_lo, n_hi],
    kernels cycling through the three families above; leaf size and maximum
    rank are the family's, at least 256 (512 from N = 131072 up); near budget
    3%, raised for small trees so that a leaf may take at least 4 other near
    leaves (cap = floor(budget N / m))."""
    ns = np.unique(np.round(np.geomspace(n_lo, n_hi, count)).astype(np.int64))
    fams = [small_gaussian(), clustered_gaussian(), large_imq()]
    out = []
    for k, n in enumerate(ns):
        f = fams[k % 3]
        m = max(f.leaf_size, 256 if n < 131072 else 512)
        out.append(dataclasses.replace(
            f, name=f"serve{k:02d}_{f.kernel}_n{n}", n=int(n), leaf_size=m, max_rank=m,
            budget=_serving_budget(int(n), m), seed=_cfg_seed(5, k + 1)))
    return out


def serving_admissions(count: int = 4, n_lo: int = 16384, n_hi: int = 65536) -> List[Workload]:
    """Fresh compressions admitted while the serving loop runs: N log-spaced
    in [n_lo, n_hi], kernels cycling through the three families (leaf size
    and maximum rank the family's, at least 256; budget as for the resident
    set), seeds disjoint from the resident ones."""
    ns = np.round(np.geomspace(n_lo, n_hi, count)).astype(np.int64)
    fams = [small_gaussian(), clustered_gaussian(), large_imq()]
    out = []
    for k, n in enumerate(ns):
        f = fams[(k + 1) % 3]
        m = max(f.leaf_size, 256)
        out.append(dataclasses.replace(
            f, name=f"admit{k:02d}_{f.kernel}_n{n}", n=int(n), leaf_size=m, max_rank=m,
            budget=_serving_budget(int(n), m), seed=_cfg_seed(5, 100 + k)))
    return out


def points(w: Workload) -> np.ndarray:
    """(n, dim) FP64 points from the workload's seed, randomly permuted.

    uniform:  U[0,1]^d.
    clusters: n_clusters centres ~ U[0,1]^d, equal weights,
              x = centre + sigma * N(0, I), no clipping.
    """
    rng = np.random.default_rng(w.seed)
    if w.points_kind == "uniform":
        x = rng.random((w.n, w.dim))
    elif w.points_kind == "clusters":
        centres = rng.random((w.n_clusters, w.dim))
        lab = rng.integers(0, w.n_clusters, size=w.n)
        x = centres[lab] + w.cluster_sigma * rng.standard_normal((w.n, w.dim))
    else:
        raise ValueError(w.points_kind)
    x = x[rng.permutation(w.n)]
    return np.ascontiguousarray(x, dtype=np.float64)


def rhs(n: int, r: int, seed: int, dtype=np.float64) -> np.ndarray:
    """(n, r) standard normal right-hand sides, row-major."""
    rng = np.random.default_rng(seed + 77)
    return np.ascontiguousarray(rng.standard_normal((n, r)).astype(dtype))


def sample_rows(n: int, count: int, seed: int) -> np.ndarray:
    """Sorted set of `count` distinct row indices used for sampled error checks."""
    rng = np.random.default_rng(seed + 991)
    return np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int64)


def random_spd(n: int, seed: int, decay: Optional[float] = None) -> np.ndarray:
    """Dense SPD matrix A A^T / n + I with a Gaussian A (used by small pins).

    With `decay`, column j of A is scaled by decay**j, giving a matrix whose
    off-diagonal blocks have quickly decaying singular values.
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    if decay is not None:
        a = a * (decay ** np.arange(n))[None, :]
    return a @ a.T / n + np.eye(n)
