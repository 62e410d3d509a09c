"""In-memory compression record and its file format (oracle side).

A compression is everything that defines K~ except the cached kernel blocks,
which are K(I, J) entries re-sampled from the kernel by whoever evaluates:

  params       n, leaf size m, max rank s, tolerance tau, kappa, budget,
               distance id (0 Gram-l2, 1 Gram angle), depth D
  perm         perm[k] = original index at permuted position k (leaf order)
  node_start,  for every heap node h (root 0, children 2h+1, 2h+2) the range
  node_size    of its indices in permuted order
  split_p/q    the metricSplit poles of each internal node (-1 for leaves)
  centroid     the centroid sample of each internal node
  knn          kappa nearest neighbours of each original index
  near         Near(beta) for every leaf, as heap ids of leaves
  far          Far(alpha) for every node, as heap ids
  skel         skeleton indices (original numbering) of every non-root node
  samp         the sampled row set I' used by the node's ID
  proj         P of every non-root node: s x |alpha| for a leaf (columns in
               permuted order), s x (s_l + s_r) for an internal node (columns
               are the left skeletons followed by the right skeletons)

File layout (little-endian): 8-byte magic b"GOFMMC1\\0", int64 array count,
then per array a 24-byte zero-padded name, int32 dtype code (1 int32, 2 int64,
3 float64), int32 ndim, two int64 dims, and the raw data.  Ragged lists are
stored as a `<name>_ptr` (length count+1) / `<name>_val` pair.

Parity: the reader and writer round-trip each other (tested); the library
implements the same layout independently in C++.
"""
from __future__ import annotations

import dataclasses
import struct
from typing import Dict, List, Optional

import numpy as np

MAGIC = b"GOFMMC1\0"
_DT = {1: np.int32, 2: np.int64, 3: np.float64}
_DT_INV = {np.dtype(np.int32): 1, np.dtype(np.int64): 2, np.dtype(np.float64): 3}


def n_nodes(depth: int) -> int:
    return (1 << (depth + 1)) - 1


def first_leaf(depth: int) -> int:
    return (1 << depth) - 1


def level_of(h: int) -> int:
    return (h + 1).bit_length() - 1


@dataclasses.dataclass
class Compression:
    n: int
    depth: int
    leaf_size: int
    max_rank: int
    tol: float
    kappa: int
    budget: float
    distance: int
    perm: np.ndarray
    node_start: np.ndarray
    node_size: np.ndarray
    split_p: np.ndarray
    split_q: np.ndarray
    centroid: List[np.ndarray]
    knn: Optional[np.ndarray]
    near: List[np.ndarray]        # indexed by leaf number 0..L-1
    far: List[np.ndarray]         # indexed by heap id
    skel: List[np.ndarray]        # indexed by heap id (root: empty)
    samp: List[np.ndarray]
    proj: List[Optional[np.ndarray]]

    @property
    def nn(self) -> int:
        return n_nodes(self.depth)

    @property
    def n_leaves(self) -> int:
        return 1 << self.depth

    def is_leaf(self, h: int) -> bool:
        return h >= first_leaf(self.depth)

    def indices(self, h: int) -> np.ndarray:
        """Original indices of node h, in permuted order."""
        a = int(self.node_start[h])
        return self.perm[a:a + int(self.node_size[h])]

    def rank(self, h: int) -> int:
        return len(self.skel[h])


def _put(buf: list, name: str, arr: np.ndarray):
    arr = np.ascontiguousarray(arr)
    if arr.dtype not in _DT_INV:
        raise TypeError(arr.dtype)
    if arr.ndim == 1:
        shape = (arr.shape[0], 1)
    elif arr.ndim == 2:
        shape = arr.shape
    else:
        raise ValueError("ndim")
    nm = name.encode()
    assert len(nm) < 24
    buf.append(nm + b"\0" * (24 - len(nm)))
    buf.append(struct.pack("<iiqq", _DT_INV[arr.dtype], arr.ndim, shape[0], shape[1]))
    buf.append(arr.tobytes())


def _ragged(lists, dtype) -> (np.ndarray, np.ndarray):
    ptr = np.zeros(len(lists) + 1, dtype=np.int64)
    for i, x in enumerate(lists):
        ptr[i + 1] = ptr[i] + (0 if x is None else np.asarray(x).size)
    val = np.concatenate([np.asarray(x, dtype=dtype).reshape(-1) for x in lists if x is not None]
                         + [np.zeros(0, dtype=dtype)])
    return ptr, val


def write(c: Compression, path: str):
    arrays = []
    params = np.array([c.n, c.leaf_size, c.max_rank, c.tol, c.kappa, c.budget,
                       c.distance, c.depth], dtype=np.float64)
    arrays.append(("params", params))
    arrays.append(("perm", np.asarray(c.perm, dtype=np.int64)))
    arrays.append(("node_start", np.asarray(c.node_start, dtype=np.int64)))
    arrays.append(("node_size", np.asarray(c.node_size, dtype=np.int64)))
    arrays.append(("split_p", np.asarray(c.split_p, dtype=np.int64)))
    arrays.append(("split_q", np.asarray(c.split_q, dtype=np.int64)))
    for nm, lst in (("centroid", c.centroid), ("near", c.near), ("far", c.far),
                    ("skel", c.skel), ("samp", c.samp)):
        p, v = _ragged(lst, np.int64)
        arrays.append((nm + "_ptr", p))
        arrays.append((nm + "_val", v))
    if c.knn is not None:
        arrays.append(("knn", np.asarray(c.knn, dtype=np.int64)))
    p, v = _ragged(c.proj, np.float64)
    arrays.append(("proj_ptr", p))
    arrays.append(("proj_val", v))
    buf = [MAGIC, struct.pack("<q", len(arrays))]
    for nm, a in arrays:
        _put(buf, nm, a)
    with open(path, "wb") as f:
        for b in buf:
            f.write(b)


def read_arrays(path: str) -> Dict[str, np.ndarray]:
    out = {}
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError("not a compression file")
        (cnt,) = struct.unpack("<q", f.read(8))
        for _ in range(cnt):
            name = f.read(24).split(b"\0", 1)[0].decode()
            dt, nd, d0, d1 = struct.unpack("<iiqq", f.read(24))
            dtype = np.dtype(_DT[dt])
            a = np.frombuffer(f.read(dtype.itemsize * d0 * d1), dtype=dtype)
            out[name] = a.reshape(d0, d1) if nd == 2 else a.reshape(d0)
    return out


def _split(ptr, val):
    return [val[ptr[i]:ptr[i + 1]].copy() for i in range(len(ptr) - 1)]


def read(path: str) -> Compression:
    a = read_arrays(path)
    p = a["params"]
    n, depth = int(p[0]), int(p[7])
    skel = _split(a["skel_ptr"], a["skel_val"])
    projflat = _split(a["proj_ptr"], a["proj_val"])
    node_size = a["node_size"].copy()
    proj: List[Optional[np.ndarray]] = []
    for h in range(n_nodes(depth)):
        s = len(skel[h])
        if h == 0 or s == 0:
            proj.append(None)
            continue
        if h >= first_leaf(depth):
            cols = int(node_size[h])
        else:
            cols = len(skel[2 * h + 1]) + len(skel[2 * h + 2])
        proj.append(projflat[h].reshape(s, cols))
    return Compression(
        n=n, depth=depth, leaf_size=int(p[1]), max_rank=int(p[2]), tol=float(p[3]),
        kappa=int(p[4]), budget=float(p[5]), distance=int(p[6]),
        perm=a["perm"].copy(), node_start=a["node_start"].copy(), node_size=node_size,
        split_p=a["split_p"].copy(), split_q=a["split_q"].copy(),
        centroid=_split(a["centroid_ptr"], a["centroid_val"]),
        knn=a["knn"].copy() if "knn" in a else None,
        near=_split(a["near_ptr"], a["near_val"]),
        far=_split(a["far_ptr"], a["far_val"]),
        skel=skel, samp=_split(a["samp_ptr"], a["samp_val"]), proj=proj)
