"""K~ W with the operators as a device stores them (oracle side, test
infrastructure).

The paper computes in single or double precision (Sec. 3); the library adds
BF16 storage forms.  To separate the error of a storage form from the error
of the kernels that use it, this module evaluates the same compression as
`evaluate.tree_walk` (Alg. Evaluate: N2S, S2S, S2N, L2L), with every product's
operands rounded the way the form defines them and every sum taken in FP64:

  fp32     A rounded to FP32 (RNE); right-hand operands as they are.
  bf16     A rounded to BF16 (RNE from the FP64 value); each right-hand operand
           (W, w~, u~) rounded to BF16 (RNE) before its product.
  bf16x3   split operands x = hi + lo with hi = bf16(x), lo = bf16(x - hi),
           for A (from the FP64 value) and for every right-hand operand; a
           product is a_hi b_hi + a_hi b_lo + a_lo b_hi (the lo*lo term is
           not formed).

A is P (N2S, S2N at every level), a coupling block K(b~, a~) (S2S) or a near
block K(b, a) (L2L).  P and coupling blocks use the `storage` form, near
blocks the `near_storage` form.  The intermediate w~ and u~ are carried in
FP64 between the steps by default; only the operand of each product is
rounded.  With carry="fp32" every intermediate is rounded to FP32 where a
device keeps it in an FP32 workspace: w~ of a node once formed, u~ of a node
once its far-field sum is formed, and again after each parent's S2N
contribution is added (the sums themselves stay in FP64).  Plain BF16 needs
this reading to be compared element by element: its BF16 rounding of an
intermediate amplifies any difference in the value rounded, and FP64 against
FP32 intermediates differ enough to flip many roundings up a deep tree.

BF16 here is the IEEE-style binary format with 8 significant bits and the
exponent range of FP32 (subnormals included), rounded to nearest with ties to
even; `bf16` writes that definition out with frexp/rint.

Parity: bf16 is pinned against hand-worked values, ties, the binade edges
and PyTorch's own float32 -> bfloat16 conversion; split against its error
bound (|x - hi - lo| <= 2^-17 |x|) and exactness on 16-bit integers;
tree_walk_stored against the exact tree walk where every operand is exactly
representable (it must then agree to the last bit in every form) and against
dense products for a single leaf.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from .cfile import Compression, first_leaf

FP32, BF16, BF16X3 = "fp32", "bf16", "bf16x3"


def bf16(x) -> np.ndarray:
    """Nearest BF16 value of each entry (ties to even), as FP64."""
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)                            # x = f 2^e with 1/2 <= |f| < 1
    q = np.ldexp(1.0, np.maximum(e, -125) - 8)    # BF16 spacing at x (2^-133 below 2^-126)
    with np.errstate(over="ignore", invalid="ignore"):
        y = np.rint(x / q) * q                    # rint rounds ties to even
        y = np.where(np.abs(y) >= 2.0 ** 128, np.copysign(np.inf, x), y)
    return np.where(np.isfinite(x), y, x)


def split(x):
    """(hi, lo) with hi = bf16(x) and lo = bf16(x - hi)."""
    x = np.asarray(x, dtype=np.float64)
    hi = bf16(x)
    return hi, bf16(x - hi)


def fp32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def product(A: np.ndarray, B: np.ndarray, form: str) -> np.ndarray:
    """A @ B with both operands in the given storage form, summed in FP64."""
    if form == FP32:
        return fp32(A) @ np.asarray(B, dtype=np.float64)
    if form == BF16:
        return bf16(A) @ bf16(B)
    if form == BF16X3:
        ah, al = split(A)
        bh, bl = split(B)
        return ah @ bh + ah @ bl + al @ bh
    raise ValueError(form)


def _wanted(c: Compression, rows):
    """Leaves holding the rows and the nodes on their paths to the root (all
    of them when rows is None)."""
    fl = first_leaf(c.depth)
    if rows is None:
        want_leaf = np.ones(1 << c.depth, dtype=bool)
    else:
        pos_of = np.empty(c.n, dtype=np.int64)
        pos_of[c.perm] = np.arange(c.n)
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
    return want_leaf, want


def tree_walk_stored(c: Compression, K, W: np.ndarray, storage: str, near_storage: Optional[str] = None,
                     rows: Optional[np.ndarray] = None, carry: str = "fp64") -> np.ndarray:
    """Rows `rows` (default all) of K~ W, each product in its storage form;
    intermediates carried in FP64 or, with carry="fp32", rounded to FP32."""
    near_storage = storage if near_storage is None else near_storage
    if carry not in ("fp64", "fp32"):
        raise ValueError(carry)
    keep = fp32 if carry == "fp32" else (lambda x: x)
    W = np.asarray(W, dtype=np.float64)
    r = W.shape[1]
    fl = first_leaf(c.depth)
    Wp = W[c.perm]
    # N2S (POST)
    wt: List[Optional[np.ndarray]] = [None] * c.nn
    for h in range(c.nn - 1, 0, -1):
        if h >= fl:
            a = int(c.node_start[h])
            wt[h] = keep(product(c.proj[h], Wp[a:a + int(c.node_size[h])], storage))
        else:
            wt[h] = keep(product(c.proj[h], np.vstack([wt[2 * h + 1], wt[2 * h + 2]]), storage))
    want_leaf, want = _wanted(c, rows)
    # S2S
    ut: List[Optional[np.ndarray]] = [None] * c.nn
    for h in range(1, c.nn):
        acc = np.zeros((c.rank(h), r))
        if want[h]:
            for a in c.far[h]:
                a = int(a)
                acc += product(K(c.skel[h], c.skel[a]), wt[a], storage)
        ut[h] = keep(acc)
    # S2N (PRE: heap order visits a parent before its children)
    Up = np.zeros((c.n, r))
    for h in range(1, c.nn):
        if not want[h]:
            continue
        if h >= fl:
            a0 = int(c.node_start[h])
            Up[a0:a0 + int(c.node_size[h])] += product(c.proj[h].T, ut[h], storage)
        else:
            d = product(c.proj[h].T, ut[h], storage)
            sl = c.rank(2 * h + 1)
            ut[2 * h + 1] = keep(ut[2 * h + 1] + d[:sl])
            ut[2 * h + 2] = keep(ut[2 * h + 2] + d[sl:])
    # L2L
    for b in np.flatnonzero(want_leaf):
        h = fl + int(b)
        a0 = int(c.node_start[h])
        nb = int(c.node_size[h])
        ib = c.indices(h)
        for a in c.near[b]:
            a = int(a)
            s0 = int(c.node_start[a])
            Up[a0:a0 + nb] += product(K(ib, c.indices(a)), Wp[s0:s0 + int(c.node_size[a])], near_storage)
    U = np.empty_like(Up)
    U[c.perm] = Up
    return U if rows is None else U[np.asarray(rows)]


def _round_dev(x: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Largest distance from bf16(x) of bf16(y) for any y in [x - d, x + d]
    (rounding is monotone, so the interval's ends give it)."""
    b = bf16(x)
    return np.maximum(np.abs(bf16(x + d) - b), np.abs(bf16(x - d) - b))


def bf16_allowance(c: Compression, K, W: np.ndarray, near_storage: Optional[str] = None,
                   acc: float = 2.0 ** -20, rows: Optional[np.ndarray] = None) -> np.ndarray:
    """Per-element allowance |U_device - U_oracle| for plain BF16 storage.

    The device forms each intermediate (w~, u~) in FP32 and rounds it to BF16
    as the next product's operand; the oracle rounds its FP64 value.  Model
    the FP32 value as lying within acc * S of the FP64 one, S being the sum of
    |a||b| that formed it (acc = 2^-20 is 16 FP32 units, well above the
    accumulation error of these sums).  Where that interval, widened by what
    earlier roundings may already have moved x, holds a BF16 rounding
    midpoint, the two sides may round to neighbouring values: the operand
    then carries the distance between them.  Those distances travel to U
    through |A| of every later product (rounded as stored); the result is
    that propagated radius plus acc * S of U itself, for the rows `rows`
    (default all)."""
    near_storage = BF16 if near_storage is None else near_storage
    W = np.asarray(W, dtype=np.float64)
    r = W.shape[1]
    fl = first_leaf(c.depth)
    Wp = W[c.perm]
    want_leaf, want = _wanted(c, rows)

    def step(A, x, rho, s):
        """Value, radius and |a||b| sum of A @ bf16(x) for an intermediate x
        with radius rho and magnitude sum s."""
        Ar = np.abs(bf16(A))
        dev = _round_dev(x, rho + acc * s)
        return bf16(A) @ bf16(x), Ar @ dev, Ar @ np.abs(bf16(x))

    wt, wr, ws = [None] * c.nn, [None] * c.nn, [None] * c.nn
    for h in range(c.nn - 1, 0, -1):
        if h >= fl:
            a = int(c.node_start[h])
            B = Wp[a:a + int(c.node_size[h])]
            wt[h] = bf16(c.proj[h]) @ bf16(B)
            wr[h] = np.zeros_like(wt[h])
            ws[h] = np.abs(bf16(c.proj[h])) @ np.abs(bf16(B))
        else:
            l, rr = 2 * h + 1, 2 * h + 2
            wt[h], wr[h], ws[h] = step(c.proj[h], np.vstack([wt[l], wt[rr]]), np.vstack([wr[l], wr[rr]]),
                                       np.vstack([ws[l], ws[rr]]))
    ut, ur, us = [None] * c.nn, [None] * c.nn, [None] * c.nn
    for h in range(1, c.nn):
        ut[h] = np.zeros((c.rank(h), r))
        ur[h] = np.zeros((c.rank(h), r))
        us[h] = np.zeros((c.rank(h), r))
        if not want[h]:
            continue
        for a in c.far[h]:
            a = int(a)
            v, rho, s = step(K(c.skel[h], c.skel[a]), wt[a], wr[a], ws[a])
            ut[h] += v
            ur[h] += rho
            us[h] += s
    Ur = np.zeros((c.n, r))
    Us = np.zeros((c.n, r))
    for h in range(1, c.nn):
        if not want[h]:
            continue
        v, rho, s = step(c.proj[h].T, ut[h], ur[h], us[h])
        if h >= fl:
            a0 = int(c.node_start[h])
            Ur[a0:a0 + int(c.node_size[h])] += rho
            Us[a0:a0 + int(c.node_size[h])] += s
        else:
            sl = c.rank(2 * h + 1)
            for ch, sel in ((2 * h + 1, slice(0, sl)), (2 * h + 2, slice(sl, None))):
                ut[ch] = ut[ch] + v[sel]
                ur[ch] = ur[ch] + rho[sel]
                us[ch] = us[ch] + s[sel]
    for b in np.flatnonzero(want_leaf):
        h = fl + int(b)
        a0 = int(c.node_start[h])
        nb = int(c.node_size[h])
        for a in c.near[b]:
            a = int(a)
            s0 = int(c.node_start[a])
            Ab = K(c.indices(h), c.indices(a))
            B = Wp[s0:s0 + int(c.node_size[a])]
            if near_storage == BF16:
                Us[a0:a0 + nb] += np.abs(bf16(Ab)) @ np.abs(bf16(B))
            else:
                Us[a0:a0 + nb] += np.abs(Ab) @ np.abs(B)
    out = Ur + acc * Us
    U = np.empty_like(out)
    U[c.perm] = out
    return U if rows is None else U[np.asarray(rows)]
