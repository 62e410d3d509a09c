"""GPU K~W against the oracle's storage-form evaluation (oracle/stored.py):
the same compression, every product's operands rounded the way the storage
form defines them (BF16 round to nearest even, or the hi + lo split), sums in
FP64.  This separates the error a storage form introduces from the error of
the kernels that use it.

* Integer grid compressions (tests/grid_cases.py): ranks and leaf sizes on
  the kernel's row, slab and column edges (1, 31-33, 63-65, 127-129,
  255-257, 511-513), integer P, K and W.  Every sum either side forms is an
  exact integer, so the device must equal the oracle to the last bit in every
  storage form (FP32, BF16, split BF16, and BF16 far with FP32 near), under
  every tile shape, at a vector-aligned and a ragged column count.
* Kernel compressions: split BF16 and FP32 within 1e-5 Frobenius and
  1e-5 x max|U| per element of the stored-form walk (the device's FP32 sums
  against FP64); plain BF16 within the per-element allowance of
  `stored.bf16_allowance` (an intermediate whose FP32 and FP64 values straddle
  a BF16 rounding midpoint may round to either neighbour) and 1e-3 Frobenius.
"""
import os
import tempfile

import numpy as np
import pytest

import grid_cases
import workloads
from gpu_util import cuda_rhs, export_read, log, rel_err
from oracle import cfile, kernels, stored

pytestmark = pytest.mark.gpu

FORMS = {  # name: (storage, near storage) of the library and of the oracle
    "fp32": ("FP32", "FP32", "fp32", "fp32"),
    "bf16": ("BF16", "BF16", "bf16", "bf16"),
    "bf16x3": ("BF16X3", "BF16X3", "bf16x3", "bf16x3"),
    "bf16_far_fp32_near": ("BF16", "FP32", "bf16", "fp32"),
}
N_TILE_SHAPES = 11


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "no GPU"
    import paper_1707_00164_amd as g
    g.lib()
    return t


def _load(g, c, A, form):
    """The grid compression imported by the library, sampling A."""
    sp, sn = getattr(g, FORMS[form][0]), getattr(g, FORMS[form][1])
    S = g.PySampler(lambda I, J: A[np.ix_(I, J)], c.n)
    fd, path = tempfile.mkstemp(suffix=".gofmm")
    os.close(fd)
    try:
        cfile.write(c, path)
        return g.Compression.load(path, S, storage=sp, near_storage=sn, threads=1)
    finally:
        os.unlink(path)


@pytest.mark.parametrize("form", sorted(FORMS))
@pytest.mark.parametrize("case", sorted(grid_cases.CASES))
def test_grid_edges_bit_exact(torch, case, form, monkeypatch):
    import paper_1707_00164_amd as g
    c, A = grid_cases.build(*grid_cases.CASES[case], seed=1)
    K = kernels.DenseMatrix(A)
    comp = _load(g, c, A, form)
    st = comp.stats()
    log(f"case grid {case} form {form}: n={c.n}, rank max {st.rank_max}, launches {len(comp.launches())}")
    for r in (37, 64):
        W64 = grid_cases.integer_rhs(c.n, r, 3 + r)
        want = stored.tree_walk_stored(c, K, W64, FORMS[form][2], FORMS[form][3])
        assert np.array_equal(want, np.rint(want)) and np.abs(want).max() < 2.0 ** 24
        W = torch.from_numpy(W64.astype(np.float32)).cuda()
        for t in [None] + list(range(N_TILE_SHAPES)):
            if t is None:
                monkeypatch.delenv("GOFMM_TILE", raising=False)
            else:
                monkeypatch.setenv("GOFMM_TILE", str(t))
            log(f"  r={r} tile {'model' if t is None else t}")
            U = comp.evaluate(W)
            torch.cuda.synchronize()
            got = U.cpu().numpy().astype(np.float64)
            bad = np.argwhere(got != want)
            assert bad.size == 0, (r, t, bad[:5].tolist(), got[tuple(bad[0])], want[tuple(bad[0])])
    monkeypatch.delenv("GOFMM_TILE", raising=False)
    comp.free()


def _kernel_case(g, prec, near_prec):
    rng = np.random.default_rng(4)
    n = 3001
    pts = rng.random((n, 3))
    S = g.KernelSampler(pts, "gaussian", 0.3, 1e-3)
    comp = g.Compression.compress(S, leaf_size=100, max_rank=64, tol=1e-6, kappa=16, budget=0.1, seed=5,
                                  storage=prec, near_storage=near_prec)
    return comp, kernels.KernelMatrix(pts, "gaussian", 0.3, 1e-3), n


@pytest.mark.parametrize("form", ["fp32", "bf16x3"])
def test_kernel_case_elementwise(torch, form):
    import paper_1707_00164_amd as g
    sp, sn, osp, osn = FORMS[form]
    comp, K, n = _kernel_case(g, getattr(g, sp), getattr(g, sn))
    log(f"case ragged fmm n={n} form {form} vs stored-form oracle")
    _, Wd = cuda_rhs(n, 45, 77)
    U = comp.evaluate(Wd)
    torch.cuda.synchronize()
    W32 = Wd.cpu().numpy().astype(np.float64)
    want = stored.tree_walk_stored(export_read(comp), K, W32, osp, osn)
    got = U.cpu().numpy().astype(np.float64)
    e = rel_err(got, want)
    emax = float(np.max(np.abs(got - want)) / np.max(np.abs(want)))
    log(f"  rel_F={e:.3e} max_elem_rel={emax:.3e}")
    assert e <= 1e-5 and emax <= 1e-5


@pytest.mark.parametrize("form", ["bf16", "bf16_far_fp32_near"])
def test_kernel_case_bf16_within_allowance(torch, form):
    import paper_1707_00164_amd as g
    sp, sn, osp, osn = FORMS[form]
    comp, K, n = _kernel_case(g, getattr(g, sp), getattr(g, sn))
    log(f"case ragged fmm n={n} form {form} vs stored-form oracle")
    _, Wd = cuda_rhs(n, 45, 78)
    U = comp.evaluate(Wd)
    torch.cuda.synchronize()
    W32 = Wd.cpu().numpy().astype(np.float64)
    c = export_read(comp)
    want = stored.tree_walk_stored(c, K, W32, osp, osn)
    allow = stored.bf16_allowance(c, K, W32, near_storage=osn)
    got = U.cpu().numpy().astype(np.float64)
    diff = np.abs(got - want)
    e = rel_err(got, want)
    log(f"  rel_F={e:.3e}, max diff / allowance {float(np.max(diff / np.maximum(allow, 1e-300))):.3f}, "
        f"max allowance / max|U| {float(allow.max() / np.abs(want).max()):.2e}")
    assert np.all(diff <= allow)
    assert e <= 1e-3
