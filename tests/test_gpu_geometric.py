"""Near blocks computed on the device from the points (gofmm_use_device_kernel)
against the FP64 oracle on the same compression.

The oracle evaluates every block from its own FP64 kernel code; the device
computes the near blocks in FP32 from FP32-rounded points (relative entry
error ~1e-7), so the same 1e-5 Frobenius / 1e-5 x max per-element bound as
the stored FP32 form applies.  The A values of a tile do not depend on the
tile shape and the k order per output element is fixed, so every tile shape
gives the same bits.
"""
import numpy as np
import pytest

import workloads
from gpu_util import cuda_rhs, export_read, log, rel_err
from oracle import dense, evaluate, kernels

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "no GPU"
    import paper_1707_00164_amd as g
    g.lib()
    return t


def _check(U_gpu, U_ref, tol=TOL, tol_elem=TOL, what=""):
    U_gpu = np.asarray(U_gpu, dtype=np.float64)
    e = rel_err(U_gpu, U_ref)
    emax = float(np.max(np.abs(U_gpu - U_ref)) / np.max(np.abs(U_ref)))
    log(f"  {what}: rel_F={e:.3e} max_elem_rel={emax:.3e}")
    assert np.all(np.isfinite(U_gpu))
    assert e <= tol and emax <= tol_elem, (e, emax)


def _compress(pts, kind, h, shift, storage=None, **kw):
    import paper_1707_00164_amd as g
    S = g.KernelSampler(pts, kind, h, shift)
    args = dict(leaf_size=100, max_rank=64, tol=1e-6, kappa=16, budget=0.1, seed=5)
    args.update(kw)
    if storage is not None:
        args.update(storage=storage, near_storage=storage)
    comp = g.Compression.compress(S, **args)
    return S, comp


@pytest.mark.parametrize("kind,h,shift,dim", [("gaussian", 0.3, 1e-3, 3), ("imq", 0.3, 1e-2, 4),
                                              ("laplace_like", 0.0, 1e-2, 8)])
@pytest.mark.parametrize("r", [45, 48])
def test_geometric_matches_oracle(torch, kind, h, shift, dim, r):
    """Ragged leaves (3001 points, leaves of 93/94), all three kernels, both
    row alignments (r = 45: scalar B loads, r = 48: 16-byte loads)."""
    rng = np.random.default_rng(21)
    n = 3001
    pts = rng.random((n, dim))
    S, comp = _compress(pts, kind, h, shift)
    stored_bytes = comp.stats().operator_bytes
    comp.use_device_kernel(S)
    names = [l[0] for l in comp.launches()]
    log(f"case geometric {kind} d={dim} r={r}: launches {names[-2:]}, operator "
        f"{stored_bytes} -> {comp.stats().operator_bytes} bytes")
    assert names[-2:] == ["s2n_leaf", "l2l"]
    assert comp.stats().operator_bytes < stored_bytes
    K = kernels.KernelMatrix(pts, kind, h, shift)
    W64, Wd = cuda_rhs(n, r, 3)
    U = comp.evaluate(Wd)
    torch.cuda.synchronize()
    ref = evaluate.tree_walk(export_read(comp), K, Wd.cpu().numpy().astype(np.float64))
    _check(U.cpu().numpy(), ref, what=f"{kind} r={r}")


def test_geometric_every_tile_shape_same_bits(torch, monkeypatch):
    rng = np.random.default_rng(4)
    n = 3001
    pts = rng.random((n, 3))
    S, comp = _compress(pts, "gaussian", 0.3, 1e-3)
    comp.use_device_kernel(S)
    K = kernels.KernelMatrix(pts, "gaussian", 0.3, 1e-3)
    W64, Wd = cuda_rhs(n, 45, 77)
    ref = evaluate.tree_walk(export_read(comp), K, Wd.cpu().numpy().astype(np.float64))
    outs = []
    for t in range(11):                            # every tile shape the library has
        monkeypatch.setenv("GOFMM_TILE", str(t))
        log(f"case geometric tile shape {t}")
        U = comp.evaluate(Wd)
        torch.cuda.synchronize()
        outs.append(U.cpu().numpy())
        _check(outs[-1], ref, what=f"tile {t}")
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_geometric_single_leaf_is_dense(torch):
    """N <= m: one leaf, no far field; K~ = K, and the L2L launch writes U
    without accumulating (nothing precedes it)."""
    rng = np.random.default_rng(8)
    n = 200
    pts = rng.random((n, 3))
    S, comp = _compress(pts, "gaussian", 0.5, 1e-3, leaf_size=256)
    comp.use_device_kernel(S)
    assert [l[0] for l in comp.launches()] == ["l2l"]
    K = kernels.KernelMatrix(pts, "gaussian", 0.5, 1e-3)
    W64, Wd = cuda_rhs(n, 7, 9)
    U = comp.evaluate(Wd)
    torch.cuda.synchronize()
    _check(U.cpu().numpy(), dense.kw(K, Wd.cpu().numpy().astype(np.float64)), what="single leaf")


def test_geometric_with_split_bf16_far_field(torch):
    """Split-BF16 P and coupling blocks with the near blocks from the points."""
    import paper_1707_00164_amd as g
    rng = np.random.default_rng(5)
    n = 4000
    pts = rng.random((n, 4))
    S, comp = _compress(pts, "imq", 0.3, 1e-2, storage=g.BF16X3)
    comp.use_device_kernel(S)
    K = kernels.KernelMatrix(pts, "imq", 0.3, 1e-2)
    W64, Wd = cuda_rhs(n, 64, 12)
    U = comp.evaluate(Wd)
    torch.cuda.synchronize()
    ref = evaluate.tree_walk(export_read(comp), K, Wd.cpu().numpy().astype(np.float64))
    _check(U.cpu().numpy(), ref, tol=3e-5, tol_elem=1e-4, what="split-BF16 far field")


def test_geometric_clustered_gaussian_full_size(torch):
    """The N=65536 clustered Gaussian at r=512, autotuned, 128 sampled rows
    against the oracle, and the error against the exact K W stated."""
    import paper_1707_00164_amd as g
    w = workloads.clustered_gaussian()
    log(f"case geometric {w.name} r={w.r}")
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    comp = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol, kappa=w.kappa,
                                  budget=w.budget, seed=w.seed)
    comp.use_device_kernel(S)
    W64, Wd = cuda_rhs(w.n, w.r, w.seed)
    U = comp.autotune(Wd)
    comp.evaluate(Wd, U)
    torch.cuda.synchronize()
    K = kernels.KernelMatrix(pts, w.kernel, w.h, w.shift)
    rows = workloads.sample_rows(w.n, 128, w.seed + 5)
    Wc = Wd.cpu().numpy().astype(np.float64)
    ref = evaluate.tree_walk(export_read(comp), K, Wc, rows)
    got = U.cpu().numpy()[rows]
    e = rel_err(got, ref)
    eps = rel_err(got, dense.kw(K, Wc, rows))
    log(f"  vs oracle {e:.2e}, eps2 vs exact {eps:.2e}")
    assert e <= TOL and eps <= 1e-4


def test_geometric_not_batched_or_served(torch):
    import paper_1707_00164_amd as g
    rng = np.random.default_rng(2)
    pts = rng.random((1500, 3))
    S, comp = _compress(pts, "gaussian", 0.3, 1e-3)
    comp.use_device_kernel(S)
    W64, Wd = cuda_rhs(1500, 8, 1)
    with pytest.raises(g.GofmmError):
        g.evaluate_batched([comp], [Wd])
    srv = g.Server(hbm_budget_bytes=1 << 30, streams=1, max_batch=2)
    with pytest.raises(g.GofmmError):
        srv.add(comp, 8)
    srv.close()


def test_geometric_one_column_and_strided_rows(torch):
    """r = 1 and W, U with row strides larger than r (columns past r of U
    untouched)."""
    rng = np.random.default_rng(13)
    n = 2100
    pts = rng.random((n, 5))
    S, comp = _compress(pts, "gaussian", 0.4, 1e-3)
    comp.use_device_kernel(S)
    K = kernels.KernelMatrix(pts, "gaussian", 0.4, 1e-3)
    for r, ld in ((1, 1), (6, 11)):
        log(f"case geometric r={r} ld={ld}")
        W64, Wd = cuda_rhs(n, r, 40 + r, ld)
        big = torch.full((n, ld + 3), 7.0, device="cuda")
        Ud = big[:, :r]
        comp.evaluate(Wd, Ud)
        torch.cuda.synchronize()
        ref = evaluate.tree_walk(export_read(comp), K, Wd.cpu().numpy().astype(np.float64))
        _check(Ud.cpu().numpy(), ref, what=f"r={r} ld={ld}")
        assert torch.all(big[:, r:] == 7.0)


def test_geometric_with_persistent_tree_passes(torch, monkeypatch):
    """The opt-in persistent upward and downward passes in front of the
    device-computed near field give the same bits as separate launches."""
    import paper_1707_00164_amd as g
    rng = np.random.default_rng(17)
    n = 5000
    pts = rng.random((n, 4))
    S, comp = _compress(pts, "gaussian", 0.4, 1e-3, leaf_size=96)
    comp.use_device_kernel(S)
    W64, Wd = cuda_rhs(n, 40, 6)
    monkeypatch.setenv("GOFMM_PASSES", "0")
    ref = comp.evaluate(Wd)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    monkeypatch.setenv("GOFMM_PASSES", "1")
    log(f"case geometric with persistent passes: launches {[l[0] for l in comp.launches()]}")
    U = torch.empty_like(Wd)
    for rep in range(3):
        comp.evaluate(Wd, U)
        torch.cuda.synchronize()
        assert np.array_equal(U.cpu().numpy(), ref), rep
    assert comp.status() == 0
