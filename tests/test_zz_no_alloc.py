"""The allocation-free evaluate (gofmm_evaluate_noalloc, C ABI through
ctypes): its workspace and work items live in the library's fixed scratch
array.  Its output must equal gofmm_evaluate's bit for bit (same kernels, same
k order per element), on two calls in a row, the second with a smaller input
(fewer right-hand sides, then a smaller compression), and sizes beyond the
array are rejected before anything is launched."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import cuda_rhs, log

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 256 << 20


def _comp(g, n, seed, **kw):
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    S = g.KernelSampler(pts, "gaussian", 0.3, 1e-3)
    return g.Compression.compress(S, leaf_size=100, max_rank=64, tol=1e-6, kappa=16, budget=0.1, seed=seed, **kw)


def _noalloc(g, comp, W, U):
    rc = g.lib().gofmm_evaluate_noalloc(comp.h, W.shape[1], W.data_ptr(), W.stride(0), U.data_ptr(),
                                        U.stride(0), C.c_void_p(None))
    return rc


def test_noalloc_matches_evaluate_on_consecutive_calls():
    import torch
    import paper_1707_00164_amd as g
    assert torch.cuda.is_available()
    g.lib()
    big = _comp(g, 3001, 4)
    small = _comp(g, 1300, 6, storage=g.BF16X3, near_storage=g.BF16X3)
    cases = [(big, 130), (big, 45), (small, 33)]
    for comp in (big, small):
        comp.prepare(130)
    for comp, r in cases:
        log(f"case noalloc n={comp.n} r={r}")
        _, W = cuda_rhs(comp.n, r, 10 + r)
        want = comp.evaluate(W)
        torch.cuda.synchronize()
        U = torch.full_like(W, float("nan"))
        assert _noalloc(g, comp, W, U) == 0, g.lib().gofmm_last_error()
        torch.cuda.synchronize()
        assert np.array_equal(U.cpu().numpy(), want.cpu().numpy())
    # strided operands, and a repeat of the first case after the smaller ones
    _, W = cuda_rhs(big.n, 37, 3, ld=40)
    want = big.evaluate(W)
    Ubig = torch.full((big.n, 41), float("nan"), device="cuda")
    U = Ubig[:, :37]
    assert _noalloc(g, big, W, U) == 0
    torch.cuda.synchronize()
    assert np.array_equal(U.cpu().numpy(), want.cpu().numpy())
    assert torch.isnan(Ubig[:, 37:]).all()


def test_noalloc_rejects_what_does_not_fit_and_unprepared():
    import torch
    import paper_1707_00164_amd as g
    g.lib()
    comp = _comp(g, 3001, 4)
    _, W = cuda_rhs(comp.n, 8, 1)
    U = torch.empty_like(W)
    assert _noalloc(g, comp, W, U) == -1                     # not on the device yet
    comp.prepare(8)
    ws_rows = comp.stats().workspace_rows
    r = (SCRATCH_BYTES // (4 * ws_rows) + 8) // 4 * 4        # workspace alone exceeds the array
    Wb = torch.zeros((comp.n, r), device="cuda")
    Ub = torch.empty_like(Wb)
    log(f"case noalloc over the limit: workspace rows {ws_rows}, r={r}")
    assert _noalloc(g, comp, Wb, Ub) == -7                   # GOFMM_ELIMIT
    assert b"scratch" in g.lib().gofmm_last_error()
    assert _noalloc(g, comp, W, U) == 0
    want = comp.evaluate(W)
    torch.cuda.synchronize()
    assert np.array_equal(U.cpu().numpy(), want.cpu().numpy())
