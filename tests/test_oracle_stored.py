"""Pins of the oracle's storage-form evaluation (oracle/stored.py), CPU only.

BF16 rounding is checked against hand-worked values and PyTorch's own
float32 -> bfloat16 conversion (round to nearest, ties to even); the split
against its error bound; the evaluation against the exact tree walk where
every operand is exactly representable, against dense products for a single
leaf, and against a step-by-step depth-1 walk rounded by PyTorch.
"""
import numpy as np
import pytest

import grid_cases
import workloads
from oracle import compress, evaluate, kernels, stored


def test_bf16_hand_values():
    u = 2.0 ** -8
    cases = [
        (1.0, 1.0),
        (1.0 + u, 1.0),                          # tie between 1 and 1 + 2^-7: even is 1
        (1.0 + 3 * u, 1.0 + 4 * u),              # tie: 1 + 2^-6 has the even last bit
        (1.0 + u + 2.0 ** -30, 1.0 + 2 * u),     # just above the tie
        (255.5, 256.0),                          # spacing 1 below 256, tie to even
        (257.0, 256.0),                          # spacing 2 above 256, tie to even
        (259.0, 260.0),
        (-(1.0 + 3 * u), -(1.0 + 4 * u)),
        (2.0 ** -130 + 2.0 ** -134, 2.0 ** -130),  # subnormal spacing 2^-133, tie to even
        (3 * 2.0 ** -134, 2 * 2.0 ** -133),
        (3.4e38, np.inf),                        # past the largest finite BF16
        (0.0, 0.0),
    ]
    for x, want in cases:
        assert stored.bf16(x) == want, (x, stored.bf16(x), want)
    assert np.isnan(stored.bf16(np.nan))
    assert stored.bf16(-np.inf) == -np.inf


def test_bf16_matches_torch_on_float32_values():
    import torch
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        rng.standard_normal(20000)]).astype(np.float32)
    bits = x.view(np.uint32)
    ties = ((bits & ~np.uint32(0xFFFF)) | np.uint32(0x8000)).view(np.float32)   # exact midpoints
    for v in (x, ties):
        ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
        assert np.array_equal(stored.bf16(v.astype(np.float64)), ref)


def test_split_error_bound_and_exact_integers():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(50000) * 10.0 ** rng.integers(-8, 8, 50000)
    hi, lo = stored.split(x)
    assert np.array_equal(hi, stored.bf16(hi)) and np.array_equal(lo, stored.bf16(lo))
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -17 * np.abs(x))
    k = rng.integers(-(1 << 16) + 1, 1 << 16, 10000).astype(np.float64)   # 16-bit integers
    hi, lo = stored.split(k)
    assert np.array_equal(hi + lo, k)


def _walks(name):
    c, A = grid_cases.build(*grid_cases.CASES[name], seed=1)
    K = kernels.DenseMatrix(A)
    W = grid_cases.integer_rhs(c.n, 6, 3)
    return c, A, K, W


@pytest.mark.parametrize("name", sorted(grid_cases.CASES))
def test_grid_case_sums_are_exact_and_forms_agree(name, monkeypatch):
    """Integer grid: every operand magnitude and every |A| |B| bound stays
    below 2^22, so FP64 (and FP32) sums are exact; FP32 and split storage then
    equal the exact tree walk bit for bit, and split equals it because the
    split of an integer below 2^16 is exact."""
    c, A, K, W = _walks(name)
    exact = evaluate.tree_walk(c, K, W)
    biggest = [0.0]
    real = stored.product

    def tracked(Aop, B, form):
        bound = np.abs(np.asarray(Aop)) @ np.abs(np.asarray(B))
        biggest[0] = max(biggest[0], float(np.max(np.abs(B), initial=0)), float(np.max(bound, initial=0)))
        return real(Aop, B, form)

    monkeypatch.setattr(stored, "product", tracked)
    f32 = stored.tree_walk_stored(c, K, W, "fp32")
    assert biggest[0] < 2.0 ** 22
    assert np.array_equal(f32, exact)
    x3 = stored.tree_walk_stored(c, K, W, "bf16x3")
    if biggest[0] < 2.0 ** 16:
        assert np.array_equal(x3, exact)
    b16 = stored.tree_walk_stored(c, K, W, "bf16")
    assert np.array_equal(b16, np.rint(b16))        # BF16 of an integer >= 1 is an integer
    assert not np.array_equal(b16, exact)           # some intermediate exceeded 8 bits


def test_single_leaf_bf16_is_dense_product_rounded_by_torch():
    import torch
    rng = np.random.default_rng(4)
    n = 90
    Kk = kernels.KernelMatrix(rng.random((n, 3)), "gaussian", 0.5, 1e-3)
    c = compress.compress(Kk, n, leaf_size=128, max_rank=8, tol=1e-3, kappa=4, budget=0.0, seed=1)
    assert c.depth == 0
    W = workloads.rhs(n, 5, 2).astype(np.float32).astype(np.float64)
    Kd = Kk(np.arange(n), np.arange(n))

    def tb(x):
        return torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()

    # K is rounded from FP64 directly; its FP32 image rounds the same way
    # unless FP32 rounding lands on a BF16 midpoint, which these entries avoid
    want = tb(Kd) @ tb(W)
    got = stored.tree_walk_stored(c, Kk, W, "bf16")
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_depth_one_hss_bf16_step_by_step():
    """Two leaves, HSS: U_b = P_b^T bf16(u~_b) + K_bb W_b with u~_b =
    K(b~, a~) bf16(w~_a) and w~_a = P_a bf16(W_a); every rounding by torch."""
    import torch

    def tb(x):
        return torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()

    rng = np.random.default_rng(5)
    n = 200
    Kk = kernels.KernelMatrix(rng.random((n, 2)), "imq", 0.3, 1e-2)
    c = compress.compress(Kk, n, leaf_size=100, max_rank=12, tol=1e-7, kappa=4, budget=0.0, seed=2)
    assert c.depth == 1
    W = workloads.rhs(n, 3, 4).astype(np.float32).astype(np.float64)
    Wp = W[c.perm]
    rows = {h: slice(int(c.node_start[h]), int(c.node_start[h] + c.node_size[h])) for h in (1, 2)}
    # FP32 images of the FP64 operators round to BF16 like the FP64 values here
    # (checked below), so torch's float32 conversion stands in for the direct one
    for h in (1, 2):
        assert np.array_equal(tb(c.proj[h]), stored.bf16(c.proj[h]))
    wt = {h: tb(c.proj[h]) @ tb(Wp[rows[h]]) for h in (1, 2)}
    ut = {1: tb(Kk(c.skel[1], c.skel[2])) @ tb(wt[2]), 2: tb(Kk(c.skel[2], c.skel[1])) @ tb(wt[1])}
    Up = np.zeros_like(Wp)
    for h in (1, 2):
        Up[rows[h]] = tb(c.proj[h]).T @ tb(ut[h]) + tb(Kk(c.indices(h), c.indices(h))) @ tb(Wp[rows[h]])
    want = np.empty_like(Up)
    want[c.perm] = Up
    got = stored.tree_walk_stored(c, Kk, W, "bf16")
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_planted_rounding_mistakes_are_caught():
    """Truncation instead of rounding, or forming the lo*lo product, changes
    what the pins above check."""
    x = np.array([1.0 + 3 * 2.0 ** -8])
    trunc = np.floor(x * 2 ** 7) / 2 ** 7
    assert stored.bf16(x)[0] != trunc[0]
    a = np.array([[1.0 + 2.0 ** -10]])
    b = np.array([[1.0 + 2.0 ** -11]])
    ah, al = stored.split(a)
    bh, bl = stored.split(b)
    full = ah @ bh + ah @ bl + al @ bh + al @ bl
    assert stored.product(a, b, "bf16x3")[0, 0] != full[0, 0]


@pytest.mark.parametrize("seed", [0, 1])
def test_bf16_allowance_covers_a_simulated_device(seed, monkeypatch):
    """A walk whose every intermediate is moved, before its BF16 rounding, by
    an FP32-sized error (up to 4 FP32 units of the |a||b| sum that formed it)
    stays within the allowance of every element.  (The allowance is loose,
    about 1e-3 of max |U| here: once an intermediate may round either way,
    everything downstream of it carries the BF16 spacing.)"""
    rng = np.random.default_rng(seed)
    n = 1500
    Kk = kernels.KernelMatrix(rng.random((n, 3)), "gaussian", 0.3, 1e-3)
    c = compress.compress(Kk, n, leaf_size=96, max_rank=40, tol=1e-7, kappa=8, budget=0.1, seed=seed)
    W = workloads.rhs(n, 6, seed).astype(np.float32).astype(np.float64)
    ref = stored.tree_walk_stored(c, Kk, W, "bf16")
    allow = stored.bf16_allowance(c, Kk, W)
    real = stored.product
    noise = np.random.default_rng(seed + 10)

    def device_like(A, B, form):
        out = real(A, B, form)
        s = np.abs(stored.bf16(A)) @ np.abs(stored.bf16(B))
        return out + s * 4 * 2.0 ** -24 * noise.uniform(-1, 1, size=out.shape)

    monkeypatch.setattr(stored, "product", device_like)
    sim = stored.tree_walk_stored(c, Kk, W, "bf16")
    monkeypatch.setattr(stored, "product", real)
    diff = np.abs(sim - ref)
    assert diff.max() > 0
    assert np.all(diff <= allow)


def test_sampled_rows_equal_the_full_walk():
    rng = np.random.default_rng(9)
    n = 1200
    Kk = kernels.KernelMatrix(rng.random((n, 3)), "imq", 0.3, 1e-2)
    c = compress.compress(Kk, n, leaf_size=64, max_rank=32, tol=1e-6, kappa=8, budget=0.05, seed=1)
    W = workloads.rhs(n, 4, 1)
    rows = workloads.sample_rows(n, 50, 2)
    for form in ("fp32", "bf16", "bf16x3"):
        assert np.array_equal(stored.tree_walk_stored(c, Kk, W, form, rows=rows),
                              stored.tree_walk_stored(c, Kk, W, form)[rows])
    assert np.array_equal(stored.bf16_allowance(c, Kk, W, rows=rows), stored.bf16_allowance(c, Kk, W)[rows])


@pytest.mark.parametrize("name", sorted(grid_cases.CASES))
def test_fp32_carry_is_exact_on_integer_grids(name):
    """Integer intermediates below 2^24 are FP32 values: carrying them in FP32
    changes nothing in any form."""
    c, A, K, W = _walks(name)
    for form in ("fp32", "bf16", "bf16x3"):
        assert np.array_equal(stored.tree_walk_stored(c, K, W, form, carry="fp32"),
                              stored.tree_walk_stored(c, K, W, form))


def test_depth_one_hss_bf16_fp32_carry_step_by_step():
    """Two leaves, HSS, plain BF16 P and coupling blocks, FP32 near blocks,
    FP32 intermediates: w~ and u~ rounded to FP32 once formed, each rounded to
    BF16 (by torch, from its FP32 value) as an operand."""
    import torch

    def tb(x):
        return torch.from_numpy(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()

    def f32(x):
        return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)

    rng = np.random.default_rng(6)
    n = 200
    Kk = kernels.KernelMatrix(rng.random((n, 2)), "gaussian", 0.4, 1e-2)
    c = compress.compress(Kk, n, leaf_size=100, max_rank=12, tol=1e-7, kappa=4, budget=0.0, seed=3)
    assert c.depth == 1
    W = workloads.rhs(n, 3, 7).astype(np.float32).astype(np.float64)
    Wp = W[c.perm]
    rows = {h: slice(int(c.node_start[h]), int(c.node_start[h] + c.node_size[h])) for h in (1, 2)}
    ba = stored.bf16                  # stored operators: BF16 of the FP64 value (pinned above)
    wt = {h: f32(ba(c.proj[h]) @ tb(Wp[rows[h]])) for h in (1, 2)}
    ut = {1: f32(ba(Kk(c.skel[1], c.skel[2])) @ tb(wt[2])), 2: f32(ba(Kk(c.skel[2], c.skel[1])) @ tb(wt[1]))}
    Up = np.zeros_like(Wp)
    for h in (1, 2):
        Up[rows[h]] = (ba(c.proj[h]).T @ tb(ut[h]) +
                       Kk(c.indices(h), c.indices(h)).astype(np.float32).astype(np.float64) @ Wp[rows[h]])
    want = np.empty_like(Up)
    want[c.perm] = Up
    got = stored.tree_walk_stored(c, Kk, W, "bf16", "fp32", carry="fp32")
    assert np.allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())
    # the carry is live: split BF16 reads the low bits of each intermediate
    assert not np.array_equal(stored.tree_walk_stored(c, Kk, W, "bf16x3", carry="fp32"),
                              stored.tree_walk_stored(c, Kk, W, "bf16x3"))


def test_plain_bf16_is_sensitive_to_fp32_level_differences():
    """Why plain BF16 is compared element by element only on exact (integer)
    inputs: each intermediate is rounded to 8 significant bits before it is
    used, so a difference of a few FP32 units in the sums that form it (a
    different accumulation order) flips some of those roundings, and the
    flips compound up the tree.  Two walks that differ only by such noise
    differ by far more than FP32 roundoff, though by less than one BF16 unit
    (2^-8) and less than the form's own storage error."""
    rng = np.random.default_rng(1)
    n = 3000
    Kk = kernels.KernelMatrix(rng.random((n, 4)), "imq", 0.3, 1e-2)
    c = compress.compress(Kk, n, leaf_size=96, max_rank=96, tol=1e-6, kappa=16, budget=0.03, seed=1)
    W = workloads.rhs(n, 8, 2).astype(np.float32).astype(np.float64)
    ref = stored.tree_walk_stored(c, Kk, W, "bf16", "fp32", carry="fp32")
    real = stored.product
    noise = np.random.default_rng(5)

    def perturbed(A, B, form):
        out = real(A, B, form)
        s = np.abs(stored.bf16(A)) @ np.abs(stored.bf16(B))
        return out + s * 4 * 2.0 ** -24 * noise.uniform(-1, 1, size=out.shape)

    try:
        stored.product = perturbed
        sim = stored.tree_walk_stored(c, Kk, W, "bf16", "fp32", carry="fp32")
    finally:
        stored.product = real
    d = np.linalg.norm(sim - ref) / np.linalg.norm(ref)
    storage = np.linalg.norm(ref - stored.tree_walk_stored(c, Kk, W, "fp32")) / np.linalg.norm(ref)
    assert 1e-5 < d < min(2.0 ** -8, storage)
