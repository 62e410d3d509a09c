"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself by retyping its formulas: each
test checks it against brute force, a library routine, a closed form, an
invariant the paper states, or the worked example of Fig. 2.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import workloads
from oracle import cfile, compress, dense, evaluate, kernels

HERE = os.path.dirname(os.path.abspath(__file__))


def _small_kernel(n=512, d=3, kind="gaussian", h=0.5, shift=1e-3, seed=5):
    rng = np.random.default_rng(seed)
    return kernels.KernelMatrix(rng.random((n, d)), kind, h, shift)


# ------------------------------------------------------------------ kernels
@pytest.mark.parametrize("kind,h", [("gaussian", 0.5), ("imq", 0.3), ("laplace_like", 1.0)])
def test_kernel_entries_match_scalar_math(kind, h):
    K = _small_kernel(64, 4, kind, h, 1e-2)
    blk = K(np.arange(64), np.arange(64))
    for i, j in [(0, 0), (3, 17), (17, 3), (63, 1), (10, 10)]:
        d2 = math.fsum((K.x[i, c] - K.x[j, c]) ** 2 for c in range(4))
        if kind == "gaussian":
            v = math.exp(-d2 / (2 * h * h))
        elif kind == "imq":
            v = 1.0 / math.sqrt(1.0 + d2 / (h * h))
        else:
            v = 1.0 / (math.sqrt(d2) + 0.05)
        v += 1e-2 if i == j else 0.0
        assert blk[i, j] == pytest.approx(v, rel=1e-14, abs=1e-300)
    assert np.array_equal(blk, blk.T)
    np.linalg.cholesky(blk)                      # SPD
    assert np.allclose(K.diag(), np.diag(blk), rtol=1e-15)


def test_dense_kw_entries_by_fsum():
    K = _small_kernel(300)
    W = workloads.rhs(300, 3, 11)
    U = dense.kw(K, W)
    full = K(np.arange(300), np.arange(300))
    for i, c in [(0, 0), (150, 1), (299, 2)]:
        assert U[i, c] == pytest.approx(math.fsum(full[i, j] * W[j, c] for j in range(300)), rel=1e-13)
    rows = np.array([5, 77, 299])
    assert np.allclose(dense.kw(K, W, rows), U[rows], rtol=1e-14, atol=0)


# ------------------------------------------------------------------ distances
def test_gram_l2_equals_distance_of_cholesky_vectors():
    A = workloads.random_spd(200, 3)
    K = kernels.DenseMatrix(A)
    phi = np.linalg.cholesky(A)                   # K = phi phi^T: rows are Gram vectors
    I = np.arange(200)
    d = compress.distance(K, K.diag(), I, I, compress.GRAM_L2)
    ref = np.linalg.norm(phi[:, None, :] - phi[None, :, :], axis=2)
    assert np.max(np.abs(d ** 2 - ref ** 2)) <= 1e-12 * np.max(np.diag(A))


def test_angle_distance_equals_sin2_of_cholesky_vectors():
    A = workloads.random_spd(120, 4)
    K = kernels.DenseMatrix(A)
    phi = np.linalg.cholesky(A)
    I = np.arange(120)
    d = compress.distance(K, K.diag(), I, I, compress.ANGLE)
    nrm = np.linalg.norm(phi, axis=1)
    cos = (phi @ phi.T) / np.outer(nrm, nrm)
    assert np.allclose(d, 1.0 - cos ** 2, atol=1e-13)
    assert d.min() >= 0.0 and d.max() <= 1.0


def test_exact_knn_by_brute_force():
    K = _small_kernel(60, 2)
    diag = K.diag()
    knn = compress.exact_knn(K, diag, 60, 7, compress.GRAM_L2)
    full = K(np.arange(60), np.arange(60))
    for i in range(60):
        ds = []
        for j in range(60):
            d2 = full[i, i] + full[j, j] - 2 * full[i, j]
            ds.append((math.sqrt(max(d2, 0.0)), j))
        ds.sort()
        assert [j for _, j in ds[:7]] == list(knn[i])
        assert knn[i][0] == i                         # an index is its own nearest neighbour


# ------------------------------------------------------------------ tree
def test_metric_split_is_algorithm_1():
    K = _small_kernel(257, 3)
    diag = K.diag()
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(1000, 257, replace=False)) % 257
    idx = np.unique(idx)
    left, right, p, q, C = compress.metric_split(idx, K, diag, compress.GRAM_L2, np.random.default_rng(3))
    assert len(left) == (len(idx) + 1) // 2 and len(left) + len(right) == len(idx)
    assert np.array_equal(np.sort(np.concatenate([left, right])), idx)
    phi = np.linalg.cholesky(K(np.arange(257), np.arange(257)))
    c = phi[C].mean(axis=0)
    dc = np.linalg.norm(phi[idx] - c, axis=1)
    assert p == idx[np.argmax(dc)]
    dp = np.linalg.norm(phi[idx] - phi[p], axis=1)
    assert q == idx[np.argmax(dp)]
    v = dp - np.linalg.norm(phi[idx] - phi[q], axis=1)
    vl = v[np.isin(idx, left)]
    vr = v[np.isin(idx, right)]
    assert vl.max() <= vr.min() + 1e-9


def test_tree_is_balanced_partition():
    K = _small_kernel(1000, 3)
    c = compress.compress(K, 1000, leaf_size=64, max_rank=32, tol=1e-5, kappa=8, budget=0.0, seed=2)
    assert c.depth == 4
    assert np.array_equal(np.sort(c.perm), np.arange(1000))
    fl = cfile.first_leaf(c.depth)
    sizes = c.node_size[fl:]
    assert sizes.max() - sizes.min() <= 1 and sizes.max() <= 64
    for h in range(fl):
        assert c.node_size[h] == c.node_size[2 * h + 1] + c.node_size[2 * h + 2]
        assert c.node_start[2 * h + 1] == c.node_start[h]
        assert c.node_start[2 * h + 2] == c.node_start[h] + c.node_size[2 * h + 1]


# ------------------------------------------------------------------ lists
def test_fig2_findfar_and_mergefar_worked_example():
    g = json.load(open(os.path.join(HERE, "golden", "fig2_findfar_mergefar.json")))
    D = g["depth"]
    fl = cfile.first_leaf(D)
    far = [set() for _ in range(cfile.n_nodes(D))]
    for b in range(1 << D):
        far[fl + b] = set(compress.find_far(D, {fl + b}))
    assert sorted(far[g["l"]]) == g["findfar_l"]
    assert sorted(far[g["r"]]) == g["findfar_r"]
    compress.merge_far(D, far, at=g["alpha"])
    for node, expect in g["after_mergefar_at_alpha"].items():
        assert sorted(far[int(node)]) == expect


def _sibling(h):
    return h + 1 if h % 2 == 1 else h - 1


@pytest.mark.parametrize("D", [1, 2, 3, 5])
def test_hss_far_is_sibling(D):
    fl = cfile.first_leaf(D)
    far = [set() for _ in range(cfile.n_nodes(D))]
    for b in range(1 << D):
        far[fl + b] = set(compress.find_far(D, {fl + b}))
    compress.merge_far(D, far)
    assert far[0] == set()
    for h in range(1, cfile.n_nodes(D)):
        assert far[h] == {_sibling(h)}


def _covered_once(D, near_lists, far):
    fl = cfile.first_leaf(D)
    L = 1 << D
    cnt = np.zeros((L, L), dtype=int)
    for b in range(L):
        for a in near_lists[b]:
            cnt[b, a] += 1
    for h in range(cfile.n_nodes(D)):
        for a in far[h]:
            for bl in range(L):
                if compress._contains(h, fl + bl):
                    for al in range(L):
                        if compress._contains(a, fl + al):
                            cnt[bl, al] += 1
    return cnt


def _random_near(D, seed, p=0.15):
    L = 1 << D
    rng = np.random.default_rng(seed)
    near = [{b} for b in range(L)]
    for b in range(L):
        for a in range(L):
            if rng.random() < p:
                near[b].add(a)
                near[a].add(b)
    return near


@pytest.mark.parametrize("D,seed", [(2, 0), (3, 1), (4, 2), (5, 3)])
def test_far_lists_cover_every_pair_once_and_refinement_is_symmetric(D, seed):
    fl = cfile.first_leaf(D)
    near = _random_near(D, seed)
    far = [set() for _ in range(cfile.n_nodes(D))]
    for b in range(1 << D):
        far[fl + b] = set(compress.find_far(D, {fl + a for a in near[b]}))
    compress.merge_far(D, far)
    assert far[0] == set()
    assert np.all(_covered_once(D, near, far) == 1)
    ref = compress.symmetric_refinement(D, far, [np.array(sorted(x)) for x in near])
    assert np.all(_covered_once(D, near, ref) == 1)
    pairs = {(h, a) for h in range(len(ref)) for a in ref[h]}
    assert pairs == {(a, h) for (h, a) in pairs}
    for (h, a) in pairs:                          # refined pairs are disjoint nodes
        assert not compress._contains(h, a) and not compress._contains(a, h)


def test_refinement_fixes_the_asymmetric_four_leaf_case():
    # 4 leaves (heap 3..6), Near = self plus leaf 0 ~ leaf 2 (heap 3 ~ 5).
    D = 2
    near = [{0, 2}, {1}, {2, 0}, {3}]
    fl = cfile.first_leaf(D)
    far = [set() for _ in range(cfile.n_nodes(D))]
    for b in range(4):
        far[fl + b] = set(compress.find_far(D, {fl + a for a in near[b]}))
    compress.merge_far(D, far)
    pairs = {(h, a) for h in range(7) for a in far[h]}
    assert (4, 2) in pairs and (2, 4) not in pairs     # Alg. 3/4 alone are not symmetric here
    ref = compress.symmetric_refinement(D, far, [np.array(sorted(x)) for x in near])
    rp = {(h, a) for h in range(7) for a in ref[h]}
    assert rp == {(a, h) for (h, a) in rp}
    assert (4, 5) in rp and (4, 6) in rp and (5, 4) in rp and (6, 4) in rp


def test_leaf_near_ballot_and_budget():
    # 4 leaves of 3 indices; hand-made neighbour lists give known votes.
    leaves = [np.array([0, 1, 2]), np.array([3, 4, 5]), np.array([6, 7, 8]), np.array([9, 10, 11])]
    leaf_of = np.repeat(np.arange(4), 3)
    knn = np.array([[i, (i + 3) % 12, (i + 6) % 12] for i in range(12)])
    knn[0] = [0, 9, 10]
    knn[1] = [1, 11, 7]                              # leaf 0 votes: leaf 3 x3, leaf 2 x2, leaf 1 x1
    near = compress.leaf_near(knn, leaf_of, leaves, budget=0.25, n=12, m=3)
    # cap = floor(budget * N / m) = 1 other leaf
    assert 0 in near[0]
    pre = {int(a) for a in near[0]}
    assert 3 in pre                                  # the most voted other leaf of leaf 0
    for b in range(4):
        for a in near[b]:
            assert b in near[int(a)]                 # symmetric
    hss = compress.leaf_near(knn, leaf_of, leaves, budget=0.0, n=12, m=3)
    assert all(list(x) == [b] for b, x in enumerate(hss))


# ------------------------------------------------------------------ skeletons
def test_interp_decomp_matches_pivoted_qr_and_bounds():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((80, 12)) @ rng.standard_normal((12, 40))
    A += 1e-9 * rng.standard_normal(A.shape)
    piv, P = compress.interp_decomp(A, 1e-6, 40)
    assert len(piv) == 12                            # numerical rank
    assert np.allclose(P[:, piv], np.eye(12), atol=0)
    assert np.linalg.norm(A - A[:, piv] @ P) <= 1e-6 * np.linalg.norm(A)
    # Pivots are those of a greedy largest-residual-norm column selection.
    R = A.copy()
    greedy = []
    for _ in range(12):
        nrm = np.linalg.norm(R, axis=0)
        nrm[greedy] = -1
        j = int(np.argmax(nrm))
        greedy.append(j)
        v = R[:, j] / np.linalg.norm(R[:, j])
        R = R - np.outer(v, v @ R)
    assert greedy == list(piv)


def test_interp_decomp_full_rank_is_permutation():
    rng = np.random.default_rng(8)
    A = rng.standard_normal((30, 10))
    piv, P = compress.interp_decomp(A, 0.0, 10)
    assert sorted(piv) == list(range(10))
    assert np.array_equal(np.sort(P, axis=1)[:, -1], np.ones(10))
    assert np.count_nonzero(P) == 10
    assert np.array_equal(A[:, piv] @ P, A)


def _case(n=1024, m=64, s=64, tol=1e-6, kappa=16, budget=0.05, seed=1, kind="gaussian"):
    K = _small_kernel(n, 3, kind, 0.4, 1e-3, seed=seed + 10)
    c = compress.compress(K, n, leaf_size=m, max_rank=s, tol=tol, kappa=kappa, budget=budget, seed=seed)
    return K, c


def test_skeletons_are_nested():
    _, c = _case()
    fl = cfile.first_leaf(c.depth)
    for h in range(1, c.nn):
        if h < fl:
            kids = set(c.skel[2 * h + 1]) | set(c.skel[2 * h + 2])
            assert set(c.skel[h]) <= kids
        else:
            assert set(c.skel[h]) <= set(c.indices(h))
        assert 1 <= c.rank(h) <= c.max_rank


def test_telescoped_P_equals_upward_pass():
    K, c = _case()
    W = workloads.rhs(c.n, 5, 3)
    wt = evaluate.upward(c, W[c.perm])
    ph = evaluate.telescoped(c)
    for h in range(1, c.nn):
        a = int(c.node_start[h])
        ref = ph[h] @ W[c.perm][a:a + int(c.node_size[h])]
        assert np.allclose(wt[h], ref, rtol=0, atol=1e-13 * max(1.0, np.abs(ref).max()))


# ------------------------------------------------------------------ K~ as a whole
def test_full_rank_gives_exact_K():
    K = _small_kernel(256, 3, "gaussian", 0.3, 1e-3)
    c = compress.compress(K, 256, leaf_size=32, max_rank=256, tol=0.0, kappa=8, budget=0.0, seed=4)
    Kt = evaluate.assemble(c, K)
    Kd = K(np.arange(256), np.arange(256))
    assert np.linalg.norm(Kt - Kd) <= 1e-14 * np.linalg.norm(Kd)
    W = workloads.rhs(256, 4, 2)
    assert np.allclose(evaluate.tree_walk(c, K, W), Kd @ W, rtol=1e-13, atol=1e-13)


def test_all_near_gives_exact_K():
    K = _small_kernel(256, 2)
    c = compress.compress(K, 256, leaf_size=32, max_rank=8, tol=1e-2, kappa=256, budget=1.0, seed=4)
    assert all(len(x) == 8 for x in c.near) and all(len(f) == 0 for f in c.far)
    Kd = K(np.arange(256), np.arange(256))
    assert np.array_equal(evaluate.assemble(c, K), Kd)


def test_single_leaf_gives_exact_K():
    K = _small_kernel(100, 2)
    c = compress.compress(K, 100, leaf_size=128, max_rank=8, tol=1e-2, kappa=4, budget=0.0, seed=4)
    assert c.depth == 0
    W = workloads.rhs(100, 3, 1)
    Kd = K(np.arange(100), np.arange(100))
    assert np.allclose(evaluate.tree_walk(c, K, W), Kd @ W, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("budget", [0.0, 0.1])
def test_K_tilde_is_symmetric_and_walk_equals_assembly(budget):
    K, c = _case(n=1024, budget=budget)
    Kt = evaluate.assemble(c, K)
    assert np.linalg.norm(Kt - Kt.T) <= 1e-14 * np.linalg.norm(Kt)
    W = workloads.rhs(c.n, 6, 9)
    U = evaluate.tree_walk(c, K, W)
    assert np.linalg.norm(U - Kt @ W) <= 1e-12 * np.linalg.norm(U)
    rows = workloads.sample_rows(c.n, 40, 1)
    assert np.allclose(evaluate.tree_walk(c, K, W, rows), U[rows], rtol=1e-13, atol=1e-13)


def test_brute_force_assembly_small():
    # N <= 512: every entry of K~ recomputed pair by pair from its definition.
    K, c = _case(n=256, m=32, s=16, tol=1e-4, budget=0.1)
    ph = evaluate.telescoped(c)
    Kt = evaluate.assemble(c, K)
    fl = cfile.first_leaf(c.depth)
    pos = np.empty(c.n, dtype=int)
    pos[c.perm] = np.arange(c.n)
    leaf_of_pos = np.searchsorted(c.node_start[fl:], np.arange(c.n), side="right") - 1
    rng = np.random.default_rng(0)
    for _ in range(300):
        i, j = rng.integers(0, c.n, 2)
        bi, bj = fl + leaf_of_pos[pos[i]], fl + leaf_of_pos[pos[j]]
        if (bj - fl) in set(int(a) - fl for a in c.near[bi - fl]):
            ref = K([i], [j])[0, 0]
        else:
            hits = []
            x = bi
            while x > 0:
                y = bj
                while y > 0:
                    if y in set(c.far[x]):
                        hits.append((x, y))
                    y = (y - 1) // 2
                x = (x - 1) // 2
            assert len(hits) == 1
            x, y = hits[0]
            ci = pos[i] - c.node_start[x]
            cj = pos[j] - c.node_start[y]
            ref = ph[x][:, ci] @ K(c.skel[x], c.skel[y]) @ ph[y][:, cj]
        assert Kt[i, j] == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_small_gaussian_workload_accuracy():
    w = workloads.small_gaussian()
    K = kernels.for_workload(w)
    c = compress.compress(K, w.n, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol,
                          kappa=w.kappa, budget=w.budget, seed=1)
    W = workloads.rhs(w.n, w.r, w.seed)
    rows = workloads.sample_rows(w.n, 100, w.seed)
    e = dense.eps2(evaluate.tree_walk(c, K, W, rows), dense.kw(K, W, rows))
    print(f"eps2(small gaussian, HSS, tau=1e-5) = {e:.3e}")
    assert e < 1e-3


# ------------------------------------------------------------------ file format
def test_cfile_roundtrip(tmp_path):
    K, c = _case(n=600, m=64, s=32)
    p = str(tmp_path / "c.bin")
    cfile.write(c, p)
    d = cfile.read(p)
    assert d.n == c.n and d.depth == c.depth and d.tol == c.tol
    assert np.array_equal(d.perm, c.perm)
    for h in range(c.nn):
        assert np.array_equal(d.far[h], c.far[h]) and np.array_equal(d.skel[h], c.skel[h])
        if c.proj[h] is not None:
            assert np.array_equal(d.proj[h], c.proj[h])
    W = workloads.rhs(c.n, 2, 0)
    assert np.array_equal(evaluate.tree_walk(d, K, W), evaluate.tree_walk(c, K, W))


# ------------------------------------------------------------------ planted mistakes
def test_planted_mistakes_fail_a_pin(monkeypatch):
    """A dropped term or a swapped operand inside the oracle must break a pin."""
    K = _small_kernel(256, 3, "gaussian", 0.3, 1e-3)
    c = compress.compress(K, 256, leaf_size=32, max_rank=256, tol=0.0, kappa=8, budget=0.0, seed=4)
    Kd = K(np.arange(256), np.arange(256))
    W = workloads.rhs(256, 4, 2)
    good = evaluate.tree_walk(c, K, W)
    assert np.allclose(good, Kd @ W, rtol=1e-13, atol=1e-13)
    orig_upward = evaluate.upward

    def swapped_children(cc, Wp):                  # [w_r; w_l] instead of [w_l; w_r]
        wt = orig_upward(cc, Wp)
        fl = cfile.first_leaf(cc.depth)
        for h in range(fl - 1, 0, -1):
            wt[h] = cc.proj[h] @ np.vstack([wt[2 * h + 2], wt[2 * h + 1]]) if \
                cc.rank(2 * h + 1) == cc.rank(2 * h + 2) else wt[h]
        return wt
    monkeypatch.setattr(evaluate, "upward", swapped_children)
    assert not np.allclose(evaluate.tree_walk(c, K, W), Kd @ W, rtol=1e-6, atol=1e-6)
    monkeypatch.setattr(evaluate, "upward", orig_upward)
    c2 = compress.compress(K, 256, leaf_size=32, max_rank=256, tol=0.0, kappa=8, budget=0.0, seed=4)
    c2.far[1] = np.zeros(0, dtype=np.int64)        # a dropped far pair
    assert not np.allclose(evaluate.tree_walk(c2, K, W), Kd @ W, rtol=1e-6, atol=1e-6)


# ------------------------------------------------------------------ row samples (reading R10)
def test_sample_rows_hand_example_neighbours_first():
    """Hand-worked: members {2, 5, 7} of N = 20, kappa = 4.  Outside the node,
    index 9 gets 3 votes, 3 and 11 get 2 each; |I'| = min(20 - 3, 2 * 3) = 6,
    at most half (3) from the neighbours by (-votes, index): [9, 3, 11], then 3
    distinct uniform draws from the rest of the complement."""
    knn = np.tile(np.arange(20)[:, None], (1, 4))
    knn[2] = [2, 9, 11, 5]
    knn[5] = [5, 9, 3, 11]
    knn[7] = [7, 3, 9, 2]
    members = np.array([2, 5, 7])
    for seed in range(20):
        rows = compress.sample_rows(members, knn, 20, 3, np.random.default_rng(seed))
        assert len(rows) == 6
        assert list(rows[:3]) == [9, 3, 11]
        rest = rows[3:]
        assert len(set(rows.tolist())) == 6
        assert not set(rest.tolist()) & {2, 5, 7, 9, 3, 11}
        assert list(rest) == sorted(rest)


def test_sample_rows_invariants_by_brute_force():
    """Random neighbour lists: rows lie outside the node, are distinct, number
    min(N - |a|, 2 ncols), and start with the ceil-free half of the outside
    neighbours ranked by a vote count taken here with a plain loop."""
    rng = np.random.default_rng(3)
    n, kappa = 60, 5
    knn = np.column_stack([np.arange(n), rng.integers(0, n, size=(n, kappa - 1))])
    for trial in range(40):
        size = int(rng.integers(1, 40))
        members = np.sort(rng.choice(n, size=size, replace=False))
        ncols = int(rng.integers(1, 30))
        rows = compress.sample_rows(members, knn, n, ncols, np.random.default_rng(trial))
        ns = min(n - size, 2 * ncols)
        assert len(rows) == ns
        assert len(set(rows.tolist())) == ns
        assert not set(rows.tolist()) & set(members.tolist())
        votes = {}
        for i in members:
            for j in knn[i]:
                if j not in set(members.tolist()):
                    votes[int(j)] = votes.get(int(j), 0) + 1
        ranked = sorted(votes, key=lambda j: (-votes[j], j))
        head = ranked[:ns // 2]
        assert list(rows[:len(head)]) == head


def test_sample_rows_whole_complement_and_uniform_fill():
    """When 2 ncols reaches N - |a| the sample is the whole complement; the
    uniform part draws every free index about equally often."""
    knn = np.array([[i, (i + 1) % 6] for i in range(6)])
    rows = compress.sample_rows(np.array([0, 1, 2, 3]), knn, 6, 4, np.random.default_rng(0))
    assert sorted(rows.tolist()) == [4, 5] and rows[0] == 4          # 4 is 3's neighbour
    n = 40
    knn = np.tile(np.arange(n)[:, None], (1, 2))                       # no outside neighbours
    counts = np.zeros(n)
    for seed in range(2000):
        rows = compress.sample_rows(np.array([0]), knn, n, 2, np.random.default_rng(seed))
        counts[rows] += 1
    assert counts[0] == 0
    free = counts[1:]
    assert free.sum() == 2000 * 4
    expect = 2000 * 4 / 39
    assert np.all(np.abs(free - expect) < 5 * np.sqrt(expect))


# ------------------------------------------------------------------ eps_2 (Sec. 3)
def test_eps2_hand_value():
    exact = np.array([[1.0, 2.0], [3.0, 5.0]])
    approx = np.array([[1.0, 2.0], [3.0, 4.0]])
    assert dense.eps2(approx, exact) == pytest.approx(1.0 / math.sqrt(39.0), rel=1e-15)
    assert dense.eps2(exact, exact) == 0.0
    assert dense.eps2(2.0 * approx, 2.0 * exact) == pytest.approx(1.0 / math.sqrt(39.0), rel=1e-15)
    assert dense.eps2(np.zeros((2, 2)), exact) == 1.0


# ------------------------------------------------------------------ Table 2 flop count
def test_algorithmic_flops_hss_closed_form():
    """HSS (budget 0) on N = m 2^D with every rank forced to s (tau = 0): Table 2
    gives per right-hand side N2S = 2 m s L + 2 s (2 s)(L - 2), S2S = 2 s^2 (2L - 2)
    (the far pairs are the 2L - 2 sibling pairs), S2N = N2S, L2L = 2 m^2 L."""
    m, s, D, r = 32, 8, 3, 3
    L = 1 << D
    n = m * L
    K = _small_kernel(n, 3, "laplace_like", 1.0, 1e-2)
    c = compress.compress(K, n, leaf_size=m, max_rank=s, tol=0.0, kappa=8, budget=0.0, seed=2)
    assert all(c.rank(h) == s for h in range(1, c.nn))
    assert sum(len(f) for f in c.far) == 2 * L - 2
    n2s = 2 * m * s * L + 2 * s * (2 * s) * (L - 2)
    closed = r * (2 * n2s + 2 * s * s * (2 * L - 2) + 2 * m * m * L)
    assert evaluate.algorithmic_flops(c, r) == closed


def test_algorithmic_flops_all_near_closed_form():
    """Every leaf near every other (kappa = N): no far pairs, L2L is the dense
    product 2 N^2 r, and N2S/S2N keep their HSS counts."""
    m, s, D, r = 16, 4, 2, 5
    L = 1 << D
    n = m * L
    K = _small_kernel(n, 2, "gaussian", 0.5, 1e-3)
    c = compress.compress(K, n, leaf_size=m, max_rank=s, tol=0.0, kappa=n, budget=1.0, seed=3)
    assert all(len(f) == 0 for f in c.far) and all(len(x) == L for x in c.near)
    n2s = 2 * m * s * L + 2 * s * (2 * s) * (L - 2)
    assert evaluate.algorithmic_flops(c, r) == r * (2 * n2s + 2 * n * n)
