"""The benchmark's command-line contract on a machine without a GPU: more
than one GPU is refused with a JSON message and exit status 2 (the
evaluator measures one GPU), and the stored counter figures match the kernel
sources they were taken on, or the benchmark reports them as null."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_counter_figures_follow_the_sources():
    sys.path.insert(0, ROOT)
    import bench

    class Launches:
        def launches(self):
            return [("leaf", 1.0e9, 1 << 20)]

    rl = bench.roofline(Launches(), 0, 1.0, {"leaf": 1.0}, 512, "f32", workload="gauss6d_n65536_r512")
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        entries = [e for e in json.load(f) if e["launch"] == "leaf" and e["form"] == "f32"
                   and e["workload"] == "gauss6d_n65536_r512"]
    current = [e for e in entries if e["fingerprint"] == bench._fingerprint()]
    if current:
        assert rl["traffic"] == current[-1]["bytes_per_launch"]
    else:
        assert rl["traffic"] is None
    assert rl["frac"] == round(rl["achieved"] / 157.3, 4)


def test_sampled_walk_flops():
    """The CPU baseline's flop count of a row-restricted oracle walk equals
    the whole K~W's Table 2 count when every row is asked for, and counts the
    upward pass once and nothing else when no row is."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    import workloads
    from oracle import compress, evaluate, kernels
    rng = np.random.default_rng(3)
    n = 700
    K = kernels.KernelMatrix(rng.random((n, 3)), "gaussian", 0.3, 1e-3)
    c = compress.compress(K, n, leaf_size=64, max_rank=24, tol=1e-6, kappa=8, budget=0.1, seed=2)
    assert bench.sample_flops(c, np.arange(n), 5) == evaluate.algorithmic_flops(c, 5)
    up = 0.0
    for h in range(1, c.nn):
        fl = (1 << c.depth) - 1
        ncol = int(c.node_size[h]) if h >= fl else c.rank(2 * h + 1) + c.rank(2 * h + 2)
        up += 2.0 * c.rank(h) * ncol * 5
    assert bench.sample_flops(c, np.zeros(0, dtype=np.int64), 5) == up
    rows = workloads.sample_rows(n, 10, 1)
    assert up < bench.sample_flops(c, rows, 5) < evaluate.algorithmic_flops(c, 5)
