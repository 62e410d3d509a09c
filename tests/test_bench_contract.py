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

    rl = bench.roofline(Launches(), 0, 1.0, {"leaf": 1.0}, 512, "f32")
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        traffic = json.load(f)
    if traffic["fingerprint"] == bench._fingerprint():
        assert rl["traffic"] == traffic["bytes_per_launch"]
    else:
        assert rl["traffic"] is None
    assert rl["frac"] == round(rl["achieved"] / 157.3, 4)
