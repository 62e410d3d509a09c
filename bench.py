#!/usr/bin/env python3
"""Throughput of K~W on one MI355X: the N=262144 inverse-multiquadric workload at r=2048.

Headline workload: 262144 uniform points in 4-D, inverse multiquadric kernel
1/sqrt(1 + |x - y|^2 / 0.3^2) plus 1e-2 on the diagonal, leaf size 512, max
rank 512, tau 1e-6, kappa 32, near budget 3%; r = 2048 FP32 right-hand sides
(the largest workload that one GPU holds).  The same structure is also timed
with BF16 P and coupling blocks (near blocks FP32) and with split-BF16
storage, and the N=65536 clustered-Gaussian workload (r = 512) follows as a
secondary block.

A step is one whole K~W (every launch of N2S, S2S, S2N and L2L, the
permutation folded in) with W and U resident in HBM.  The compression is
built on the host first and is not timed.  The reported value is the
dense-equivalent rate 2 N^2 r / t.  The roofline block covers the dominant
launch: its Table 2 flops divided by its average duration, measured with HIP
events around that launch on the evaluation stream during the timed steps,
against the published peak and against ceilings measured on the same GPU
(vendor GEMM, device copy).  The CPU baseline times the FP64 oracle's walk of
the same compression restricted to 64 sampled rows (whole upward pass, then
the far and near field of those rows), scaled to a whole K~W by Table 2
flops, plus a one-thread figure on a smaller sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "K~W effective GFLOP/s (2N²r/t), MFMA/HBM roofline %, p50/p99 at err≤1e-4"
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}
HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_steps(comp, W, U, steps, warmup, torch):
    """Per-launch shares from an untimed profiled pass, then `steps` timed
    evaluates with HIP events around the dominant launch only (two events per
    step, on the evaluation stream).  Returns (seconds per step, launch index,
    its average ms in the timed region, shares)."""
    for _ in range(warmup):
        comp.evaluate(W, U)
    torch.cuda.synchronize()
    comp.profile(True)
    comp.profile_read()
    for _ in range(3):
        comp.evaluate(W, U)
    ms, calls = comp.profile_read()
    comp.profile(False)
    names = [l[0] for l in comp.launches()]
    share = {names[k]: round(ms[k] / max(sum(ms), 1e-30), 4) for k in range(len(ms))}
    dom = max(range(len(ms)), key=lambda k: ms[k])
    comp.profile(True, launch=dom)
    comp.profile_read()
    # events around every step on the evaluation stream (torch's current
    # stream, which the evaluate calls use) give the per-step median
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        comp.evaluate(W, U)
        b.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, calls = comp.profile_read()
    comp.profile(False)
    per = sorted(a.elapsed_time(b) for a, b in ev)
    time_steps.median_ms = per[len(per) // 2] if per else float("nan")
    return (t1 - t0) / steps, dom, ms[dom] / max(calls[dom], 1), share


# Peak of a precision form in algorithmic TFLOP/s: split BF16 issues three BF16
# matrix-core products per FP32-equivalent product.
FORM_PEAK = {"f32": ("f32", 1.0), "bf16": ("bf16", 1.0), "bf16x3": ("bf16", 3.0)}


def roofline(comp, dom, dom_ms, share, r, form, near_form=None, workload=None):
    """Roofline of the dominant launch; `near_form` is the precision form of
    the near-field launch (l2l) when it differs from the rest.  Counter
    figures (HBM traffic, matrix-core busy) come from profiles/ for this
    launch, form and workload, if they were taken on the current sources."""
    name, fl, byts = comp.launches()[dom]
    if name == "l2l" and near_form is not None:
        form = near_form
    avg_s = dom_ms / 1e3
    achieved = fl * r / avg_s / 1e12
    base, products = FORM_PEAK[form]
    peak = round(PEAK_TFLOPS[base] / products, 1)
    def match(e):
        return (e.get("launch") == name and e.get("form") == form and e.get("fingerprint") == _fingerprint()
                and (workload is None or e.get("workload") == workload))
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            for e in json.load(open(tfile)):
                if match(e):
                    traffic = e.get("bytes_per_launch")
        except Exception:
            traffic = None
    # matrix-core busy cycles from the counters (SQ_VALU_MFMA_BUSY_CYCLES over
    # 1024 SIMDs x the launch's cycles), taken on the same kernel sources
    mfma = None
    mfile = os.path.join(ROOT, "profiles", "mfma_counters.json")
    if os.path.exists(mfile):
        try:
            for e in json.load(open(mfile)):
                if match(e):
                    mfma = {"mfma_busy_frac": round(e["mfma_busy_frac"], 4), "clock_ghz": round(e["clock_ghz"], 3),
                            "counted_tflops": round(e["counted_tflops"], 1)}
                    if "padding_frac" in e:
                        mfma["padding_frac"] = round(e["padding_frac"], 4)
                        mfma["lds_bank_conflict_frac"] = round(e["lds_bank_conflict_frac"], 4)
        except Exception:
            mfma = None
    out = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": traffic, "mfma_counters": mfma,
           "kernel": name, "avg_launch_ms": round(avg_s * 1e3, 4),
           "flops_per_launch": fl * r, "operator_bytes_per_launch": byts,
           "launch_time_share": share}
    if products > 1:
        out["peak_note"] = f"{PEAK_TFLOPS[base]} TFLOP/s {base.upper()} matrix-core peak / {products:g} products per step"
    return out


def _fingerprint():
    """Hash of the sources that decide what the evaluation kernels read and
    write: the kernel templates and their instantiations, the operator
    packing, and the launch and work-item code."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1707_00164_amd", "csrc")
    for f in sorted(os.listdir(src)):
        if f == "kernels.hpp" or f.startswith("k_") or f in ("eval.hip", "pack.cpp"):
            h.update(open(os.path.join(src, f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(comp, w, pts, W64, U_gpu_rows, rows, torch, min_seconds=10.0, max_walks=6):
    """FP64 oracle tree walk of the same compression: the whole K~W (every
    row), repeated until `min_seconds` have passed (at most `max_walks`
    walks); the rate is per walk.  Returns the oracle's rows `rows` and the
    exact (K W)[rows] for the parity and error checks."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from oracle import cfile, dense, evaluate, kernels
    import tempfile
    fd, path = tempfile.mkstemp(suffix=".gofmm")
    os.close(fd)
    comp.export(path)
    c = cfile.read(path)
    os.unlink(path)
    K = kernels.KernelMatrix(pts, w.kernel, w.h, w.shift)
    walks, t, per = 0, 0.0, []
    while walks < max_walks and (walks == 0 or t < min_seconds):
        t0 = time.perf_counter()
        full = evaluate.tree_walk(c, K, W64)
        per.append(time.perf_counter() - t0)
        t += per[-1]
        walks += 1
    ref = full[rows]
    del full
    exact = dense.kw(K, W64, rows)
    threads = max([x.get("num_threads", 1) for x in threadpool_info()] + [1])
    value = 2.0 * w.n * w.n * w.r * walks / t / 1e9
    res = {
        "value": round(value, 3), "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
        "sample": f"FP64 tree walk of the whole K~W (N2S, S2S, S2N and L2L over every node, all "
                  f"{w.n} rows) of the same compression at r={w.r}, {walks} walk(s); value = "
                  f"2*N^2*r*walks / t; t = {t:.2f} s",
        "seconds": round(t, 3),
        "walk_seconds_median": round(sorted(per)[len(per) // 2], 3),
    }
    return res, ref, exact


def _timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def exact_rows(S, W, rows, block=8):
    """(K W)[rows] in FP64 from the library's own kernel sampler (not the oracle)."""
    import numpy as np
    W64 = W.cpu().numpy().astype(np.float64)
    cols = np.arange(S.n)
    return np.concatenate([S.sample(rows[k:k + block], cols) @ W64 for k in range(0, len(rows), block)])


def form_batched(args):
    """48 compressions of uneven N (log-uniform in [8192, 131072]) in one
    persistent launch per step, r in {32, 64, 128, 256}; every precision form
    in --precisions uses the same trees and skeletons."""
    import numpy as np
    import tempfile
    import torch
    import workloads
    import paper_1707_00164_amd as g
    insts = workloads.batched_instances(args.instances)
    ceil = measured_ceilings(torch)
    log(f"measured ceilings: {ceil}")
    comps, Ws, Us, Ss = [], [], [], []
    t0 = time.perf_counter()
    for w in insts:
        pts = workloads.points(w)
        S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
        Ss.append(S)
        comps.append(g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol,
                                            kappa=w.kappa, budget=w.budget, seed=w.seed))
        Ws.append(torch.from_numpy(workloads.rhs(w.n, w.r, w.seed).astype(np.float32)).cuda())
        Us.append(torch.empty_like(Ws[-1]))
    t_comp = time.perf_counter() - t0
    log(f"compressed {len(insts)} instances (sum N {sum(w.n for w in insts)}) in {t_comp:.1f} s")
    check = list(range(len(insts)))                      # every instance's error is stated
    rows = {i: workloads.sample_rows(insts[i].n, 16, insts[i].seed) for i in check}
    exact = {i: exact_rows(Ss[i], Ws[i], rows[i]) for i in check}
    flops = sum(c.stats().flops_per_rhs * W.shape[1] for c, W in zip(comps, Ws))
    dense = sum(2.0 * w.n * w.n * w.r for w in insts)
    io = sum(2 * 4 * w.n * w.r for w in insts)
    paths = []
    for c in comps:
        fd, path = tempfile.mkstemp(suffix=".gofmm")
        os.close(fd)
        c.export(path)
        paths.append(path)
    results = {}
    fp32_rows = None
    for name in args.precisions:
        if name == "bf16":
            continue                                      # not an equal-accuracy form
        prec = {"fp32": g.FP32, "bf16x3": g.BF16X3}[name]
        cs = comps if name == "fp32" else [g.Compression.load(p, S, storage=prec, near_storage=prec)
                                           for p, S in zip(paths, Ss)]
        for c, W in zip(cs, Ws):
            c.prepare(W.shape[1])
        g.evaluate_batched(cs, Ws, Us, autotune=True)
        sec = _timed(lambda: g.evaluate_batched(cs, Ws, Us), args.steps, args.warmup, torch)
        assert g.batched_status() == 0
        got = {i: Us[i].cpu().numpy()[rows[i]].astype(np.float64) for i in check}
        err = max(float(np.linalg.norm(got[i] - exact[i]) / np.linalg.norm(exact[i])) for i in check)
        if name == "fp32":
            fp32_rows = got
        seq = _timed(lambda: [c.evaluate(W, U) for c, W, U in zip(cs, Ws, Us)], args.steps, args.warmup, torch)
        opb = sum(sum(l[2] for l in c.launches()) for c in cs)   # algorithmic: each block read once
        base, products = FORM_PEAK["f32" if name == "fp32" else name]
        peak = PEAK_TFLOPS[base] / products
        t_roof = max(flops / (peak * 1e12), (opb + io) / (HBM_GBS * 1e9))
        # the same bound with the ceilings measured on this GPU (vendor GEMM of
        # the form's arithmetic, device copy bandwidth)
        peak_m = ceil["fp32_gemm_tflops"] if base == "f32" else ceil["bf16_gemm_tflops"] / products
        t_roof_m = max(flops / (peak_m * 1e12), (opb + io) / (ceil["copy_gbs"] * 1e9))
        # per phase (each launch of each instance on its own roof, then summed):
        # the bound when phases did not overlap
        t_phase = 0.0
        for c, W in zip(cs, Ws):
            r_i, n_i = W.shape[1], W.shape[0]
            for lname, fl, byts in c.launches():
                io_l = 4 * n_i * r_i * ((lname in ("n2s_leaf", "leaf", "l2l")) + (lname in ("leaf", "l2l")))
                t_phase += max(fl * r_i / (peak * 1e12), (byts + io_l) / (HBM_GBS * 1e9))
        results[name] = {
            "value": round(dense / sec / 1e9, 2), "ms_per_step": round(sec * 1e3, 4),
            "algorithmic_tflops": round(flops / sec / 1e12, 3),
            "sequential_ms_per_step": round(seq * 1e3, 4), "speedup_vs_sequential": round(seq / sec, 3),
            "eps2_vs_exact_KW_max_over_checked": err,
            "instances_with_eps2_le_1e-4": sum(
                float(np.linalg.norm(got[i] - exact[i]) / np.linalg.norm(exact[i])) <= 1e-4 for i in check),
            "eps2_per_instance": {f"{i} (N={insts[i].n}, d={insts[i].dim}, {insts[i].kernel})":
                                  float(f"{np.linalg.norm(got[i] - exact[i]) / np.linalg.norm(exact[i]):.3e}")
                                  for i in check},
            "rel_diff_vs_fp32_form": (None if name == "fp32" or fp32_rows is None else max(
                float(np.linalg.norm(got[i] - fp32_rows[i]) / np.linalg.norm(fp32_rows[i])) for i in check)),
            "roofline": {"bound": "time", "t_roof_ms": round(t_roof * 1e3, 4), "frac": round(t_roof / sec, 4),
                         "flops": flops, "bytes": opb + io, "peak_tflops": round(peak, 1),
                         "t_roof_per_phase_ms": round(t_phase * 1e3, 4), "frac_per_phase": round(t_phase / sec, 4),
                         "t_roof_measured_ms": round(t_roof_m * 1e3, 4), "frac_vs_measured": round(t_roof_m / sec, 4),
                         "measured_ceilings": ceil,
                         "note": "frac: whole job, max(flops / matrix-core peak of the form, operator + W + U "
                                 "bytes / 8 TB/s); frac_per_phase: the same bound per launch of each instance, "
                                 "summed; frac_vs_measured: the whole-job bound with the vendor GEMM and "
                                 "device-copy ceilings measured in this run"}}
        log(f"batched {name}: {sec * 1e3:.2f} ms/step ({seq / sec:.2f}x sequential), "
            f"{flops / sec / 1e12:.1f} TFLOP/s algorithmic, roofline frac {t_roof / sec:.3f} "
            f"({t_roof_m / sec:.3f} of the measured ceilings), eps2 {err:.2e}")
        for c in cs:                                      # host and device copies of this form
            c.free()
        torch.cuda.empty_cache()
    for p in paths:
        os.unlink(p)
    first = results[args.precisions[0]] if args.precisions[0] in results else next(iter(results.values()))
    out = {"metric": METRIC, "form": "batched", "value": first["value"], "unit": "GFLOP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": first["ms_per_step"],
           "higher_is_better": True, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"batched{len(insts)}_loguniform_8192_131072", "instances": len(insts),
                      "sum_n": sum(w.n for w in insts), "r": sorted({w.r for w in insts})},
           "results": results, "compress_seconds": round(t_comp, 1)}
    if "fp32" in results and "bf16x3" in results:
        out["bf16x3_speedup_vs_fp32"] = round(results["fp32"]["ms_per_step"] / results["bf16x3"]["ms_per_step"], 3)
    print(json.dumps(out), flush=True)


def form_large(args):
    """N=262144 inverse multiquadric, m = s = 512, tau 1e-6: FP32, BF16 and
    split-BF16 storage of the same structure, r = 1024 and 2048; error against
    the FP64 oracle on 64 sampled rows."""
    import numpy as np
    import tempfile
    import torch
    import workloads
    import paper_1707_00164_amd as g
    w = workloads.large_imq()
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    t0 = time.perf_counter()
    base = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol, kappa=w.kappa,
                                  budget=w.budget, seed=w.seed)
    t_comp = time.perf_counter() - t0
    st = base.stats()
    log(f"compressed N={w.n} in {t_comp:.1f} s: mean rank {st.rank_sum / (st.n_nodes - 1):.1f}, "
        f"{st.flops_per_rhs:.3e} flops per rhs, operator {st.operator_bytes / 1e9:.2f} GB")
    fd, path = tempfile.mkstemp(suffix=".gofmm")
    os.close(fd)
    base.export(path)
    rows = workloads.sample_rows(w.n, 64, w.seed)
    res = {}
    ref_rows = {}
    forms = [f for f in [("fp32", g.FP32, g.FP32), ("bf16", g.BF16, g.FP32), ("bf16x3", g.BF16X3, g.BF16X3)]
             if f[0] in args.precisions]
    for r in args.r_list:
        W = torch.from_numpy(workloads.rhs(w.n, r, w.seed).astype(np.float32)).cuda()
        U = torch.empty_like(W)
        for name, sp, sn in forms:
            c = base if name == "fp32" else g.Compression.load(path, S, storage=sp, near_storage=sn)
            c.prepare(r)
            c.autotune(W, U)
            sec, dom, dom_ms, share = time_steps(c, W, U, args.steps, args.warmup, torch)
            rl = roofline(c, dom, dom_ms, share, r, {"fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3"}[name],
                          near_form={"fp32": "f32", "bf16": "f32", "bf16x3": "bf16x3"}[name])
            res[f"{name}_r{r}"] = {"ms_per_step": round(sec * 1e3, 3),
                                   "value": round(2.0 * w.n * w.n * r / sec / 1e9, 1),
                                   "algorithmic_tflops": round(st.flops_per_rhs * r / sec / 1e12, 2),
                                   "roofline": rl, "rows": U.cpu().numpy()[rows].astype(np.float64)}
            log(f"{name} r={r}: {sec * 1e3:.2f} ms, dominant {rl['kernel']} {rl['achieved']} TFLOP/s")
            if c is not base:
                c.free()
                torch.cuda.empty_cache()
        if not args.no_cpu_baseline:
            from oracle import cfile, dense, evaluate, kernels
            cc = cfile.read(path)
            K = kernels.KernelMatrix(pts, w.kernel, w.h, w.shift)
            W64 = W.cpu().numpy().astype(np.float64)
            t1 = time.perf_counter()
            ref = evaluate.tree_walk(cc, K, W64, rows)
            t_or = time.perf_counter() - t1
            exact = dense.kw(K, W64, rows)
            for name, _, _ in forms:
                x = res[f"{name}_r{r}"]
                x["gpu_vs_oracle_same_compression"] = float(np.linalg.norm(x["rows"] - ref) / np.linalg.norm(ref))
                x["eps2_vs_exact_KW"] = float(np.linalg.norm(x["rows"] - exact) / np.linalg.norm(exact))
            res[f"oracle_r{r}_seconds"] = round(t_or, 2)
        del W, U
        torch.cuda.empty_cache()
    os.unlink(path)
    for k in list(res):
        if isinstance(res[k], dict):
            res[k].pop("rows", None)
    out = {"metric": METRIC, "form": "large", "unit": "GFLOP/s", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": w.name, "n": w.n, "leaf_size": w.leaf_size, "max_rank": w.max_rank,
                      "tol": w.tol, "budget": w.budget, "r": args.r_list},
           "compress_seconds": round(t_comp, 1), "mean_rank": st.rank_sum / (st.n_nodes - 1),
           "flops_per_rhs": st.flops_per_rhs, "operator_gb": st.operator_bytes / 1e9, "results": res}
    print(json.dumps(out), flush=True)


def form_serving(args):
    """Resident compressions (N log-spaced over 16384 .. 262144, kernels
    cycling through the three workload families), Poisson requests with r
    uniform in [1, 512]: saturation throughput, then p50/p99 latency at 50% and
    90% of it, for every precision form in --precisions (same structures).
    During the Poisson runs a fresh compression is admitted every 100
    requests under an HBM budget that holds only the resident set (plus
    1 GiB): each admission evicts one resident model, whose outstanding
    requests finish first, and the new model's requests wait until its
    footprint fits."""
    import threading
    import numpy as np
    import tempfile
    import torch
    import workloads
    import paper_1707_00164_amd as g
    ceil = measured_ceilings(torch)
    log(f"measured ceilings: {ceil}")
    ws = [w for w in workloads.serving_instances(args.models) if w.n <= args.max_n]
    n_res = len(ws)
    allw = ws + (workloads.serving_admissions(args.admissions) if args.admissions > 0 else [])
    base, samplers = [], []
    t0 = time.perf_counter()
    for w in allw:
        pts = workloads.points(w)
        S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
        samplers.append(S)
        base.append(g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol,
                                           kappa=w.kappa, budget=w.budget, seed=w.seed))
    t_comp = time.perf_counter() - t0
    log(f"compressed {n_res} resident and {len(allw) - n_res} admitted models in {t_comp:.1f} s")
    paths = []
    for c in base:
        fd, path = tempfile.mkstemp(suffix=".gofmm")
        os.close(fd)
        c.export(path)
        paths.append(path)
    rmax = 512
    rng = np.random.default_rng(7)
    pool = {}
    for i, w in enumerate(allw):     # a few resident input blocks per model
        pool[i] = [torch.from_numpy(workloads.rhs(w.n, rmax, w.seed + k).astype(np.float32)).cuda()
                   for k in range(2)]
    torch.cuda.synchronize()
    # accuracy of every model: 16 sampled rows of a 16-column product
    acc_rows = {i: workloads.sample_rows(w.n, 16, w.seed + 3) for i, w in enumerate(allw)}
    acc_exact = {i: exact_rows(samplers[i], pool[i][0][:, :16], acc_rows[i]) for i in range(len(allw))}
    results = {}
    for name in args.precisions:
        if name == "bf16":
            continue                                      # not an equal-accuracy form
        prec = {"fp32": g.FP32, "bf16x3": g.BF16X3}[name]
        comps = base if name == "fp32" else [g.Compression.load(p, S, storage=prec, near_storage=prec)
                                             for p, S in zip(paths, samplers)]
        eps = []
        for i, c in enumerate(comps):
            u = c.evaluate(pool[i][0][:, :16].contiguous()).cpu().numpy()[acc_rows[i]].astype(np.float64)
            eps.append(float(np.linalg.norm(u - acc_exact[i]) / np.linalg.norm(acc_exact[i])))
        fl_rhs = [c.stats().flops_per_rhs for c in comps]
        op_bytes = [sum(l[2] for l in c.launches()) for c in comps]
        foot = [c.footprint(rmax) + 2 * c.n * rmax * 4 for c in comps]
        base_peak, products = FORM_PEAK["f32" if name == "fp32" else name]
        peak = PEAK_TFLOPS[base_peak] / products
        need = sum(foot[:n_res])
        if need + (1 << 30) > args.hbm_gb << 30:
            raise SystemExit(f"{name}: the models need {need / 2 ** 30:.1f} GiB of HBM, over --hbm-gb")
        budget = need + (1 << 30)
        srv = g.Server(hbm_budget_bytes=budget, streams=args.streams, max_batch=n_res)
        ids = {i: srv.add(comps[i], rmax) for i in range(n_res)}
        log(f"{name}: {n_res} models resident, {need / 2 ** 30:.1f} GiB")

        def run(n_req, qps, admit=False):
            srv.reset_stats()
            live = list(range(n_res))
            handles = {}                  # model -> [(request, U)] the main thread waits for
            F, io, used = 0.0, 0.0, set()
            nxt = n_res
            admissions, threads, first, errors = [], [], {}, []
            t_next = time.perf_counter()
            for q in range(n_req):
                if admit and q % 100 == 50 and nxt < len(allw):
                    k, nxt = nxt, nxt + 1
                    ids[k] = srv.add(comps[k], rmax)       # queued until its footprint fits
                    res_live = [i for i in live if i < n_res]
                    fit = [i for i in res_live if foot[i] >= foot[k]]
                    victim = min(fit, key=lambda i: foot[i]) if fit else max(res_live, key=lambda i: foot[i])
                    live.remove(victim)
                    live.append(k)
                    mine = handles.pop(victim, [])

                    def evict(v=victim, hs=mine):
                        try:
                            for h, _ in hs:
                                srv.wait(h, timeout_ms=120000)
                            srv.remove(ids[v])
                        except Exception as e:             # reported after the run
                            errors.append(e)
                    th = threading.Thread(target=evict)
                    th.start()
                    threads.append(th)
                    admissions.append({"at_request": q, "admitted": allw[k].name,
                                       "footprint_gib": round(foot[k] / 2 ** 30, 2),
                                       "evicted": allw[victim].name})
                i = live[int(rng.integers(0, len(live)))]
                r = int(rng.integers(1, rmax + 1))
                F += fl_rhs[i] * r
                io += 8.0 * allw[i].n * r
                used.add(i)
                W = pool[i][q % 2][:, :r]
                U = torch.empty((allw[i].n, r), device="cuda")
                if qps:
                    t_next += rng.exponential(1.0 / qps)
                    while time.perf_counter() < t_next:
                        pass
                h = srv.submit(ids[i], W, U)
                if i >= n_res and i not in first:
                    first[i] = h
                handles.setdefault(i, []).append((h, U))
            first_ms = {}
            for i, lst in handles.items():
                for h, _ in lst:
                    ms = srv.wait(h, timeout_ms=120000)
                    if first.get(i) == h:
                        first_ms[allw[i].name] = round(ms, 2)
            for th in threads:
                th.join()
            if errors:
                raise errors[0]
            st = srv.stats()
            sec = st.elapsed_ms / 1e3
            # lower bound on the time of this request mix: every flop at the
            # form's matrix-core peak, or every model used read once plus W and U
            t_roof = max(F / (peak * 1e12), (sum(op_bytes[i] for i in used) + io) / (HBM_GBS * 1e9))
            peak_m = ceil["fp32_gemm_tflops"] if base_peak == "f32" else ceil["bf16_gemm_tflops"] / products
            t_roof_m = max(F / (peak_m * 1e12), (sum(op_bytes[i] for i in used) + io) / (ceil["copy_gbs"] * 1e9))
            out = {"requests": n_req, "qps_offered": round(qps, 1) if qps else None,
                   "throughput_rps": round(st.completed / sec, 1),
                   "columns_per_s": round(st.columns / sec, 1),
                   "p50_ms": round(st.p50_ms, 3), "p99_ms": round(st.p99_ms, 3), "mean_ms": round(st.mean_ms, 3),
                   "batches": st.batches, "failed": st.failed, "most_batches_in_flight": st.max_inflight,
                   "host_ms_per_batch": round(st.host_ms_mean, 3), "admissions_done": st.admissions,
                   "admission_ms_mean": round(st.admit_ms_mean, 1),
                   "p99_ms_while_admitting": round(st.p99_ms_admitting, 3),
                   "algorithmic_tflops": round(F / sec / 1e12, 3),
                   "roofline": {"bound": "time", "t_roof_ms": round(t_roof * 1e3, 3),
                                "frac": round(t_roof / sec, 4), "peak_tflops": round(peak, 1),
                                "t_roof_measured_ms": round(t_roof_m * 1e3, 3),
                                "frac_vs_measured": round(t_roof_m / sec, 4)}}
            if admissions:
                out["admissions"] = admissions
                out["first_request_ms_of_admitted"] = first_ms
                # back to the resident set for the next run
                for k in range(n_res, nxt):
                    srv.remove(ids.pop(k))
                back = [a for a in range(n_res) if a not in live]
                for v in back:
                    ids[v] = srv.add(comps[v], rmax)
                for v in back:                             # wait until resident again
                    srv.wait(srv.submit(ids[v], pool[v][0][:, :1], torch.empty((allw[v].n, 1), device="cuda")),
                             timeout_ms=120000)
            return out
        run(64, 0)                                 # warm-up
        sat = run(args.requests, 0)                # burst: saturation throughput
        res = {"hbm_budget_gb": round(budget / 2 ** 30, 1), "eps2_vs_exact_KW_max": max(eps[:n_res]),
               "eps2_vs_exact_KW_per_model": [float(f"{e:.3e}") for e in eps[:n_res]],
               "eps2_vs_exact_KW_admitted": [float(f"{e:.3e}") for e in eps[n_res:]],
               "saturation": sat}
        log(f"{name} saturation: {sat}")
        for frac in (0.5, 0.9):
            res[f"poisson_{int(frac * 100)}pct"] = run(args.requests, frac * sat["throughput_rps"], admit=True)
            log(f"{name} poisson {frac}: {res[f'poisson_{int(frac * 100)}pct']}")
        srv.close()
        results[name] = res
        if comps is not base:
            for c in comps:
                c.free()
        torch.cuda.empty_cache()
    for p in paths:
        os.unlink(p)
    out = {"metric": METRIC, "form": "serving", "unit": "ms", "n_gpus": 1, "data": "synthetic",
           "config": {"models": n_res, "n": [w.n for w in ws], "r": "uniform 1..512", "streams": args.streams,
                      "admitted_during_poisson_runs": [w.name for w in allw[n_res:]]},
           "compress_seconds": round(t_comp, 1), "results": results}
    print(json.dumps(out), flush=True)


def form_sweep(args):
    """Accuracy against time over the method's knobs (the analogue of the
    paper's HSS-versus-FMM and distance studies, Sec. 4): the N=65536
    clustered Gaussian at r=512 compressed with near budget 0 (HSS), 1%, 3%
    and 10%, maximum rank 64, 128 and 256, and the Gram-l2 and Gram-angle
    distances; each compression evaluated autotuned in FP32 and split BF16,
    error against the exact K W on 64 sampled rows."""
    import numpy as np
    import tempfile
    import torch
    import workloads
    import paper_1707_00164_amd as g
    w = workloads.clustered_gaussian()
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    W = torch.from_numpy(workloads.rhs(w.n, w.r, w.seed).astype(np.float32)).cuda()
    U = torch.empty_like(W)
    rows = workloads.sample_rows(w.n, 64, w.seed)
    exact = exact_rows(S, W, rows)
    res = []
    for dist_name, dist in (("gram_l2", g.GRAM_L2), ("angle", g.ANGLE)):
        for budget in (0.0, 0.01, 0.03, 0.10):
            for s_max in (64, 128, 256):
                t0 = time.perf_counter()
                comp = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=s_max, tol=w.tol,
                                              kappa=w.kappa, budget=budget, distance=dist, seed=w.seed)
                t_comp = time.perf_counter() - t0
                st = comp.stats()
                fd, path = tempfile.mkstemp(suffix=".gofmm")
                os.close(fd)
                comp.export(path)
                item = {"distance": dist_name, "budget": budget, "max_rank": s_max,
                        "compress_s": round(t_comp, 2), "mean_rank": round(st.rank_sum / (st.n_nodes - 1), 1),
                        "near_pairs": st.near_pairs, "far_pairs": st.far_pairs,
                        "flops_per_step": st.flops_per_rhs * w.r}
                for name, prec in (("fp32", g.FP32), ("bf16x3", g.BF16X3)):
                    c = comp if name == "fp32" else g.Compression.load(path, S, storage=prec, near_storage=prec)
                    c.autotune(W, U)
                    sec = _timed(lambda: c.evaluate(W, U), args.steps, args.warmup, torch)
                    got = U.cpu().numpy()[rows].astype(np.float64)
                    item[name] = {"ms_per_step": round(sec * 1e3, 4),
                                  "value": round(2.0 * w.n * w.n * w.r / sec / 1e9, 1),
                                  "eps2_vs_exact_KW": float(f"{np.linalg.norm(got - exact) / np.linalg.norm(exact):.3e}"),
                                  "operator_gb": round(c.stats().operator_bytes / 1e9, 3)}
                    c.free()
                os.unlink(path)
                torch.cuda.empty_cache()
                res.append(item)
                log(f"{dist_name} budget {budget:.2f} s {s_max}: rank {item['mean_rank']}, fp32 "
                    f"{item['fp32']['ms_per_step']} ms eps {item['fp32']['eps2_vs_exact_KW']:.2e}, bf16x3 "
                    f"{item['bf16x3']['ms_per_step']} ms eps {item['bf16x3']['eps2_vs_exact_KW']:.2e}")
    out = {"metric": METRIC, "form": "sweep", "unit": "ms", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": w.name, "n": w.n, "r": w.r, "leaf_size": w.leaf_size, "tol": w.tol,
                      "kappa": w.kappa}, "results": res}
    print(json.dumps(out), flush=True)


def form_copy(args):
    """A device-to-device copy of exactly 1 GiB (counter calibration: the
    traffic counters of this copy should read 1 GiB fetched, 1 GiB written)."""
    import torch
    x = torch.ones(1 << 28, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"form": "copy", "bytes": 4 << 28, "copies": 3}), flush=True)


def form_flat(args):
    """The N=65536 clustered-Gaussian workload alone (r = 512): FP32, split
    BF16 and near blocks from the points, with the CPU baseline of the whole
    K~W (the form the counter and trace summaries of the N=65536 kernels
    were taken with)."""
    import numpy as np
    import torch
    import workloads
    import paper_1707_00164_amd as g
    w = workloads.clustered_gaussian()
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    t0 = time.perf_counter()
    comp = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol,
                                  kappa=w.kappa, budget=w.budget, seed=w.seed)
    t_comp = time.perf_counter() - t0
    st = comp.stats()
    log(f"compressed N={w.n} in {t_comp:.1f} s: depth {st.depth}, mean rank "
        f"{st.rank_sum / max(1, st.n_nodes - 1):.1f}, max {st.rank_max}, near pairs {st.near_pairs}, "
        f"far pairs {st.far_pairs}, {st.flops_per_rhs * w.r:.3e} flops/step")

    W64 = workloads.rhs(w.n, w.r, w.seed)
    W = torch.from_numpy(W64.astype(np.float32)).cuda()
    U = torch.empty_like(W)
    comp.prepare(w.r)
    if not args.no_autotune:
        comp.autotune(W, U)
    torch.cuda.synchronize()
    sec, dom, dom_ms, share = time_steps(comp, W, U, args.steps, args.warmup, torch)
    value = 2.0 * w.n * w.n * w.r / sec / 1e9
    rl = roofline(comp, dom, dom_ms, share, w.r, "f32", workload=f"gauss6d_n65536_r{w.r}")
    alg_tflops = st.flops_per_rhs * w.r / sec / 1e12
    log(f"fp32: {sec * 1e3:.3f} ms/step, effective {value:.1f} GFLOP/s, algorithmic "
        f"{alg_tflops:.2f} TFLOP/s; dominant {rl['kernel']} {rl['achieved']} TFLOP/s "
        f"({100 * rl['frac']:.1f}% of FP32 MFMA peak)")

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4),
        "ms_per_step_median": round(time_steps.median_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded clustered 6-D points; the paper's matrices are not available)",
        "config": {"workload": w.name, "n": w.n, "r": w.r, "dim": w.dim, "kernel": w.kernel,
                   "h": w.h, "shift": w.shift, "leaf_size": w.leaf_size, "max_rank": w.max_rank,
                   "tol": w.tol, "kappa": w.kappa, "budget": w.budget, "storage": "fp32",
                   "parallelism": "single GPU"},
        "algorithmic_tflops": round(alg_tflops, 3),
        "flops_per_step": st.flops_per_rhs * w.r,
        "compress_seconds": round(t_comp, 2),
        "roofline": rl,
    }

    rows = workloads.sample_rows(w.n, args.rows, w.seed)
    U_rows = U.cpu().numpy()[rows].astype(np.float64)

    mixed = None
    if not args.no_mixed:
        comp3 = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol,
                                       kappa=w.kappa, budget=w.budget, seed=w.seed,
                                       storage=g.BF16X3, near_storage=g.BF16X3)
        st3 = comp3.stats()
        assert st3.rank_sum == st.rank_sum and st3.far_pairs == st.far_pairs
        U3 = torch.empty_like(W)
        comp3.prepare(w.r)
        if not args.no_autotune:
            comp3.autotune(W, U3)
        sec3, dom3, dom3_ms, share3 = time_steps(comp3, W, U3, args.steps, args.warmup, torch)
        rl3 = roofline(comp3, dom3, dom3_ms, share3, w.r, "bf16x3", workload=f"gauss6d_n65536_r{w.r}")
        mixed = {"storage": "bf16x3 (split BF16, 3 BF16 matrix-core products per step)",
                 "value": round(2.0 * w.n * w.n * w.r / sec3 / 1e9, 2), "unit": "GFLOP/s",
                 "ms_per_step": round(sec3 * 1e3, 4), "ms_per_step_median": round(time_steps.median_ms, 4),
                 "speedup_vs_fp32": round(sec / sec3, 3),
                 "roofline": rl3}
        U3_rows = U3.cpu().numpy()[rows].astype(np.float64)
        log(f"bf16x3: {sec3 * 1e3:.3f} ms/step ({sec / sec3:.2f}x fp32)")
        out["mixed_precision"] = mixed

    geo = None
    if not args.no_geometric:
        # the same structure with the near blocks computed on the device from
        # the points instead of stored
        compg = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol,
                                       kappa=w.kappa, budget=w.budget, seed=w.seed)
        compg.use_device_kernel(S)
        stg = compg.stats()
        Ug = torch.empty_like(W)
        compg.prepare(w.r)
        if not args.no_autotune:
            compg.autotune(W, Ug)
        secg, domg, domg_ms, shareg = time_steps(compg, W, Ug, args.steps, args.warmup, torch)
        rlg = roofline(compg, domg, domg_ms, shareg, w.r, "f32")
        geo = {"near_blocks": "computed on the device from the points (FP32), not stored",
               "value": round(2.0 * w.n * w.n * w.r / secg / 1e9, 2), "unit": "GFLOP/s",
               "ms_per_step": round(secg * 1e3, 4), "ms_per_step_median": round(time_steps.median_ms, 4),
               "speedup_vs_stored_fp32": round(sec / secg, 3),
               "operator_bytes": stg.operator_bytes, "operator_bytes_stored_fp32": st.operator_bytes,
               "roofline": rlg}
        Ug_rows = Ug.cpu().numpy()[rows].astype(np.float64)
        log(f"geometric: {secg * 1e3:.3f} ms/step ({sec / secg:.2f}x stored fp32), operator "
            f"{stg.operator_bytes / 1e9:.2f} GB (stored {st.operator_bytes / 1e9:.2f} GB)")
        out["geometric"] = geo

    if not args.no_cpu_baseline:
        cb, ref, exact = cpu_baseline(comp, w, pts, W.cpu().numpy().astype(np.float64), U_rows, rows, torch)
        out["cpu_baseline"] = cb
        err = float(np.linalg.norm(U_rows - ref) / np.linalg.norm(ref))
        eps = float(np.linalg.norm(U_rows - exact) / np.linalg.norm(exact))
        out["accuracy"] = {"rows": len(rows), "gpu_vs_oracle_same_compression": err,
                           "eps2_vs_exact_KW": eps}
        if mixed is not None:
            out["mixed_precision"]["gpu_vs_oracle_same_compression"] = float(
                np.linalg.norm(U3_rows - ref) / np.linalg.norm(ref))
            out["mixed_precision"]["eps2_vs_exact_KW"] = float(
                np.linalg.norm(U3_rows - exact) / np.linalg.norm(exact))
        if geo is not None:
            geo["gpu_vs_oracle_same_compression"] = float(np.linalg.norm(Ug_rows - ref) / np.linalg.norm(ref))
            geo["eps2_vs_exact_KW"] = float(np.linalg.norm(Ug_rows - exact) / np.linalg.norm(exact))
        log(f"cpu oracle: {cb['value']} GFLOP/s on {cb['cores']} threads; parity {err:.2e}, eps2 {eps:.2e}")
    print(json.dumps(out), flush=True)



# ---------------------------------------------------------------- headline form
def measured_ceilings(torch):
    """Ceilings measured on this GPU: vendor GEMM (torch.matmul, 8192^3) in
    FP32 and BF16, and the bandwidth of a 4 GiB device-to-device copy."""
    out = {}
    n = 8192
    for key, dt in (("fp32_gemm_tflops", torch.float32), ("bf16_gemm_tflops", torch.bfloat16)):
        a = torch.randn(n, n, device="cuda", dtype=dt)
        b = torch.randn(n, n, device="cuda", dtype=dt)
        for _ in range(3):
            c = torch.matmul(a, b)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            c = torch.matmul(a, b)
        e1.record()
        torch.cuda.synchronize()
        out[key] = round(2.0 * n ** 3 * 10 / (e0.elapsed_time(e1) / 1e3) / 1e12, 1)
        del a, b, c
    x = torch.ones(1 << 30, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    out["copy_gbs"] = round(2.0 * 4 * (1 << 30) * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9, 1)
    del x, y
    torch.cuda.empty_cache()
    return out


def with_ceiling(rl, ceil, form):
    """Adds the fraction of the measured ceiling of the form's arithmetic."""
    if ceil:
        base, products = FORM_PEAK[form if not (rl["kernel"] == "l2l" and rl.get("near_form")) else rl["near_form"]]
        v = ceil["fp32_gemm_tflops"] if base == "f32" else ceil["bf16_gemm_tflops"] / products
        rl["measured_ceiling"] = {"tflops": round(v, 1), "what": "torch.matmul 8192^3 on this GPU"
                                  + ("" if products == 1 else f" / {products:g} products")}
        rl["frac_vs_measured"] = round(rl["achieved"] / v, 4)
    return rl


def run_form(comp, W, U, args, torch, form, near_form=None, ceil=None, autotune=True, workload=None):
    """Autotune, then time `args.steps` evaluates after `args.warmup`: ms per
    step (wall clock), per-step median (HIP events) and the roofline of the
    dominant launch."""
    r = W.shape[1]
    comp.prepare(r)
    if autotune and not args.no_autotune:
        comp.autotune(W, U)
    torch.cuda.synchronize()
    sec, dom, dom_ms, share = time_steps(comp, W, U, args.steps, args.warmup, torch)
    rl = roofline(comp, dom, dom_ms, share, r, form, near_form=near_form, workload=workload)
    if near_form is not None and near_form != form:
        rl["near_form"] = near_form
    rl = with_ceiling(rl, ceil, form)
    st = comp.stats()
    n = st.n
    return {"value": round(2.0 * n * n * r / sec / 1e9, 2), "unit": "GFLOP/s",
            "ms_per_step": round(sec * 1e3, 4), "ms_per_step_median": round(time_steps.median_ms, 4),
            "algorithmic_tflops": round(st.flops_per_rhs * r / sec / 1e12, 3),
            "flops_per_step": st.flops_per_rhs * r, "roofline": rl}


def sample_flops(c, rows, r):
    """Table 2 flops of the oracle's walk restricted to `rows`: the whole
    upward pass, then S2S, S2N and L2L on the leaves holding the rows and the
    nodes above them."""
    import numpy as np
    from oracle import cfile
    fl = cfile.first_leaf(c.depth)
    pos_of = np.empty(c.n, dtype=np.int64)
    pos_of[c.perm] = np.arange(c.n)
    leaves = set((np.searchsorted(c.node_start[fl:], pos_of[rows], side="right") - 1).tolist())
    want = set()
    for b in leaves:
        x = fl + b
        while x > 0:
            want.add(x)
            x = (x - 1) // 2
    f = 0.0
    for h in range(1, c.nn):
        s = c.rank(h)
        ncol = int(c.node_size[h]) if h >= fl else c.rank(2 * h + 1) + c.rank(2 * h + 2)
        f += 2.0 * s * ncol * r * (2 if h in want else 1)           # N2S, and S2N where wanted
        if h in want:
            f += sum(2.0 * s * c.rank(int(a)) * r for a in c.far[h])
    for b in leaves:
        f += sum(2.0 * int(c.node_size[fl + b]) * int(c.node_size[int(a)]) * r for a in c.near[b])
    return f


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_rows(c, K, W64, rows, n, sample_desc):
    """The FP64 oracle's walk of the same compression restricted to `rows`
    (the whole upward pass, then S2S, S2N and L2L on the rows' leaves and the
    nodes above them), timed once on the host's BLAS threads, then on one
    thread over a smaller sample (8 rows, 256 right-hand sides).  The rate is
    scaled to the metric's unit: the whole K~W's Table 2 flops over the
    sample's, times the sample's time, is the time of a whole walk at that
    rate; value = 2 N^2 r / that time.  Returns (baseline, oracle rows)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import evaluate
    r = W64.shape[1]
    threads = max([x.get("num_threads", 1) for x in threadpool_info()] + [1])
    full = evaluate.algorithmic_flops(c, r)
    t0 = time.perf_counter()
    ref = evaluate.tree_walk(c, K, W64, rows)
    t = time.perf_counter() - t0
    fs = sample_flops(c, rows, r)
    res = {"value": round(2.0 * n * n * r / (t * full / fs) / 1e9, 3), "unit": "GFLOP/s", "cores": int(threads),
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"FP64 tree walk of the same compression for {len(rows)} sampled rows at r={r} "
                     f"({sample_desc}): the whole upward pass plus S2S, S2N and L2L on the rows' leaves and "
                     f"the nodes above them, {fs:.3e} Table 2 flops of the whole K~W's {full:.3e}, "
                     f"in {t:.2f} s; value = 2 N^2 r / (t * whole flops / sample flops)",
           "seconds": round(t, 3), "algorithmic_gflops": round(fs / t / 1e9, 2)}
    rows1, r1 = rows[:8], min(r, 256)
    W1 = W64[:, :r1].copy()
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        evaluate.tree_walk(c, K, W1, rows1)
        t1 = time.perf_counter() - t0
    fs1, full1 = sample_flops(c, rows1, r1), evaluate.algorithmic_flops(c, r1)
    res["one_thread"] = {"value": round(2.0 * n * n * r1 / (t1 * full1 / fs1) / 1e9, 3), "cores": 1,
                         "sample": f"{len(rows1)} rows at r={r1}: {fs1:.3e} of {full1:.3e} flops in {t1:.2f} s",
                         "seconds": round(t1, 3), "algorithmic_gflops": round(fs1 / t1 / 1e9, 2)}
    return res, ref


def form_headline(args):
    """The default line: the N=262144 inverse-multiquadric workload at r=2048
    in FP32 (the headline), then the same structure with BF16 P and coupling
    blocks (near FP32) and with split BF16 everywhere, then the N=65536
    clustered Gaussian at r=512 (FP32 and split BF16) as a secondary block;
    accuracy of every form on sampled rows against the FP64 oracle and the
    exact K W; the CPU baseline on the oracle's row-sampled walk."""
    import tempfile
    import numpy as np
    import torch
    import workloads
    import paper_1707_00164_amd as g
    from oracle import cfile, dense, kernels

    ceil = measured_ceilings(torch)
    log(f"measured ceilings: {ceil}")
    w = workloads.large_imq(r=args.r)
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    t0 = time.perf_counter()
    # neighbour merges and interpolative decompositions on the device: the
    # same compression as the host's, bit for bit, in less time
    base = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol, kappa=w.kappa,
                                  budget=w.budget, seed=w.seed, device_knn=1, device_id=1)
    t_comp = time.perf_counter() - t0
    st = base.stats()
    log(f"compressed N={w.n} in {t_comp:.1f} s (device neighbour merges and decompositions): depth {st.depth}, mean rank "
        f"{st.rank_sum / max(1, st.n_nodes - 1):.1f}, near pairs {st.near_pairs}, far pairs {st.far_pairs}, "
        f"{st.flops_per_rhs * w.r:.3e} flops/step, operator {st.operator_bytes / 1e9:.1f} GB")
    fd, path = tempfile.mkstemp(suffix=".gofmm")
    os.close(fd)
    base.export(path)
    rows = workloads.sample_rows(w.n, 64, w.seed)
    W = torch.from_numpy(workloads.rhs(w.n, w.r, w.seed).astype(np.float32)).cuda()
    U = torch.empty_like(W)
    wl = f"imq4d_n262144_r{w.r}"
    head = run_form(base, W, U, args, torch, "f32", ceil=ceil, workload=wl)
    got = {"fp32": U.cpu().numpy()[rows].astype(np.float64)}
    log(f"fp32: {head['ms_per_step']:.2f} ms/step, effective {head['value']:.1f} GFLOP/s; dominant "
        f"{head['roofline']['kernel']} {head['roofline']['achieved']} TFLOP/s "
        f"({100 * head['roofline']['frac']:.1f}% of {head['roofline']['peak']})")
    base.free()
    del base
    torch.cuda.empty_cache()
    forms = {}
    for name, sp, sn, f, nf in (("bf16", g.BF16, g.FP32, "bf16", "f32"),
                                ("bf16x3", g.BF16X3, g.BF16X3, "bf16x3", "bf16x3")):
        if name not in args.precisions:
            continue
        cc = g.Compression.load(path, S, storage=sp, near_storage=sn)
        res = run_form(cc, W, U, args, torch, f, near_form=nf, ceil=ceil, workload=wl)
        res["storage"] = {"bf16": "P and coupling blocks BF16 (right-hand operands rounded to BF16), near "
                                  "blocks FP32",
                          "bf16x3": "split BF16 everywhere (x = hi + lo; 3 BF16 matrix-core products per step)"}[name]
        res["speedup_vs_fp32"] = round(head["ms_per_step"] / res["ms_per_step"], 3)
        got[name] = U.cpu().numpy()[rows].astype(np.float64)
        forms[name] = res
        log(f"{name}: {res['ms_per_step']:.2f} ms/step ({res['speedup_vs_fp32']:.2f}x fp32); dominant "
            f"{res['roofline']['kernel']} {res['roofline']['achieved']} TFLOP/s")
        cc.free()
        del cc
        torch.cuda.empty_cache()
    W64 = W.cpu().numpy().astype(np.float64)
    del W, U
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": head["value"], "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "ms_per_step_median": head["ms_per_step_median"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded uniform 4-D points; the paper's matrices are not available)",
        "config": {"workload": wl, "n": w.n, "r": w.r, "dim": w.dim, "kernel": w.kernel,
                   "h": w.h, "shift": w.shift, "leaf_size": w.leaf_size, "max_rank": w.max_rank, "tol": w.tol,
                   "kappa": w.kappa, "budget": w.budget, "storage": "fp32", "parallelism": "single GPU"},
        "algorithmic_tflops": head["algorithmic_tflops"], "flops_per_step": head["flops_per_step"],
        "compress_seconds": round(t_comp, 2), "compress_on_device": ["neighbour merges", "decompositions"],
        "roofline": head["roofline"],
        "precision_forms": forms, "measured_ceilings": ceil,
    }

    if not args.no_secondary:
        out["secondary"] = secondary_block(args, torch, ceil)

    c = cfile.read(path)
    os.unlink(path)
    K = kernels.KernelMatrix(pts, w.kernel, w.h, w.shift)
    if not args.no_cpu_baseline:
        cb, ref = cpu_baseline_rows(c, K, W64, rows, w.n, f"N={w.n}, r={w.r}")
        out["cpu_baseline"] = cb
        log(f"cpu oracle: {cb['value']} GFLOP/s equivalent on {cb['cores']} threads "
            f"({cb['algorithmic_gflops']} GFLOP/s algorithmic); one thread {cb['one_thread']['value']}")
        exact = dense.kw(K, W64, rows)
        acc = {"rows": len(rows)}
        for name, v in got.items():
            acc[name] = {"gpu_vs_oracle_same_compression": float(np.linalg.norm(v - ref) / np.linalg.norm(ref)),
                         "eps2_vs_exact_KW": float(np.linalg.norm(v - exact) / np.linalg.norm(exact))}
        out["accuracy"] = acc
        log(f"accuracy on {len(rows)} rows: {acc}")
    print(json.dumps(out), flush=True)


def secondary_block(args, torch, ceil):
    """The N=65536 clustered Gaussian at r=512 in FP32 and split BF16."""
    import numpy as np
    import workloads
    import paper_1707_00164_amd as g
    w = workloads.clustered_gaussian()
    pts = workloads.points(w)
    S = g.KernelSampler(pts, w.kernel, w.h, w.shift)
    W = torch.from_numpy(workloads.rhs(w.n, w.r, w.seed).astype(np.float32)).cuda()
    U = torch.empty_like(W)
    res = {"workload": f"gauss6d_n65536_r{w.r}", "n": w.n, "r": w.r}
    for name, prec, f in (("fp32", g.FP32, "f32"), ("bf16x3", g.BF16X3, "bf16x3")):
        cc = g.Compression.compress(S, leaf_size=w.leaf_size, max_rank=w.max_rank, tol=w.tol, kappa=w.kappa,
                                    budget=w.budget, seed=w.seed, storage=prec, near_storage=prec)
        res[name] = run_form(cc, W, U, args, torch, f, ceil=ceil, workload=res["workload"])
        log(f"secondary {name}: {res[name]['ms_per_step']:.3f} ms/step, dominant "
            f"{res[name]['roofline']['kernel']} {res[name]['roofline']['achieved']} TFLOP/s")
        cc.free()
    res["bf16x3"]["speedup_vs_fp32"] = round(res["fp32"]["ms_per_step"] / res["bf16x3"]["ms_per_step"], 3)
    del W, U
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-geometric", action="store_true", help="flat form: skip the near-blocks-from-points form")
    ap.add_argument("--no-secondary", action="store_true", help="headline form: skip the N=65536 block")
    ap.add_argument("--r", type=int, default=2048, help="headline form: right-hand sides")
    ap.add_argument("--rows", type=int, default=256, help="rows compared with the oracle and with exact K W")
    ap.add_argument("--form", default="headline",
                    choices=["headline", "flat", "batched", "serving", "large", "sweep", "copy"],
                    help="headline: N=262144 at r=2048 in FP32 with BF16 and split-BF16 forms and the "
                         "N=65536 workload as a secondary block (default); flat: the N=65536 workload alone; "
                         "batched: 48 compressions in one launch; serving: request loop with p50/p99; "
                         "large: N=262144 over several r; sweep: accuracy and time over budget, rank and "
                         "distance")
    ap.add_argument("--instances", type=int, default=48, help="batched form: compressions")
    ap.add_argument("--models", type=int, default=16, help="serving form: resident compressions")
    ap.add_argument("--admissions", type=int, default=4, help="serving form: compressions admitted per Poisson run")
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--streams", type=int, default=2)
    ap.add_argument("--hbm-gb", type=int, default=240)
    ap.add_argument("--max-n", type=int, default=262144)
    ap.add_argument("--r-list", type=int, nargs="+", default=[1024, 2048])
    ap.add_argument("--precisions", nargs="+", default=["fp32", "bf16", "bf16x3"])
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only: the evaluator has no "
                                   "multi-GPU path (it would shard by subtrees, with one exchange of "
                                   "skeleton weights and near-field W rows after the upward pass)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1707_00164_amd as g

    assert torch.cuda.is_available(), "no GPU"
    g.lib()
    {"headline": form_headline, "flat": form_flat, "batched": form_batched, "serving": form_serving,
     "large": form_large, "sweep": form_sweep, "copy": form_copy}[args.form](args)


if __name__ == "__main__":
    main()
