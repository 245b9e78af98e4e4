#!/usr/bin/env python3
"""Benchmark of the b-tree hot path on one MI355X.

One step = BuildTree (btree_rebuild) + FindNeighbors pass 1 (counts,
offsets) + pass 2 (CSR lists) over the workload, inputs resident in HBM.
Prints one JSON line.  `value` is particles per second of whole steps.

  python bench.py [--steps K] [--warmup W] [--workload P8M] [--precision fp32]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Non-packed FP32 VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane-ops of one FP32-filter pair test: 3 sub, 1 mul, 2 fma, 2 compare.
OPS_PER_TEST_F32 = 8
# ... and of one FP64 pair test: 3 sub, 3 mul, 2 add, 1 compare.
OPS_PER_TEST_F64 = 9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="P8M", choices=["U10k", "L1M", "P8M", "P16M"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--bucket", type=int, default=0, help="bucket size s (0 = workload default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain-FP64 comparison")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def kernel_hash():
    h = hashlib.sha256()
    for f in ("find.hip", "common.h", "prim.h"):
        with open(os.path.join(ROOT, "paper_1910_02639_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/), or
    None when absent or taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(kernel, {}).get(workload)
        if e and e.get("source_hash") == kernel_hash():
            return e["bytes_per_launch"]
    except Exception:
        return None
    return None


def run_steps(t, dx, dy, dz, dh, counts, offsets, nbrs, k):
    for _ in range(k):
        t.rebuild(dx, dy, dz)
        t.count(dh, counts, offsets)
        t.fill(dh, counts, offsets, nbrs)


def timed(t, dx, dy, dz, dh, counts, offsets, nbrs, steps, warmup):
    import torch
    run_steps(t, dx, dy, dz, dh, counts, offsets, nbrs, warmup)
    torch.cuda.synchronize()
    s0 = t.stats()
    t0 = time.perf_counter()
    run_steps(t, dx, dy, dz, dh, counts, offsets, nbrs, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = t.stats()
    ph = {k: (s1["phase_ms"][k] - s0["phase_ms"][k]) /
          max(1, s1["phase_calls"][k] - s0["phase_calls"][k]) for k in s1["phase_ms"]}
    return t1 - t0, ph, s1


def cpu_baseline(x, y, z, h, budget_s):
    """The oracle (brute-force FP64 rows) on a bounded sample of the same
    workload: rows drawn at random, particles/s = rows / wall time."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    rng = np.random.default_rng(12345)
    n = len(x)
    probe = rng.integers(0, n, 32)
    t0 = time.perf_counter()
    oracle.counts(x, y, z, h, probe)
    dt = time.perf_counter() - t0
    m = int(max(32, min(n, 32 * budget_s / max(dt, 1e-6))))
    rows = rng.integers(0, n, m)
    t0 = time.perf_counter()
    oracle.counts(x, y, z, h, rows)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    return {"value": m / dt, "unit": "particles/s", "cores": cores, "kind": "oracle",
            "sample": "%d random rows of the %d-particle workload, each tested against all "
                      "%d particles (%.1f s)" % (m, n, n, dt)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1910_02639_amd import btree, workloads

    x, y, z, h, s = workloads.make(a.workload)
    if a.bucket:
        s = a.bucket
    n = len(x)
    dev = "cuda:0"
    dx, dy, dz, dh = (torch.from_numpy(v).to(dev) for v in (x, y, z, h))
    counts = torch.empty(n, dtype=torch.int32, device=dev)
    offsets = torch.empty(n + 1, dtype=torch.int64, device=dev)

    t = btree.BTree(dx, dy, dz, bucket_size=s, precision=a.precision, timing=True)
    _, _, total = t.count(dh, counts, offsets)
    nbrs = torch.empty(total, dtype=torch.int32, device=dev)
    elapsed, ph, st = timed(t, dx, dy, dz, dh, counts, offsets, nbrs, a.steps, a.warmup)
    ms_per_step = 1e3 * elapsed / a.steps
    value = n * a.steps / elapsed

    # Dominant kernel of the search (the sweep: walk, stage, pair tests,
    # rows) and its roofline.
    kern = "sweep_kernel" if ph["sweep_kernel"] >= ph["place_kernel"] else "place_kernel"
    kms = ph[kern]
    tests = st["pair_tests"]
    ops = OPS_PER_TEST_F32 if a.precision == "fp32" else OPS_PER_TEST_F64
    achieved = tests * ops / (kms * 1e-3) / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
            "frac": achieved / VALU_PEAK_TOPS, "kernel": "k_sweep<%s>" % (
                "fp32" if a.precision == "fp32" else "fp64"),
            "traffic": load_traffic(kern, a.workload),
            "algorithmic_ops_per_launch": tests * ops}
    # Compulsory HBM bytes of the whole search (both passes), per particle:
    # coordinates 24 B + h 8 B + count 4 B + offset 8 B, plus 4 B per entry.
    alg_bytes = n * (24 + 8 + 4 + 8) + 4 * total
    find_ms = ph["pass1"] + ph["pass2"]
    hbm = {"algorithmic_bytes": alg_bytes, "search_ms": find_ms,
           "achieved_GBs": alg_bytes / (find_ms * 1e-3) / 1e9,
           "frac": alg_bytes / (find_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}

    out = {
        "metric": "FindNeighbors particles/s (BuildTree + FindNeighbors per step)",
        "value": value, "unit": "particles/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if a.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "n": n, "bucket_size": s,
                   "precision": "fp32_filter+fp64_band" if a.precision == "fp32" else "fp64",
                   "neighbours_total": total, "neighbours_mean": total / n},
        "phases_ms": ph,
        "search_particles_per_s": n / (find_ms * 1e-3),
        "pair_tests_per_s": tests / (ph["sweep_kernel"] * 1e-3),
        "pair_tests_per_particle": tests / n,
        "fp64_confirmed_fraction": st["fp64_confirms"] / max(1, tests),
        "exhaustive_items": st["brute_chunks"],
        "tree": {"depth": st["depth"], "internal": st["n_internal"], "leaves": st["n_leaves"],
                 "b_hist": st["b_hist"]},
        "roofline": roof,
        "search_hbm": hbm,
    }
    t.close()
    if not a.no_compare and a.precision == "fp32":
        t2 = btree.BTree(dx, dy, dz, bucket_size=s, precision="fp64", timing=True)
        k2 = max(2, min(a.steps, 5))
        el2, ph2, _ = timed(t2, dx, dy, dz, dh, counts, offsets, nbrs, k2, 1)
        out["fp64_plain"] = {"value": n * k2 / el2, "ms_per_step": 1e3 * el2 / k2,
                             "search_ms": ph2["pass1"] + ph2["pass2"], "steps": k2}
        out["fp32_filter_speedup"] = out["value"] / out["fp64_plain"]["value"]
        t2.close()
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(x, y, z, h, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
