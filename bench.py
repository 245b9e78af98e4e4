#!/usr/bin/env python3
"""Benchmark of the b-tree hot path (BuildTree + FindNeighbors) on one MI355X.

Default workload Batch64: 64 independent particle sets, sizes log-uniform in
[1e4, 1e6], even sets uniform cubes and odd sets Plummer spheres.  One step
is one batched run: BuildTree and both FindNeighbors passes of every set as
one captured HIP graph (FP32 filter + FP64 band), parameters per set from
the autotuner's cache.  Compared in the same run with the plain FP64 form
launched one set at a time (and the FP32 form one set at a time), with the
8M-particle Plummer sphere (P8M) as a single-set block, and with the FP64
oracle on the host cores.  Inputs are resident in HBM before timing.

  python bench.py [--steps K] [--warmup W] [--workload Batch64|P8M|...]

Prints one JSON line.
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

from paper_1910_02639_amd import profiling  # noqa: E402  (no GPU or HIP use)

HBM_PEAK_GBS = 8000.0
# Non-packed VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-ops/s.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane-ops of one FP32-filter pair test: 3 sub, 1 mul, 2 fma, 2 compare.
OPS_PER_TEST_F32 = 8
# ... and of one FP64 pair test: 3 sub, 3 mul, 2 add, 1 compare.
OPS_PER_TEST_F64 = 9
METRIC = "FindNeighbors particles/s (BuildTree + FindNeighbors per step)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="Batch64",
                    choices=["Batch64", "U10k", "L1M", "P8M", "P16M"])
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--bucket", type=int, default=0, help="single set: bucket size (0 = tuned)")
    ap.add_argument("--tune-cache", default=None, help="autotuner JSON cache (default: package)")
    ap.add_argument("--tune-out", default=None, help="write the cache here after tuning")
    ap.add_argument("--tune-budget", type=float, default=120.0,
                    help="seconds of tuning allowed for absent or stale cache keys (0: none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the comparison forms")
    ap.add_argument("--no-single", action="store_true",
                    help="Batch64: skip the single-set blocks (P8M, P16M, L1M, U10k)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def log(*a):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print("[bench %s]" % time.strftime("%H:%M:%S"), *a, file=sys.stderr, flush=True)


def load_traffic(kernel, workload):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/), or
    None when absent or taken on a different kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(kernel, {}).get(workload)
        if e and e.get("source_hash") == profiling.source_hash():
            return e["bytes_per_launch"]
    except Exception:
        return None
    return None


def phase_delta(s0, s1):
    return {k: (s1["phase_ms"][k] - s0["phase_ms"][k]) /
            max(1, s1["phase_calls"][k] - s0["phase_calls"][k]) for k in s1["phase_ms"]}


def roofline(kernel_ms, tests, ops, kernel, workload):
    achieved = tests * ops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
            "frac": achieved / VALU_PEAK_TOPS, "kernel": kernel,
            "traffic": load_traffic("sweep_kernel", workload),
            "algorithmic_ops_per_launch": tests * ops}


def hbm_measured(ph, workload):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    profiles/traffic.json) over the kernels' time in this run, against the
    8 TB/s peak: the sweep, and the placement (k_expand and k_place, timed
    together as the placement phase; in the batched graph the phase also
    holds the exhaustive fill)."""
    out = {}
    t = load_traffic("sweep_kernel", workload)
    if t is not None and ph.get("sweep_kernel", 0.0) > 0.0:
        gbs = t / (ph["sweep_kernel"] * 1e-3) / 1e9
        out["k_sweep"] = {"hbm_bytes": t, "ms": ph["sweep_kernel"], "GB_s": gbs,
                          "frac": gbs / HBM_PEAK_GBS}
    te, tp = load_traffic("expand_kernel", workload), load_traffic("place_kernel", workload)
    if te is not None and tp is not None and ph.get("place_kernel", 0.0) > 0.0:
        gbs = (te + tp) / (ph["place_kernel"] * 1e-3) / 1e9
        out["k_expand+k_place"] = {"hbm_bytes": te + tp, "ms": ph["place_kernel"], "GB_s": gbs,
                                   "frac": gbs / HBM_PEAK_GBS}
    return out or None


def roofline_hbm(n, total, kernel_ms, workload):
    """The dominant kernel against the HBM roofline: the search's compulsory
    bytes (coordinates 24 B, h 8 B, count 4 B, offset 8 B per particle, 4 B
    per list entry) over the sweep kernel's time, with the measured traffic
    (rocprofv3 counters, profiles/traffic.json) and its ratio to them."""
    alg = n * (24 + 8 + 4 + 8) + 4 * total
    gbs = alg / (kernel_ms * 1e-3) / 1e9
    t = load_traffic("sweep_kernel", workload)
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": alg, "traffic": t,
            "traffic_ratio": (t / alg) if t else None}


def pair_rates(tests, step_ms, sweep_ms):
    """Pair tests per second over the whole step and over the sweep kernel."""
    return {"per_step": tests / (step_ms * 1e-3),
            "sweep_kernel": tests / (sweep_ms * 1e-3) if sweep_ms > 0 else None}


# The paper's own figures (CPU only; context, not a target): one Intel Xeon
# E5-2640 v4 node, 20 cores + 20 hyper-threads, 40 OpenMP threads (Table 2).
PAPER_CONTEXT = {
    "hardware": "Intel Xeon E5-2640 v4, 20 cores (40 threads), CPU only (Table 2)",
    "btree_vs_octree": {"find_neighbors": "up to 1.6x faster", "build_tree": "up to 12x faster"},
    "find_neighbors_s": {"evrard_collapse_1e6_100nb": 0.15, "square_patch_1e7_500nb": 4.0},
    "derived_particles_per_s": {"evrard_collapse": 6.7e6, "square_patch": 2.5e6},
    "note": "Section 4 prose (the figures are not in the source); the GPU workloads here are "
            "synthetic stand-ins, so no ratio to these is reported",
}


def search_hbm(n, total, search_ms):
    # Compulsory HBM bytes of the whole search (both passes), per particle:
    # coordinates 24 B + h 8 B + count 4 B + offset 8 B, plus 4 B per entry.
    alg = n * (24 + 8 + 4 + 8) + 4 * total
    gbs = alg / (search_ms * 1e-3) / 1e9
    return {"algorithmic_bytes": alg, "search_ms": search_ms, "achieved_GBs": gbs,
            "frac": gbs / HBM_PEAK_GBS}


# ---------------------------------------------------------------------------
# Single set: BuildTree (btree_rebuild) + pass 1 + pass 2 per step, eager.
# ---------------------------------------------------------------------------
def single_steps(t, dx, dy, dz, dh, counts, offsets, nbrs, k):
    for _ in range(k):
        t.rebuild(dx, dy, dz)
        t.count(dh, counts, offsets)
        t.fill(dh, counts, offsets, nbrs)


def single_timed(t, args, steps, warmup):
    import torch
    single_steps(t, *args, warmup)
    torch.cuda.synchronize()
    s0 = t.stats()
    t0 = time.perf_counter()
    single_steps(t, *args, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s1 = t.stats()
    return el, phase_delta(s0, s1), s1


def bench_single(name, precision, steps, warmup, compare, tuner, bucket=0):
    import torch
    from paper_1910_02639_amd import btree, workloads as W
    log("generate", name)
    x, y, z, h, s = W.make(name)
    n = len(x)
    dx, dy, dz, dh = (torch.from_numpy(v).to("cuda:0") for v in (x, y, z, h))
    if bucket:
        prm = {"bucket_size": bucket}
    else:
        log("tune", name, precision)
        prm = tuner.params_for(dx, dy, dz, dh, precision)
    log("time", name, precision, prm)
    counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
    t = btree.BTree(dx, dy, dz, precision=precision, timing=True, **prm)
    _, _, total = t.count(dh, counts, offsets)
    nbrs = torch.empty(total, dtype=torch.int32, device="cuda:0")
    args = (dx, dy, dz, dh, counts, offsets, nbrs)
    el, ph, st = single_timed(t, args, steps, warmup)
    t.close()
    ops = OPS_PER_TEST_F32 if precision == "fp32" else OPS_PER_TEST_F64
    out = {"workload": name, "n": n, "params": prm, "value": n * steps / el,
           "ms_per_step": 1e3 * el / steps, "phases_ms": ph,
           "neighbours_total": total, "pair_tests_per_particle": st["pair_tests"] / n,
           "pair_tests_per_s": pair_rates(st["pair_tests"], 1e3 * el / steps, ph["sweep_kernel"]),
           "fp64_confirmed_fraction": st["fp64_confirms"] / max(1, st["pair_tests"]),
           "exhaustive_items": st["brute_chunks"],
           "exhaustive_units": st["brute_units"], "split_items": st["split_items"],
           "tree": {"depth": st["depth"], "internal": st["n_internal"],
                    "leaves": st["n_leaves"], "b_hist": st["b_hist"]},
           "roofline": roofline(ph["sweep_kernel"], st["pair_tests"], ops,
                                "k_sweep<%s>" % precision, name),
           "roofline_hbm": roofline_hbm(n, total, ph["sweep_kernel"], name),
           "search_hbm": search_hbm(n, total, ph["pass1"] + ph["pass2"]),
           "hbm_measured": hbm_measured(ph, name) if precision == "fp32" else None}
    if compare and precision == "fp32":
        log("fp64 plain", name)
        p64 = tuner.params_for(dx, dy, dz, dh, "fp64") if not bucket else prm
        t2 = btree.BTree(dx, dy, dz, precision="fp64", timing=True, **p64)
        k2 = max(2, min(steps, 5))
        el2, ph2, st2 = single_timed(t2, args, k2, 1)
        t2.close()
        out["fp64_plain"] = {"value": n * k2 / el2, "ms_per_step": 1e3 * el2 / k2,
                             "params": p64, "search_ms": ph2["pass1"] + ph2["pass2"], "steps": k2,
                             "pair_tests_per_s": pair_rates(st2["pair_tests"], 1e3 * el2 / k2,
                                                           ph2["sweep_kernel"])}
        out["fp32_filter_speedup"] = out["value"] / out["fp64_plain"]["value"]
    return out, (x, y, z, h)


# ---------------------------------------------------------------------------
# Batch64: one captured graph per step vs one set per launch.
# ---------------------------------------------------------------------------
def per_set_loop(handles, views, bufs, k):
    for _ in range(k):
        for t, (x, y, z, h), (c, o, nb) in zip(handles, views, bufs):
            t.rebuild(x, y, z)
            t.count(h, c, o)
            t.fill(h, c, o, nb)


def bench_per_set(views, prms, precision, steps, warmup):
    """Every set built and searched by its own calls, one after the other."""
    import torch
    from paper_1910_02639_amd import btree
    handles, bufs = [], []
    for (x, y, z, h), p in zip(views, prms):
        t = btree.BTree(x, y, z, precision=precision, **p)
        c = torch.empty(x.shape[0], dtype=torch.int32, device="cuda:0")
        o = torch.empty(x.shape[0] + 1, dtype=torch.int64, device="cuda:0")
        _, _, tot = t.count(h, c, o)
        nb = torch.empty(max(tot, 1), dtype=torch.int32, device="cuda:0")
        handles.append(t)
        bufs.append((c, o, nb))
    per_set_loop(handles, views, bufs, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per_set_loop(handles, views, bufs, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for t in handles:
        t.close()
    n = sum(v[0].shape[0] for v in views)
    return {"value": n * steps / el, "ms_per_step": 1e3 * el / steps, "steps": steps}


def bench_batch(a, tuner):
    import numpy as np
    import torch
    from paper_1910_02639_amd import btree, workloads as W
    log("generate Batch64")
    sets = W.batch(64, 0)
    sizes = [len(s[0]) for s in sets]
    n = int(sum(sizes))
    host = [np.concatenate([s[c] for s in sets]) for c in range(4)]
    dx, dy, dz, dh = (torch.from_numpy(v).to("cuda:0") for v in host)
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    views = [tuple(t[int(offs[k]):int(offs[k + 1])] for t in (dx, dy, dz, dh))
             for k in range(len(sizes))]
    log("tune fp32 (%d sets, %d particles)" % (len(sizes), n))
    prm32 = [tuner.params_for(*v, "fp32") for v in views]
    log("batched graph runs")

    B = btree.Batch(sizes, prm32, precision="fp32", timing=True)
    counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
    c, o, nb, totals = B.find(dx, dy, dz, dh)
    total = int(totals.sum())
    del c, o, nb
    nbrs = torch.empty(total, dtype=torch.int32, device="cuda:0")
    for _ in range(a.warmup):
        B.run(dx, dy, dz, dh, counts, offsets, nbrs)
    torch.cuda.synchronize()
    s0 = B.stats()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        B.run(dx, dy, dz, dh, counts, offsets, nbrs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = B.stats()
    ph = phase_delta(s0, st)
    B.close()

    out = {
        "metric": METRIC, "value": n * a.steps / el, "unit": "particles/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": 1e3 * el / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "Batch64", "sets": len(sizes), "n": n,
                   "set_sizes_min_max": [int(min(sizes)), int(max(sizes))],
                   "form": "captured HIP graph per step: 5 segments back to back, "
                           "build + both search passes of all sets",
                   "precision": "fp32_filter+fp64_band", "params": "autotuned per set",
                   "buckets_used": sorted({p["bucket_size"] for p in prm32}),
                   "neighbours_total": total, "neighbours_mean": total / n},
        "phases_ms": ph,
        "search_particles_per_s": n / ((ph["pass1"] + ph["pass2"]) * 1e-3),
        "pair_tests_per_particle": st["pair_tests"] / n,
        "pair_tests_per_s": pair_rates(st["pair_tests"], 1e3 * el / a.steps, ph["sweep_kernel"]),
        "fp64_confirmed_fraction": st["fp64_confirms"] / max(1, st["pair_tests"]),
        "exhaustive_items": st["brute_chunks"],
        "exhaustive_units": st["brute_units"], "split_items": st["split_items"],
        "graph": {"launches": st["graph_launches"], "recordings": st["graph_captures"]},
        "paper_context": PAPER_CONTEXT,
        "tree": {"depth": st["depth"], "internal": st["n_internal"], "leaves": st["n_leaves"]},
        "roofline": roofline(ph["sweep_kernel"], st["pair_tests"], OPS_PER_TEST_F32,
                             "k_sweep<fp32>", "Batch64"),
        "roofline_hbm": roofline_hbm(n, total, ph["sweep_kernel"], "Batch64"),
        "search_hbm": search_hbm(n, total, ph["pass1"] + ph["pass2"]),
        "hbm_measured": hbm_measured(ph, "Batch64"),
        "_prm32": prm32,
    }
    if not a.no_compare:
        k2 = max(2, min(a.steps, 5))
        log("tune fp64")
        prm64 = [tuner.params_for(*v, "fp64") for v in views]
        log("fp64 one set per launch")
        f64 = bench_per_set(views, prm64, "fp64", k2, 1)
        log("fp32 one set per launch")
        f32 = bench_per_set(views, prm32, "fp32", k2, 1)
        out["fp64_one_set_per_launch"] = f64
        out["fp32_one_set_per_launch"] = f32
        out["batched_fp32_vs_fp64_per_set"] = out["value"] / f64["value"]
        out["batching_speedup_fp32"] = out["value"] / f32["value"]
    return out, sets


# ---------------------------------------------------------------------------
# b-tree against the octree, build-time sweeps, the fused density and the h
# adaptation (single sets and the batch).
# ---------------------------------------------------------------------------
def _tree_view(st):
    return {"depth": st["depth"], "internal": st["n_internal"], "leaves": st["n_leaves"]}


def bench_octree_single(name, tuner, steps=5):
    """The b-tree against the octree (b = 2 at every split) with the same
    bucket size: BuildTree and FindNeighbors time per step, tree depths."""
    import torch
    from paper_1910_02639_amd import btree, workloads as W
    x, y, z, h, _ = W.make(name)
    n = len(x)
    dx, dy, dz, dh = (torch.from_numpy(v).to("cuda:0") for v in (x, y, z, h))
    prm = tuner.params_for(dx, dy, dz, dh, "fp32") or {"bucket_size": 64}
    counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
    out = {"workload": name, "n": n, "bucket_size": prm["bucket_size"]}
    for label, extra in (("btree", {}), ("octree", {"octree": True})):
        log("octree comparison", name, label)
        t = btree.BTree(dx, dy, dz, precision="fp32", timing=True, **prm, **extra)
        _, _, total = t.count(dh, counts, offsets)
        nbrs = torch.empty(max(total, 1), dtype=torch.int32, device="cuda:0")
        el, ph, st = single_timed(t, (dx, dy, dz, dh, counts, offsets, nbrs), steps, 1)
        t.close()
        del nbrs
        out[label] = {"build_ms": ph["build"], "search_ms": ph["pass1"] + ph["pass2"],
                      "ms_per_step": 1e3 * el / steps,
                      "pair_tests_per_particle": st["pair_tests"] / n, "tree": _tree_view(st)}
    out["build_speedup_btree_vs_octree"] = out["octree"]["build_ms"] / out["btree"]["build_ms"]
    out["search_speedup_btree_vs_octree"] = out["octree"]["search_ms"] / out["btree"]["search_ms"]
    return out


def bench_octree_batch(sets, prm32, steps=5):
    """Batch64 with every set's tree an octree (same bucket size per set)."""
    import numpy as np
    import torch
    from paper_1910_02639_amd import btree
    sizes = [len(s[0]) for s in sets]
    n = int(sum(sizes))
    host = [np.concatenate([s[c] for s in sets]) for c in range(4)]
    dx, dy, dz, dh = (torch.from_numpy(v).to("cuda:0") for v in host)
    out = {}
    for label, extra in (("btree", {}), ("octree", {"octree": True})):
        log("octree comparison Batch64", label)
        B = btree.Batch(sizes, [dict(p, **extra) for p in prm32], precision="fp32", timing=True)
        counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
        offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
        c, o, nb, totals = B.find(dx, dy, dz, dh)
        nbrs = torch.empty(int(totals.sum()), dtype=torch.int32, device="cuda:0")
        del c, o, nb
        B.run(dx, dy, dz, dh, counts, offsets, nbrs)
        torch.cuda.synchronize()
        s0 = B.stats()
        t0 = time.perf_counter()
        for _ in range(steps):
            B.run(dx, dy, dz, dh, counts, offsets, nbrs)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = B.stats()
        ph = phase_delta(s0, st)
        B.close()
        out[label] = {"build_ms": ph["build"], "search_ms": ph["pass1"] + ph["pass2"],
                      "ms_per_step": 1e3 * el / steps,
                      "pair_tests_per_particle": st["pair_tests"] / n, "tree": _tree_view(st)}
    out["build_speedup_btree_vs_octree"] = out["octree"]["build_ms"] / out["btree"]["build_ms"]
    out["search_speedup_btree_vs_octree"] = out["octree"]["search_ms"] / out["btree"]["search_ms"]
    return out


def bench_build_sweep(name, buckets=(16, 32, 64, 128, 256), betas=(0.3, 0.5, 0.8), reps=5):
    """BuildTree time alone (rebuilds of one handle) over (s, beta), and the
    octree at each s (the bucket-size and beta sweeps of the paper's build
    figures)."""
    import torch
    from paper_1910_02639_amd import btree, workloads as W
    x, y, z, _, _ = W.make(name)
    dx, dy, dz = (torch.from_numpy(v).to("cuda:0") for v in (x, y, z))
    table, depth = {}, {}
    for s_ in buckets:
        for key, kw in [("%d/%g" % (s_, b), {"beta": b}) for b in betas] + \
                       [("%d/octree" % s_, {"octree": True})]:
            # Rebuilds only (the first build of a handle also sizes its pools):
            # one untimed, then `reps` timed.
            t = btree.BTree(dx, dy, dz, bucket_size=s_, timing=True, **kw)
            t.rebuild(dx, dy, dz)
            torch.cuda.synchronize()
            s0 = t.stats()
            for _ in range(reps):
                t.rebuild(dx, dy, dz)
            torch.cuda.synchronize()
            st = t.stats()
            t.close()
            table[key] = (st["phase_ms"]["build"] - s0["phase_ms"]["build"]) / reps
            depth[key] = st["depth"]
    log("build sweep", name, "done")
    return {"workload": name, "build_ms": table, "depth": depth}


def bench_density_and_adapt(name, tuner, steps=5):
    """The fused density (no lists) against the lists (both passes), and the
    h adaptation from 0.7 h to the workload's target count, on the tree of
    the single-set timing's (tuned) parameters."""
    import torch
    from paper_1910_02639_amd import btree, workloads as W
    x, y, z, h, s_ = W.make(name)
    n = len(x)
    dx, dy, dz, dh = (torch.from_numpy(v).to("cuda:0") for v in (x, y, z, h))
    prm = tuner.params_for(dx, dy, dz, dh, "fp32")
    t = btree.BTree(dx, dy, dz, **prm)
    counts = torch.empty(n, dtype=torch.int32, device="cuda:0")
    offsets = torch.empty(n + 1, dtype=torch.int64, device="cuda:0")
    rho = torch.empty(n, dtype=torch.float64, device="cuda:0")
    _, _, total = t.count(dh, counts, offsets)
    nbrs = torch.empty(total, dtype=torch.int32, device="cuda:0")
    t.density(dh, rho=rho, counts=counts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t.density(dh, rho=rho, counts=counts)
    torch.cuda.synchronize()
    dens_ms = 1e3 * (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        t.count(dh, counts, offsets)
        t.fill(dh, counts, offsets, nbrs)
    torch.cuda.synchronize()
    lists_ms = 1e3 * (time.perf_counter() - t0) / steps
    del nbrs
    target = 64.0 if name == "U10k" else 100.0
    h0 = dh * 0.7
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, rounds = t.adapt_h(h0, target, 3.0, 60)
    torch.cuda.synchronize()
    adapt_ms = 1e3 * (time.perf_counter() - t0)
    within = float(((c.to(torch.float64) - target).abs() <= 3.0).double().mean())
    t.close()
    log("density and h adaptation", name, "done")
    return {"workload": name, "n": n, "params": prm, "density_ms": dens_ms, "lists_ms": lists_ms,
            "density_vs_lists_speedup": lists_ms / dens_ms,
            "adapt_h": {"from": "0.7 h", "target": target, "tol": 3.0, "rounds": rounds,
                        "ms": adapt_ms, "ms_per_round": adapt_ms / max(rounds + 1, 1),
                        "fraction_within_tol": within}}


def cpu_baseline_sets(sets, budget_s):
    """The oracle's cell list (every row of a set, FP64, OpenMP over rows) on
    a bounded sample: whole sets of the workload in a seeded random order
    until the budget is spent; particles/s = particles of the sets done /
    their wall time."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    rng = np.random.default_rng(12345)
    order = rng.permutation(len(sets))
    done, npart, dt = [], 0, 0.0
    for k in order:
        x, y, z, h = sets[k]
        t0 = time.perf_counter()
        oracle.cell_lists(x, y, z, h)
        dt += time.perf_counter() - t0
        done.append(int(k))
        npart += len(x)
        if dt >= budget_s:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    return {"value": npart / dt, "unit": "particles/s", "cores": cores, "kind": "oracle",
            "sample": "oracle cell list (all rows, FP64) over %d of the %d sets, %d particles "
                      "(%.1f s)" % (len(done), len(sets), npart, dt)}


def prm32_of(out):
    return out["_prm32"]


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    from paper_1910_02639_amd import autotune
    tuner = autotune.Tuner(a.tune_cache or autotune.CACHE, tune_missing=a.tune_budget > 0,
                           budget_s=a.tune_budget)
    if a.workload == "Batch64":
        out, sets = bench_batch(a, tuner)
        if not a.no_single:
            p8, _ = bench_single("P8M", "fp32", max(2, min(a.steps, 10)), 2, not a.no_compare,
                                 tuner)
            out["single_set_P8M"] = p8
            p16, _ = bench_single("P16M", "fp32", max(2, min(a.steps, 5)), 1, False, tuner)
            out["precision_form_P16M"] = {
                k: p16[k] for k in ("n", "params", "value", "ms_per_step", "phases_ms",
                                    "neighbours_total", "pair_tests_per_particle",
                                    "fp64_confirmed_fraction", "exhaustive_items", "search_hbm")}
            if not a.no_compare:
                out["octree_vs_btree"] = {
                    "Batch64": bench_octree_batch(sets, prm32_of(out)),
                    "P8M": bench_octree_single("P8M", tuner),
                    "L1M": bench_octree_single("L1M", tuner)}
                out["build_sweep_P8M"] = bench_build_sweep("P8M")
                out["sph_P8M"] = bench_density_and_adapt("P8M", tuner)
            for name in ("L1M", "U10k"):
                r, _ = bench_single(name, "fp32", max(2, min(a.steps, 10)), 2, not a.no_compare,
                                    tuner)
                out["single_set_" + name] = {
                    k: r[k] for k in ("n", "params", "value", "ms_per_step", "phases_ms",
                                      "neighbours_total", "pair_tests_per_particle",
                                      "fp64_confirmed_fraction", "tree", "roofline",
                                      "search_hbm", "fp64_plain", "fp32_filter_speedup")
                    if k in r}
    else:
        r, xyzh = bench_single(a.workload, a.precision, a.steps, a.warmup, not a.no_compare,
                               tuner, a.bucket)
        out = {"metric": METRIC, "value": r["value"], "unit": "particles/s", "n_gpus": 1,
               "steps": a.steps, "warmup": a.warmup, "ms_per_step": r["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f32+f64" if a.precision == "fp32" else "f64", "data": "synthetic",
               "config": {"workload": a.workload, "n": r["n"], "params": r["params"],
                          "precision": "fp32_filter+fp64_band" if a.precision == "fp32"
                          else "fp64", "neighbours_total": r["neighbours_total"]}}
        for k in ("phases_ms", "pair_tests_per_particle", "fp64_confirmed_fraction",
                  "exhaustive_items", "tree", "roofline", "search_hbm", "fp64_plain",
                  "fp32_filter_speedup"):
            if k in r:
                out[k] = r[k]
        sets = [xyzh]
    out["tuning"] = {"tuned_now": tuner.tuned_now, "tune_s": round(tuner.spent_s, 1),
                     "stale_entries_used": tuner.stale_used,
                     "defaults_used": tuner.defaults_used}
    if tuner.tuned_now and a.tune_out:
        tuner.save(a.tune_out)
    out.pop("_prm32", None)
    if not a.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline_sets(sets, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
