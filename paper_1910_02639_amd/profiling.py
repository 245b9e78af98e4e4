"""Measurement helpers: a plain copy kernel of known size for calibrating
rocprofv3 byte counters, and summaries of rocprofv3 CSV output.

  python -m paper_1910_02639_amd.profiling copy --mib 1024 --reps 5
      runs a device-to-device copy of the given size (the calibration
      kernel: it must read and write exactly that many bytes).
  python -m paper_1910_02639_amd.profiling stats DIR
      prints a markdown table of a --kernel-trace --stats run.
  python -m paper_1910_02639_amd.profiling traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR
      COPY_WRITE_DIR --kernel k_sweep --mib 1024
      HBM bytes per dispatch of a kernel from two --pmc runs (FETCH_SIZE,
      WRITE_SIZE), each scaled by what the same counter reads for the copy.
      With --store NAME --workload W the result is also written to
      profiles/traffic.json under [NAME][W], with a hash of the search
      sources so that stale figures are not reported after a kernel change.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


SEARCH_SOURCES = ("find.hip", "common.h", "prim.h")
ALL_SOURCES = ("scan.hip", "sort.hip", "build.hip", "find.hip", "api.hip", "batch.hip",
               "common.h", "prim.h")


def source_hash(files=SEARCH_SOURCES):
    """Hash of kernel sources (by default the search's, which the traffic
    figures belong to), over their code only (line comments and blank lines
    do not count)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1910_02639_amd", "csrc", f)) as fh:
            for line in fh:
                code = re.sub(r"//.*", "", line).strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def copy_kernel(mib: int, reps: int):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied %d MiB x %d" % (mib, reps))


def _one(d, pattern):
    f = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not f:
        raise FileNotFoundError("no %s under %s" % (pattern, d))
    return f[0]


def stats_table(d, top=20):
    rows = list(csv.DictReader(open(_one(d, "*kernel_stats.csv"))))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        name = r["Name"].replace("(anonymous namespace)::", "").split("(")[0]
        out.append("| %s | %s | %.1f | %.2f | %.1f |" % (
            name, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6,
            float(r["Percentage"])))
    return "\n".join(out)


def counter_per_dispatch(d, counter, kernel):
    """Mean counter value (KiB) over the dispatches whose name contains kernel."""
    f = _one(d, "*counter_collection.csv")
    vals = {}
    for r in csv.DictReader(open(f)):
        if kernel not in r.get("Kernel_Name", r.get("Kernel-Name", "")):
            continue
        if r.get("Counter_Name", counter) != counter:
            continue
        key = r.get("Dispatch_Id", r.get("Correlation_Id"))
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise ValueError("no %s dispatches of %s in %s" % (counter, kernel, f))
    return sum(vals.values()) / len(vals), len(vals)


def traffic(fetch_dir, write_dir, cfetch_dir, cwrite_dir, kernel, copy_kernel_name, mib):
    fk, nf = counter_per_dispatch(fetch_dir, "FETCH_SIZE", kernel)
    wk, nw = counter_per_dispatch(write_dir, "WRITE_SIZE", kernel)
    cf, _ = counter_per_dispatch(cfetch_dir, "FETCH_SIZE", copy_kernel_name)
    cw, _ = counter_per_dispatch(cwrite_dir, "WRITE_SIZE", copy_kernel_name)
    nbytes = mib * (1 << 20)
    # bytes per counter unit, from the copy that reads and writes nbytes
    sf, sw = nbytes / cf, nbytes / cw
    return {"fetch_kib": fk, "write_kib": wk, "dispatches": [nf, nw],
            "copy_fetch_kib": cf, "copy_write_kib": cw, "scale_fetch": sf, "scale_write": sw,
            "fetch_bytes": fk * sf, "write_bytes": wk * sw, "bytes_per_launch": fk * sf + wk * sw}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=5)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("copy_fetch_dir")
    t.add_argument("copy_write_dir")
    t.add_argument("--kernel", default="k_sweep")
    t.add_argument("--copy-kernel", default="copy")
    t.add_argument("--mib", type=int, default=1024)
    t.add_argument("--store", default=None, help="entry name in profiles/traffic.json")
    t.add_argument("--workload", default=None)
    a = ap.parse_args(argv)
    if a.cmd == "copy":
        copy_kernel(a.mib, a.reps)
    elif a.cmd == "stats":
        print(stats_table(a.dir))
    else:
        r = traffic(a.fetch_dir, a.write_dir, a.copy_fetch_dir, a.copy_write_dir,
                    a.kernel, a.copy_kernel, a.mib)
        print(json.dumps(r, indent=1))
        if a.store:
            path = os.path.join(ROOT, "profiles", "traffic.json")
            d = json.load(open(path)) if os.path.exists(path) else {}
            r["source_hash"] = source_hash()
            d.setdefault(a.store, {})[a.workload] = r
            with open(path, "w") as fh:
                json.dump(d, fh, indent=1)


if __name__ == "__main__":
    sys.exit(main())
