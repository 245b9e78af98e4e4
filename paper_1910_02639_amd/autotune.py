"""Autotuner of the bucket size s and beta (Table 1, Eq. 4), with a JSON cache.

Outputs never depend on s or beta, so a tuned choice can only change speed.
A particle set is keyed by (precision, distribution class, floor(log2 n));
the class separates sets with one smoothing length everywhere ("const_h",
e.g. a uniform cube) from sets whose h varies ("graded_h", e.g. a Plummer
sphere, whose density spans orders of magnitude).  Every cache entry records
a hash of the kernel sources it was timed on.  A missing key, or one timed
on other sources, is tuned on the GPU by btree_tune (every candidate built
and searched, median of repeats) on the first set that needs it, with one
progress line per key on stderr, within an optional time budget; past the
budget (or with tuning switched off) a stale entry is still used (it is a
valid choice, only perhaps no longer the fastest) and a missing one falls
back to the library defaults.
"""
from __future__ import annotations

import sys
import time
import ctypes
import json
import math
import os

import numpy as np

from . import btree, profiling

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


class TuneSpace(ctypes.Structure):
    _fields_ = [("n_bucket", ctypes.c_int32), ("bucket", ctypes.c_int32 * 16),
                ("n_beta", ctypes.c_int32), ("beta", ctypes.c_double * 8),
                ("repeats", ctypes.c_int32), ("n_alpha", ctypes.c_int32),
                ("alpha", ctypes.c_double * 4), ("reserved", ctypes.c_int32 * 2)]


def _lib():
    L = btree.lib()
    if not getattr(L, "_tune_bound", False):
        P = ctypes.c_void_p
        L.btree_tune_space_default.restype = ctypes.c_int
        L.btree_tune_space_default.argtypes = [ctypes.POINTER(TuneSpace)]
        L.btree_tune.restype = ctypes.c_int
        L.btree_tune.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.POINTER(btree.Params),
                                 ctypes.POINTER(TuneSpace), ctypes.POINTER(btree.Params),
                                 ctypes.POINTER(ctypes.c_double), P, P]
        L._tune_bound = True
    return L


def space(buckets=None, betas=None, repeats=None, alphas=None) -> TuneSpace:
    sp = TuneSpace()
    btree._check(_lib().btree_tune_space_default(ctypes.byref(sp)))
    if alphas is not None:
        sp.n_alpha = len(alphas)
        for k, a in enumerate(alphas):
            sp.alpha[k] = float(a)
    if buckets is not None:
        sp.n_bucket = len(buckets)
        for k, b in enumerate(buckets):
            sp.bucket[k] = int(b)
    if betas is not None:
        sp.n_beta = len(betas)
        for k, b in enumerate(betas):
            sp.beta[k] = float(b)
    if repeats is not None:
        sp.repeats = int(repeats)
    return sp


def distribution_class(h) -> str:
    """'const_h' when every positive h is within 5% of the others, else
    'graded_h'.  h: host array or device tensor."""
    a = h.detach().cpu().numpy() if hasattr(h, "detach") else np.asarray(h)
    a = a[a > 0]
    if a.size == 0 or a.max() <= 1.05 * a.min():
        return "const_h"
    return "graded_h"


def key(n: int, h, precision: str) -> str:
    return "%s/%s/%d" % (precision, distribution_class(h), int(math.floor(math.log2(max(n, 1)))))


def tune(x, y, z, h, precision="fp32", sp: TuneSpace | None = None, stream=None) -> dict:
    """Runs btree_tune on device tensors; returns the best parameters, its
    median time and the whole timing table."""
    n = int(x.shape[0])
    base = btree.params(precision=precision)
    sp = sp if sp is not None else space()
    best = btree.Params()
    best_ms = ctypes.c_double()
    na = max(sp.n_alpha, 1)
    table = np.zeros(sp.n_bucket * sp.n_beta * na, dtype=np.float64)
    btree._check(_lib().btree_tune(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(h.data_ptr()),
                                   n, ctypes.byref(base), ctypes.byref(sp), ctypes.byref(best),
                                   ctypes.byref(best_ms), table.ctypes.data,
                                   btree._stream(stream)))
    alphas = [sp.alpha[k] for k in range(sp.n_alpha)] or [float(base.alpha)]
    grid = {"%d/%g/%g" % (sp.bucket[i], sp.beta[j], alphas[a]):
            float(table[(i * sp.n_beta + j) * na + a])
            for i in range(sp.n_bucket) for j in range(sp.n_beta) for a in range(na)}
    return {"bucket_size": int(best.bucket_size), "beta": float(best.beta),
            "alpha": float(best.alpha), "ms": float(best_ms.value), "n": n, "table": grid}


def kernels_hash() -> str:
    """Hash of every kernel source of the library (code lines only)."""
    return profiling.source_hash(profiling.ALL_SOURCES)


class Tuner:
    """JSON-backed cache of tuned parameters.

    tune_missing: tune keys that are absent or stale (else use what is there,
    or the defaults).  budget_s: total seconds of tuning this object may
    spend; keys met after that are treated as with tune_missing=False."""

    def __init__(self, path: str = CACHE, sp: TuneSpace | None = None,
                 tune_missing: bool = True, budget_s: float | None = None, log=None):
        self.path = path
        self.sp = sp
        self.tune_missing = tune_missing
        self.budget_s = budget_s
        self.spent_s = 0.0
        self.entries = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)
        self.hash = kernels_hash()
        self.tuned_now = []   # keys tuned by this object
        self.stale_used = []  # keys used although timed on other sources
        self.defaults_used = []  # keys with no entry that were not tuned
        self._log = log if log is not None else (
            lambda *a: print("[tune %s]" % time.strftime("%H:%M:%S"), *a, file=sys.stderr,
                             flush=True))

    def save(self, path: str | None = None):
        p = path or self.path
        with open(p, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)

    def fresh(self, k: str) -> bool:
        e = self.entries.get(k)
        return bool(e) and e.get("source_hash") == self.hash

    def params_for(self, x, y, z, h, precision="fp32") -> dict:
        """Parameters for one set (device tensors), tuning its key if new or
        stale (and allowed)."""
        n = int(x.shape[0])
        k = key(n, h, precision)
        if not self.fresh(k):
            can = self.tune_missing and (self.budget_s is None or self.spent_s < self.budget_s)
            if can:
                sp = self.sp if self.sp is not None else space()
                self._log("tuning %s (n = %d, %d candidates)" % (
                    k, n, sp.n_bucket * sp.n_beta * max(sp.n_alpha, 1)))
                t0 = time.perf_counter()
                e = tune(x, y, z, h, precision, self.sp)
                dt = time.perf_counter() - t0
                self.spent_s += dt
                e["source_hash"] = self.hash
                e["tune_s"] = dt
                self.entries[k] = e
                self.tuned_now.append(k)
                self._log("tuned %s: s = %d, beta = %g, alpha = %g, %.3f ms (%.1f s)" % (
                    k, e["bucket_size"], e["beta"], e["alpha"], e["ms"], dt))
            elif k in self.entries:
                if k not in self.stale_used:
                    self.stale_used.append(k)
            else:
                if k not in self.defaults_used:
                    self.defaults_used.append(k)
                return {}
        e = self.entries[k]
        return {"bucket_size": e["bucket_size"], "beta": e["beta"], "alpha": e["alpha"]}
