"""Autotuner of the bucket size s and beta (Table 1, Eq. 4), with a JSON cache.

Outputs never depend on s or beta, so a tuned choice can only change speed.
A particle set is keyed by (precision, distribution class, floor(log2 n));
the class separates sets with one smoothing length everywhere ("const_h",
e.g. a uniform cube) from sets whose h varies ("graded_h", e.g. a Plummer
sphere, whose density spans orders of magnitude).  A missing key is tuned on
the GPU by btree_tune (every candidate built and searched, median of
repeats) on the first set that needs it, and stored.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np

from . import btree

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache.json")


class TuneSpace(ctypes.Structure):
    _fields_ = [("n_bucket", ctypes.c_int32), ("bucket", ctypes.c_int32 * 16),
                ("n_beta", ctypes.c_int32), ("beta", ctypes.c_double * 8),
                ("repeats", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


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


def space(buckets=None, betas=None, repeats=None) -> TuneSpace:
    sp = TuneSpace()
    btree._check(_lib().btree_tune_space_default(ctypes.byref(sp)))
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
    table = np.zeros(sp.n_bucket * sp.n_beta, dtype=np.float64)
    btree._check(_lib().btree_tune(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(h.data_ptr()),
                                   n, ctypes.byref(base), ctypes.byref(sp), ctypes.byref(best),
                                   ctypes.byref(best_ms), table.ctypes.data,
                                   btree._stream(stream)))
    grid = {"%d/%g" % (sp.bucket[i], sp.beta[j]): float(table[i * sp.n_beta + j])
            for i in range(sp.n_bucket) for j in range(sp.n_beta)}
    return {"bucket_size": int(best.bucket_size), "beta": float(best.beta),
            "alpha": float(best.alpha), "ms": float(best_ms.value), "n": n, "table": grid}


class Tuner:
    """JSON-backed cache of tuned parameters."""

    def __init__(self, path: str = CACHE, sp: TuneSpace | None = None):
        self.path = path
        self.sp = sp
        self.entries = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)
        self.tuned_now = []

    def save(self, path: str | None = None):
        p = path or self.path
        with open(p, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)

    def params_for(self, x, y, z, h, precision="fp32") -> dict:
        """Parameters for one set (device tensors), tuning its key if new."""
        k = key(int(x.shape[0]), h, precision)
        if k not in self.entries:
            self.entries[k] = tune(x, y, z, h, precision, self.sp)
            self.tuned_now.append(k)
        e = self.entries[k]
        return {"bucket_size": e["bucket_size"], "beta": e["beta"], "alpha": e["alpha"]}
