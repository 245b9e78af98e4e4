"""Python binding of libbtree (include/btree.h): argument marshalling only.

Every step of the search runs in the HIP library; this module only checks
tensor dtypes/devices, allocates outputs with torch and forwards raw device
pointers and the current HIP stream.  There is no fallback: if libbtree.so
is missing or cannot be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbtree.so")

BTREE_OK = 0
BTREE_EINVAL = -1
BTREE_ENOMEM = -2
BTREE_EDEVICE = -3
BTREE_EOVERFLOW = -4
BTREE_ESTATE = -5
BTREE_FP64 = 0
BTREE_FP32_FILTER = 1

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EOVERFLOW",
                -5: "ESTATE"}

SYMBOLS = ["btree_params_default", "btree_build", "btree_rebuild", "btree_find_neighbors",
           "btree_stats", "btree_export", "btree_destroy", "btree_last_error",
           "btree_batch_create", "btree_batch_run", "btree_batch_stats", "btree_batch_destroy",
           "btree_batch_graph_counts", "btree_tune_space_default", "btree_tune",
           "btree_find_neighbors_noalloc", "btree_density", "btree_adapt_h"]

NOALLOC_MAX_N = 65536


class Params(ctypes.Structure):
    _fields_ = [("bucket_size", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("max_depth", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("group_size", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("exclude_self", ctypes.c_int32),
                ("octree", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_internal", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("depth", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("max_leaf", ctypes.c_int64),
                ("oversized", ctypes.c_int64), ("n_chunks", ctypes.c_int64),
                ("b_hist", ctypes.c_int64 * 65), ("total", ctypes.c_int64),
                ("pair_tests", ctypes.c_int64), ("fp64_confirms", ctypes.c_int64),
                ("brute_chunks", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("phase_ms", ctypes.c_double * 5), ("phase_calls", ctypes.c_int64 * 5),
                ("split_items", ctypes.c_int64), ("brute_units", ctypes.c_int64),
                ("word_items", ctypes.c_int64), ("word_items_wide", ctypes.c_int64)]

PHASES = ["build", "sweep_kernel", "place_kernel", "pass1", "pass2"]


class BTreeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """The loaded libbtree (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbtree.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        L.btree_params_default.restype = ctypes.c_int
        L.btree_params_default.argtypes = [ctypes.POINTER(Params)]
        L.btree_build.restype = ctypes.c_int
        L.btree_build.argtypes = [P, P, P, I64, ctypes.POINTER(Params), P, ctypes.POINTER(P)]
        L.btree_rebuild.restype = ctypes.c_int
        L.btree_rebuild.argtypes = [P, P, P, P, I64, P]
        L.btree_find_neighbors.restype = ctypes.c_int
        L.btree_find_neighbors.argtypes = [P, P, P, P, P, I64, ctypes.POINTER(I64), P]
        L.btree_stats.restype = ctypes.c_int
        L.btree_stats.argtypes = [P, ctypes.POINTER(Stats)]
        L.btree_export.restype = ctypes.c_int
        L.btree_export.argtypes = [P, P, P, P, P, P]
        L.btree_destroy.restype = ctypes.c_int
        L.btree_destroy.argtypes = [P]
        L.btree_last_error.restype = ctypes.c_char_p
        L.btree_last_error.argtypes = []
        L.btree_batch_create.restype = ctypes.c_int
        L.btree_batch_create.argtypes = [ctypes.c_int32, P, ctypes.POINTER(Params),
                                         ctypes.POINTER(P)]
        L.btree_batch_run.restype = ctypes.c_int
        L.btree_batch_run.argtypes = [P, P, P, P, P, P, P, P, I64, P, ctypes.POINTER(I64), P]
        L.btree_batch_stats.restype = ctypes.c_int
        L.btree_batch_stats.argtypes = [P, ctypes.POINTER(Stats)]
        L.btree_batch_destroy.restype = ctypes.c_int
        L.btree_batch_destroy.argtypes = [P]
        L.btree_batch_graph_counts.restype = ctypes.c_int
        L.btree_batch_graph_counts.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
        L.btree_density.restype = ctypes.c_int
        L.btree_density.argtypes = [P, P, P, P, P, P]
        L.btree_adapt_h.restype = ctypes.c_int
        L.btree_adapt_h.argtypes = [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_int32, P,
                                    ctypes.POINTER(ctypes.c_int32), P]
        L.btree_find_neighbors_noalloc.restype = ctypes.c_int
        L.btree_find_neighbors_noalloc.argtypes = [P, P, P, P, I64, ctypes.POINTER(Params), P,
                                                   P, P, I64, ctypes.POINTER(I64), P]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().btree_last_error().decode()


def _check(status):
    if status != BTREE_OK:
        raise BTreeError(status, last_error())


def params(bucket_size=64, alpha=0.5, beta=0.5, max_depth=32, precision="fp32",
           group_size=0, timing=False, exclude_self=False, octree=False) -> Params:
    p = Params()
    _check(lib().btree_params_default(ctypes.byref(p)))
    p.bucket_size = int(bucket_size)
    p.alpha = float(alpha)
    p.beta = float(beta)
    p.max_depth = int(max_depth)
    if precision in ("fp32", "fp32_filter", BTREE_FP32_FILTER):
        p.precision = BTREE_FP32_FILTER
    elif precision in ("fp64", BTREE_FP64):
        p.precision = BTREE_FP64
    else:
        raise ValueError("precision must be 'fp32' or 'fp64'")
    p.group_size = int(group_size)
    p.timing = 1 if timing else 0
    p.exclude_self = 1 if exclude_self else 0
    p.octree = 1 if octree else 0
    return p


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(a, name):
    import torch
    if not isinstance(a, torch.Tensor) or not a.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % name)
    if a.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if a.dim() != 1 or not a.is_contiguous():
        raise ValueError("%s must be a contiguous 1-D tensor" % name)
    return a


class BTree:
    """A b-tree built on the GPU (btree_build) over FP64 coordinates."""

    def __init__(self, x, y, z, bucket_size=64, alpha=0.5, beta=0.5, max_depth=32,
                 precision="fp32", stream=None, timing=False, exclude_self=False,
                 octree=False):
        x = _dev_f64(x, "x")
        y = _dev_f64(y, "y")
        z = _dev_f64(z, "z")
        if not (x.shape == y.shape == z.shape):
            raise ValueError("x, y, z must have the same length")
        self.n = int(x.shape[0])
        self.device = x.device
        self._keep = (x, y, z)
        p = params(bucket_size, alpha, beta, max_depth, precision, timing=timing,
                   exclude_self=exclude_self, octree=octree)
        h = ctypes.c_void_p()
        _check(lib().btree_build(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                 ctypes.c_void_p(z.data_ptr()), self.n, ctypes.byref(p),
                                 _stream(stream), ctypes.byref(h)))
        self._h = h
        self._keep = None

    def rebuild(self, x, y, z, stream=None):
        """BuildTree again over new coordinates, reusing the handle's memory."""
        x = _dev_f64(x, "x")
        y = _dev_f64(y, "y")
        z = _dev_f64(z, "z")
        if not (x.shape == y.shape == z.shape):
            raise ValueError("x, y, z must have the same length")
        self.n = int(x.shape[0])
        _check(lib().btree_rebuild(self._h, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                   self.n, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().btree_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def count(self, h, counts=None, offsets=None, stream=None):
        """Pass 1: (counts int32[n], offsets int64[n+1], total)."""
        import torch
        h = _dev_f64(h, "h")
        if h.shape[0] != self.n:
            raise ValueError("h must have n entries")
        if counts is None:
            counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        if offsets is None:
            offsets = torch.empty(self.n + 1, dtype=torch.int64, device=self.device)
        total = ctypes.c_int64()
        _check(lib().btree_find_neighbors(self._h, ctypes.c_void_p(h.data_ptr()),
                                          ctypes.c_void_p(counts.data_ptr()),
                                          ctypes.c_void_p(offsets.data_ptr()), None, 0,
                                          ctypes.byref(total), _stream(stream)))
        return counts, offsets, int(total.value)

    def fill(self, h, counts, offsets, nbrs, stream=None):
        """Pass 2 into a caller buffer nbrs (int32, >= total entries)."""
        total = ctypes.c_int64()
        _check(lib().btree_find_neighbors(self._h, ctypes.c_void_p(h.data_ptr()),
                                          ctypes.c_void_p(counts.data_ptr()),
                                          ctypes.c_void_p(offsets.data_ptr()),
                                          ctypes.c_void_p(nbrs.data_ptr()), int(nbrs.numel()),
                                          ctypes.byref(total), _stream(stream)))
        return int(total.value)

    def find(self, h, stream=None):
        """FindNeighbors: (counts, offsets, nbrs) as device tensors; row i is
        nbrs[offsets[i]:offsets[i+1]], ascending original indices."""
        import torch
        counts, offsets, total = self.count(h, stream=stream)
        nbrs = torch.empty(max(total, 1), dtype=torch.int32, device=self.device)
        self.fill(h, counts, offsets, nbrs, stream=stream)
        return counts, offsets, nbrs[:total]

    def density(self, h, mass=None, rho=None, counts=None, stream=None):
        """Fused SPH density (btree_density): (rho float64[n], counts int32[n])."""
        import torch
        h = _dev_f64(h, "h")
        if h.shape[0] != self.n:
            raise ValueError("h must have n entries")
        if mass is not None:
            mass = _dev_f64(mass, "mass")
            if mass.shape[0] != self.n:
                raise ValueError("mass must have n entries")
        if rho is None:
            rho = torch.empty(self.n, dtype=torch.float64, device=self.device)
        if counts is None:
            counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(lib().btree_density(self._h, ctypes.c_void_p(h.data_ptr()),
                                   ctypes.c_void_p(mass.data_ptr()) if mass is not None else None,
                                   ctypes.c_void_p(rho.data_ptr()),
                                   ctypes.c_void_p(counts.data_ptr()), _stream(stream)))
        return rho, counts

    def adapt_h(self, h, target, tol=0.0, max_iter=50, counts=None, stream=None):
        """btree_adapt_h: adapts h (device float64[n], overwritten) to the
        target count; returns (counts at the final h, update rounds)."""
        import torch
        h = _dev_f64(h, "h")
        if h.shape[0] != self.n:
            raise ValueError("h must have n entries")
        if counts is None:
            counts = torch.empty(self.n, dtype=torch.int32, device=self.device)
        it = ctypes.c_int32()
        _check(lib().btree_adapt_h(self._h, ctypes.c_void_p(h.data_ptr()), float(target),
                                   float(tol), int(max_iter), ctypes.c_void_p(counts.data_ptr()),
                                   ctypes.byref(it), _stream(stream)))
        return counts, int(it.value)

    def stats(self) -> dict:
        s = Stats()
        _check(lib().btree_stats(self._h, ctypes.byref(s)))
        d = {k: getattr(s, k) for k, _ in Stats._fields_
             if k not in ("b_hist", "phase_ms", "phase_calls")}
        d["b_hist"] = {b: int(c) for b, c in enumerate(s.b_hist) if c}
        d["phase_ms"] = {k: float(s.phase_ms[i]) for i, k in enumerate(PHASES)}
        d["phase_calls"] = {k: int(s.phase_calls[i]) for i, k in enumerate(PHASES)}
        return d

    def export(self, stream=None) -> dict:
        """Leaf layout (memory order) and tree order of the particles (host)."""
        st = self.stats()
        nl = st["n_leaves"]
        beg = np.zeros(max(nl, 1), dtype=np.int32)
        cnt = np.zeros(max(nl, 1), dtype=np.int32)
        dep = np.zeros(max(nl, 1), dtype=np.int32)
        order = np.zeros(max(self.n, 1), dtype=np.int32)
        _check(lib().btree_export(self._h, beg.ctypes.data, cnt.ctypes.data, dep.ctypes.data,
                                  order.ctypes.data, _stream(stream)))
        return {"leaf_beg": beg[:nl], "leaf_cnt": cnt[:nl], "leaf_depth": dep[:nl],
                "order": order[:self.n]}


def _stats_dict(s: Stats) -> dict:
    d = {k: getattr(s, k) for k, _ in Stats._fields_
         if k not in ("b_hist", "phase_ms", "phase_calls")}
    d["b_hist"] = {b: int(c) for b, c in enumerate(s.b_hist) if c}
    return d


class Batch:
    """Many independent particle sets built and searched by one captured
    HIP graph per run (btree_batch_*).  `set_sizes` gives the particles of
    each set; arrays passed to run() hold the sets concatenated."""

    def __init__(self, set_sizes, params_per_set=None, precision="fp32", **kw):
        sizes = np.asarray(set_sizes, dtype=np.int64)
        if sizes.ndim != 1 or len(sizes) < 1 or (sizes < 0).any():
            raise ValueError("set_sizes must be a non-empty list of sizes >= 0")
        self.nsets = int(len(sizes))
        self.set_offsets = np.zeros(self.nsets + 1, dtype=np.int64)
        np.cumsum(sizes, out=self.set_offsets[1:])
        self.n = int(self.set_offsets[-1])
        if params_per_set is None:
            params_per_set = [dict(kw)] * self.nsets
        if len(params_per_set) != self.nsets:
            raise ValueError("params_per_set needs one entry per set")
        arr = (Params * self.nsets)()
        for k, d in enumerate(params_per_set):
            d = dict(kw, **d)  # keyword arguments apply to every set unless overridden
            d.setdefault("precision", precision)
            arr[k] = params(**d)
        self._params = arr
        h = ctypes.c_void_p()
        _check(lib().btree_batch_create(self.nsets, self.set_offsets.ctypes.data, arr,
                                        ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().btree_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def run(self, x, y, z, h, counts, offsets, nbrs, stream=None):
        """One batched run into caller buffers; returns (totals per set as
        numpy int64, total).  Raises BTreeError (status EOVERFLOW) when nbrs
        is too small; counts and offsets are then valid."""
        for a, nm in ((x, "x"), (y, "y"), (z, "z"), (h, "h")):
            _dev_f64(a, nm)
            if a.shape[0] != self.n:
                raise ValueError("%s must have %d entries" % (nm, self.n))
        totals = np.zeros(self.nsets, dtype=np.int64)
        total = ctypes.c_int64()
        st = lib().btree_batch_run(self._h, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                   ctypes.c_void_p(h.data_ptr()),
                                   ctypes.c_void_p(counts.data_ptr()),
                                   ctypes.c_void_p(offsets.data_ptr()),
                                   ctypes.c_void_p(nbrs.data_ptr()), int(nbrs.numel()),
                                   totals.ctypes.data, ctypes.byref(total), _stream(stream))
        self.last_totals = totals
        self.last_total = int(total.value)
        _check(st)
        return totals, int(total.value)

    def find(self, x, y, z, h, stream=None):
        """Batched FindNeighbors with outputs allocated here: (counts,
        offsets, nbrs, totals).  Rows of set k are rows set_offsets[k]..;
        their indices are local to set k."""
        import torch
        dev = x.device
        counts = torch.empty(max(self.n, 1), dtype=torch.int32, device=dev)
        offsets = torch.empty(self.n + 1, dtype=torch.int64, device=dev)
        nbrs = torch.empty(max(getattr(self, "_cap", 1), 1), dtype=torch.int32, device=dev)
        try:
            totals, total = self.run(x, y, z, h, counts, offsets, nbrs, stream)
        except BTreeError as e:
            if e.status != BTREE_EOVERFLOW:
                raise
            self._cap = self.last_total + self.last_total // 8 + 1024
            nbrs = torch.empty(self._cap, dtype=torch.int32, device=dev)
            totals, total = self.run(x, y, z, h, counts, offsets, nbrs, stream)
        return counts[:self.n], offsets, nbrs[:total], totals

    def stats(self) -> dict:
        s = Stats()
        _check(lib().btree_batch_stats(self._h, ctypes.byref(s)))
        d = _stats_dict(s)
        d["phase_ms"] = {k: float(s.phase_ms[i]) for i, k in enumerate(PHASES)}
        d["phase_calls"] = {k: int(s.phase_calls[i]) for i, k in enumerate(PHASES)}
        la, rec = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().btree_batch_graph_counts(self._h, ctypes.byref(la), ctypes.byref(rec)))
        d["graph_launches"] = int(la.value)
        d["graph_captures"] = int(rec.value)
        return d


def find_neighbors(x, y, z, h, bucket_size=64, alpha=0.5, beta=0.5, max_depth=32,
                   precision="fp32", stream=None):
    """BuildTree + FindNeighbors in one call; returns (counts, offsets, nbrs)."""
    with BTree(x, y, z, bucket_size, alpha, beta, max_depth, precision, stream) as t:
        return t.find(h, stream=stream)


def find_neighbors_noalloc(x, y, z, h, counts, offsets, nbrs, bucket_size=64, alpha=0.5,
                           beta=0.5, max_depth=32, precision="fp32", stream=None,
                           exclude_self=False, octree=False):
    """btree_find_neighbors_noalloc into caller buffers (counts int32[n],
    offsets int64[n+1], nbrs int32 of any capacity, or None): BuildTree and
    FindNeighbors with no device allocation.  Returns the total; raises
    BTreeError (EOVERFLOW when nbrs is too small: counts and offsets are then
    valid and the error's `total` holds the total)."""
    n = int(x.shape[0])
    for a, nm in ((x, "x"), (y, "y"), (z, "z"), (h, "h")):
        _dev_f64(a, nm)
        if a.shape[0] != n:
            raise ValueError("x, y, z, h must have the same length")
    p = params(bucket_size, alpha, beta, max_depth, precision, exclude_self=exclude_self,
               octree=octree)
    total = ctypes.c_int64()
    cap = int(nbrs.numel()) if nbrs is not None else 0
    st = lib().btree_find_neighbors_noalloc(
        ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
        ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(h.data_ptr()), n, ctypes.byref(p),
        ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
        ctypes.c_void_p(nbrs.data_ptr()) if nbrs is not None else None, cap,
        ctypes.byref(total), _stream(stream))
    if st != BTREE_OK:
        e = BTreeError(st, last_error())
        e.total = int(total.value)
        raise e
    return int(total.value)
