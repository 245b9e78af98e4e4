"""CPU oracle for the b-tree neighbour search (arXiv 1910.02639).

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  Nothing here is
shared with, imported by, or imports the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, FP64, no FMA contraction):

* ``lists`` / ``counts`` / ``row``: the definition of FindNeighbors' result
  (Section 3.2, Algorithm 2): for each query i, every j with
  ``((dx*dx + dy*dy) + dz*dz) < (2*h_i)*(2*h_i)``, ascending in j.
* ``cell_lists`` / ``cell_check``: the same lists by an exact multi-resolution
  cell list (every tested pair through the same predicate), for sets too
  large for the brute force; ``cell_check`` compares lists produced
  elsewhere row by row.  Pinned to the brute force byte for byte.
* ``build_tree``: Algorithm 1 (BuildTree) with Eqs. 1-4, as a recursion in
  the paper's order, reporting the tree shape and each leaf's members in a
  canonical depth-first order; ``octree=True`` gives the classical octree
  (b = 2 at every split) the paper compares against.
* ``eq1_branching``, ``eq2_subcell``, ``eq3_cell_id``, ``eq5_range``: the
  equations of Section 3, one function each.
* ``sph_shape`` / ``density``: the SPH density sum over each row (the use of
  the search inside an SPH code, Section 4.7; cubic-spline kernel of
  support 2h, since the paper fixes none), terms added in ascending j.
* ``adapt_h``: smoothing lengths driven to a target neighbour count (the
  target of Table 3): each particle repeats c = its count at h, and while
  |c - T| > tol records h as the low (c < T) or high end of a bracket and
  takes h min(2, (5c + T) / (6c)) (2 when c = 0), or the bracket's midpoint
  if that leaves the bracket.

Parity is pinned by tests/test_oracle.py against closed forms, the paper's
worked examples, invariants and an independent k-d tree (scipy).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into _oracle.so (gcc, -ffp-contract=off, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        lib.oracle_pair.restype = ctypes.c_int
        lib.oracle_pair.argtypes = [D] * 7
        lib.oracle_row.restype = I64
        lib.oracle_row.argtypes = [P, P, P, P, I64, I64, P, I64]
        lib.oracle_counts.restype = None
        lib.oracle_counts.argtypes = [P, P, P, P, I64, P, I64, P]
        lib.oracle_lists.restype = I64
        lib.oracle_lists.argtypes = [P, P, P, P, I64, P, I64, P, P, I64]
        lib.oracle_eq1_branching.restype = I64
        lib.oracle_eq1_branching.argtypes = [I64, I64]
        lib.oracle_eq2_subcell.restype = I64
        lib.oracle_eq2_subcell.argtypes = [D, D, D, I64]
        lib.oracle_eq3_cell_id.restype = I64
        lib.oracle_eq3_cell_id.argtypes = [I64, I64, I64, I64]
        lib.oracle_eq5_range.restype = None
        lib.oracle_eq5_range.argtypes = [D, D, D, D, I64, P, P]
        lib.oracle_build_tree.restype = None
        lib.oracle_build_tree.argtypes = [P, P, P, I64, I64, D, D, ctypes.c_int32,
                                          ctypes.c_int32,
                                          P, P, I64, P, P, I64, P, P, P, I64, P]
        lib.oracle_cell_lists.restype = I64
        lib.oracle_cell_lists.argtypes = [P, P, P, P, I64, P, P, P, I64]
        lib.oracle_sph_shape.restype = D
        lib.oracle_sph_shape.argtypes = [D, D]
        lib.oracle_density.restype = I64
        lib.oracle_density.argtypes = [P, P, P, P, P, I64, ctypes.c_int32, P, P]
        lib.oracle_cell_check.restype = I64
        lib.oracle_cell_check.argtypes = [P, P, P, P, I64, P, P, P, P, I64]
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def pair(xi, yi, zi, hi, xj, yj, zj) -> bool:
    """P64(i, j) for one pair of points."""
    return bool(_load().oracle_pair(xi, yi, zi, hi, xj, yj, zj))


def row(x, y, z, h, i: int) -> np.ndarray:
    """Row i of the neighbour lists (ascending original indices)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.shape[0]
    lib = _load()
    k = lib.oracle_row(_ptr(x), _ptr(y), _ptr(z), _ptr(h), n, int(i), None, 0)
    out = np.empty(max(k, 1), dtype=np.int32)
    lib.oracle_row(_ptr(x), _ptr(y), _ptr(z), _ptr(h), n, int(i), _ptr(out), k)
    return out[:k]


def counts(x, y, z, h, rows=None) -> np.ndarray:
    """Neighbour counts (int64) of the given rows (all rows by default)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.shape[0]
    if rows is None:
        m, rp = n, None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        m, rp = rows.shape[0], _ptr(rows)
    out = np.empty(max(m, 1), dtype=np.int64)
    _load().oracle_counts(_ptr(x), _ptr(y), _ptr(z), _ptr(h), n, rp, m, _ptr(out))
    return out[:m]


def lists(x, y, z, h, rows=None):
    """CSR lists of the given rows: (counts int64, offsets int64, nbrs int32)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.shape[0]
    if rows is None:
        m, rp = n, None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        m, rp = rows.shape[0], _ptr(rows)
    c = counts(x, y, z, h, rows)
    total = int(c.sum())
    offsets = np.empty(m + 1, dtype=np.int64)
    nbrs = np.empty(max(total, 1), dtype=np.int32)
    got = _load().oracle_lists(_ptr(x), _ptr(y), _ptr(z), _ptr(h), n, rp, m,
                               _ptr(offsets), _ptr(nbrs), total)
    assert got == total
    return c, offsets, nbrs[:total]


def cell_lists(x, y, z, h):
    """All rows by the cell list: (counts int64, offsets int64, nbrs int32)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.shape[0]
    lib = _load()
    c = np.empty(max(n, 1), dtype=np.int64)
    o = np.empty(n + 1, dtype=np.int64)
    got = lib.oracle_cell_lists(_ptr(x), _ptr(y), _ptr(z), _ptr(h), n, _ptr(c), _ptr(o),
                                None, 0)
    if got < 0:
        raise MemoryError("oracle cell list: out of memory")
    total = int(o[n])
    nbrs = np.empty(max(total, 1), dtype=np.int32)
    got = lib.oracle_cell_lists(_ptr(x), _ptr(y), _ptr(z), _ptr(h), n, _ptr(c), _ptr(o),
                                _ptr(nbrs), total)
    if got != total:
        raise MemoryError("oracle cell list: out of memory")
    return c[:n], o, nbrs[:total]


def cell_check(x, y, z, h, counts, offsets, nbrs, max_bad: int = 64):
    """Compares lists produced elsewhere (counts int32[n], offsets int64[n+1],
    nbrs int32) with the cell list, row by row.  Returns (number of wrong
    rows, sorted array of up to max_bad of them)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.shape[0]
    counts = np.ascontiguousarray(counts, dtype=np.int32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    nbrs = np.ascontiguousarray(nbrs, dtype=np.int32)
    if counts.shape[0] != n or offsets.shape[0] != n + 1:
        raise ValueError("counts must have n and offsets n + 1 entries")
    if n and (offsets[-1] > nbrs.shape[0] or offsets.min() < 0
              or (np.diff(offsets) < 0).any()):
        return n, np.arange(min(n, max_bad), dtype=np.int64)
    nb = nbrs if nbrs.shape[0] else np.zeros(1, dtype=np.int32)
    bad = np.empty(max(max_bad, 1), dtype=np.int64)
    k = _load().oracle_cell_check(_ptr(x), _ptr(y), _ptr(z), _ptr(h), n, _ptr(counts),
                                  _ptr(offsets), _ptr(nb), _ptr(bad), max_bad)
    if k < 0:
        raise MemoryError("oracle cell check: out of memory")
    return int(k), np.sort(bad[:min(k, max_bad)])


def cell_counts(x, y, z, h) -> np.ndarray:
    """Row lengths of all rows by the cell list (int64)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.shape[0]
    c = np.empty(max(n, 1), dtype=np.int64)
    o = np.empty(n + 1, dtype=np.int64)
    if _load().oracle_cell_lists(_ptr(x), _ptr(y), _ptr(z), _ptr(h), n, _ptr(c), _ptr(o),
                                 None, 0) < 0:
        raise MemoryError("oracle cell list: out of memory")
    return c[:n]


def sph_shape(d2: float, h: float) -> float:
    """Cubic-spline shape w(sqrt(d2) / h); W = w / (pi h^3)."""
    return float(_load().oracle_sph_shape(float(d2), float(h)))


def density(x, y, z, h, mass=None, exclude_self=False):
    """SPH density of every particle over its row: (rho float64, counts int64)."""
    x, y, z, h = map(_f64, (x, y, z, h))
    n = x.shape[0]
    m = None if mass is None else _f64(mass)
    rho = np.empty(max(n, 1), dtype=np.float64)
    c = np.empty(max(n, 1), dtype=np.int64)
    if _load().oracle_density(_ptr(x), _ptr(y), _ptr(z), _ptr(h),
                              _ptr(m) if m is not None else None, n,
                              1 if exclude_self else 0, _ptr(rho), _ptr(c)) < 0:
        raise MemoryError("oracle density: out of memory")
    return rho[:n], c[:n]


def adapt_h(x, y, z, h, target, tol=0.0, max_iter=50, exclude_self=False):
    """Smoothing lengths driven to a target count.  Every particle, on its
    own: c = its row length at its h; if |c - target| <= tol it is done;
    else h is recorded as the low end (c < target) or high end (c > target)
    of the particle's bracket (initially 0 and +inf) and replaced by
    h f, f = min(2, (5c + target) / (6c)) (f = 2 when c = 0), or by the
    bracket's midpoint (lo + hi) * 0.5 when h f is not strictly inside the
    bracket; one rounding per operation.  Rounds stop when no h changes or
    after max_iter.  A particle with h = 0 keeps it.  Returns (h, counts at
    the final h, rounds made)."""
    h = _f64(h).copy()
    T = float(target)
    lo = np.zeros_like(h)
    hi = np.full_like(h, np.inf)

    def count(hh):
        c = cell_counts(x, y, z, hh)
        if exclude_self:
            c = c - ((2.0 * hh) * (2.0 * hh) > 0.0)
        return c.astype(np.float64)

    c = count(h)
    it = 0
    while it < max_iter:
        off = (np.abs(c - T) > tol) & (h != 0.0)  # h = 0 cannot move
        if not off.any():
            break
        cc, hv, lb, ub = c[off], h[off], lo[off], hi[off]
        below = cc < T
        lb = np.where(below, hv, lb)
        ub = np.where(below, ub, hv)
        f = np.full(cc.shape, 2.0)
        pos = cc > 0.0
        f[pos] = np.minimum(2.0, (5.0 * cc[pos] + T) / (6.0 * cc[pos]))
        p = hv * f
        out = (p >= ub) | (p <= lb)
        p = np.where(out, (lb + ub) * 0.5, p)
        h[off], lo[off], hi[off] = p, lb, ub
        it += 1
        c = count(h)
    return h, c.astype(np.int64), it


def eq1_branching(n: int, s: int) -> int:
    return int(_load().oracle_eq1_branching(int(n), int(s)))


def eq2_subcell(x: float, lo: float, hi: float, b: int) -> int:
    return int(_load().oracle_eq2_subcell(float(x), float(lo), float(hi), int(b)))


def eq3_cell_id(c1: int, c2: int, c3: int, b: int) -> int:
    return int(_load().oracle_eq3_cell_id(int(c1), int(c2), int(c3), int(b)))


def eq5_range(x: float, R: float, lo: float, hi: float, b: int):
    a = ctypes.c_int64()
    c = ctypes.c_int64()
    _load().oracle_eq5_range(float(x), float(R), float(lo), float(hi), int(b),
                             ctypes.byref(a), ctypes.byref(c))
    return a.value, c.value


class Tree:
    """Result of Algorithm 1: shape statistics and canonical leaves."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    def leaf_offsets(self) -> np.ndarray:
        off = np.zeros(self.n_leaves + 1, dtype=np.int64)
        np.cumsum(self.leaf_cnt, out=off[1:])
        return off


def build_tree(x, y, z, s: int = 64, alpha: float = 0.5, beta: float = 0.5,
               max_depth: int = 32, octree: bool = False) -> Tree:
    """Algorithm 1 on all particles; leaves in canonical depth-first order
    (sub-cells in Morton order of their coordinates), members ascending.
    octree=True: b = 2 at every split (the classical octree)."""
    x, y, z = map(_f64, (x, y, z))
    n = x.shape[0]
    leaf_cap = max(n, 1)
    node_cap = max(n, 1)
    bh_len = 1 << 16
    leaf_cnt = np.zeros(leaf_cap, dtype=np.int64)
    leaf_depth = np.zeros(leaf_cap, dtype=np.int32)
    members = np.zeros(max(n, 1), dtype=np.int32)
    b_hist = np.zeros(bh_len, dtype=np.int64)
    node_b = np.zeros(node_cap, dtype=np.int32)
    node_n = np.zeros(node_cap, dtype=np.int64)
    node_depth = np.zeros(node_cap, dtype=np.int32)
    stats = np.zeros(8, dtype=np.int64)
    _load().oracle_build_tree(_ptr(x), _ptr(y), _ptr(z), n, int(s), float(alpha),
                              float(beta), int(max_depth), 1 if octree else 0,
                              _ptr(leaf_cnt),
                              _ptr(leaf_depth), leaf_cap, _ptr(members),
                              _ptr(b_hist), bh_len, _ptr(node_b), _ptr(node_n),
                              _ptr(node_depth), node_cap, _ptr(stats))
    if stats[6]:
        raise RuntimeError("oracle build_tree: capacity exceeded")
    ni, nl = int(stats[0]), int(stats[1])
    bh = {int(b): int(c) for b, c in enumerate(b_hist) if c}
    return Tree(n_internal=ni, n_leaves=nl, depth=int(stats[2]),
                rounds=int(stats[3]), max_leaf=int(stats[4]),
                leaf_cnt=leaf_cnt[:nl].copy(), leaf_depth=leaf_depth[:nl].copy(),
                members=members[:int(stats[5])].copy(), b_hist=bh,
                node_b=node_b[:ni].copy(), node_n=node_n[:ni].copy(),
                node_depth=node_depth[:ni].copy())
