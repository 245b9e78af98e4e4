"""Seeded synthetic particle sets shaped like the paper's test cases.

The paper measures on an Evrard-collapse snapshot (non-uniform, 10^6
particles, ~100 neighbours) and a Square-Patch snapshot (near-uniform, 10^7
particles, ~500 neighbours) (Section 4.1, Table 3).  Neither snapshot is
available, so these generators stand in for them: a Plummer sphere for the
centrally condensed case, a uniform cube and a jittered lattice for the
near-uniform case, and a batch of uneven sets.

This module holds no part of the search: it only draws inputs, with
``numpy.random.default_rng(seed)`` (PCG64) in FP64.  Both the GPU path and
the CPU oracle consume the same arrays.  Every generator returns
``(x, y, z, h)`` as contiguous float64 arrays.
"""
from __future__ import annotations

import math

import numpy as np

# Plummer sphere, scale radius a = 1, total mass M = 1, truncated at r <= 10.
PLUMMER_RMAX = 10.0
PLUMMER_MCUT = PLUMMER_RMAX ** 3 / (1.0 + PLUMMER_RMAX ** 2) ** 1.5  # M(<10)


def const_h(n: int, neighbours: float) -> float:
    """h such that (4/3) pi (2h)^3 n = neighbours (unit volume)."""
    return 0.5 * (neighbours / ((4.0 / 3.0) * math.pi * n)) ** (1.0 / 3.0)


def uniform_cube(n: int, seed: int = 0, neighbours: float = 64.0):
    """n points uniform in [0,1)^3 with constant h giving ~neighbours."""
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    x = np.ascontiguousarray(pos[:, 0])
    y = np.ascontiguousarray(pos[:, 1])
    z = np.ascontiguousarray(pos[:, 2])
    h = np.full(n, const_h(n, neighbours), dtype=np.float64)
    return x, y, z, h


def lattice(m: int = 100, seed: int = 0, jitter: float = 1e-4,
            neighbours: float = 100.0):
    """m^3 cubic lattice in the unit cube, point (i+0.5)/m per axis plus a
    uniform jitter in [-jitter, jitter) per coordinate (1% of the spacing
    for m = 100).  Index of lattice point (ix, iy, iz) is (ix*m + iy)*m + iz.
    Constant h giving ~neighbours."""
    rng = np.random.default_rng(seed)
    n = m ** 3
    i = np.arange(n, dtype=np.int64)
    ix, iy, iz = i // (m * m), (i // m) % m, i % m
    j = rng.uniform(-jitter, jitter, size=(n, 3))
    x = (ix + 0.5) / m + j[:, 0]
    y = (iy + 0.5) / m + j[:, 1]
    z = (iz + 0.5) / m + j[:, 2]
    h = np.full(n, const_h(n, neighbours), dtype=np.float64)
    return (np.ascontiguousarray(x), np.ascontiguousarray(y),
            np.ascontiguousarray(z), h)


def plummer_h(n: int, r: np.ndarray, neighbours: float = 100.0) -> np.ndarray:
    """h_i = 0.5 * (neighbours / ((4/3) pi n rho(r_i)))^(1/3) with the
    untruncated Plummer density rho(r) = (3 / 4 pi) (1 + r^2)^(-5/2)."""
    return 0.5 * (neighbours / n) ** (1.0 / 3.0) * (1.0 + r * r) ** (5.0 / 6.0)


def plummer(n: int, seed: int = 0, neighbours: float = 100.0):
    """Plummer sphere (a = 1) truncated at r <= 10 by inverse transform:
    m ~ U(0, M(10)), r = (m^(-2/3) - 1)^(-1/2), then an isotropic direction
    (cos theta ~ U(-1, 1), phi ~ U(0, 2 pi)), drawn in that order."""
    rng = np.random.default_rng(seed)
    m = rng.uniform(0.0, PLUMMER_MCUT, n)
    cos_t = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    with np.errstate(divide="ignore"):
        r = 1.0 / np.sqrt(np.power(m, -2.0 / 3.0) - 1.0)
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    x = r * sin_t * np.cos(phi)
    y = r * sin_t * np.sin(phi)
    z = r * cos_t
    h = plummer_h(n, r, neighbours)
    return (np.ascontiguousarray(x), np.ascontiguousarray(y),
            np.ascontiguousarray(z), np.ascontiguousarray(h))


def batch_sizes(nsets: int = 64, seed: int = 0, lo: float = 4.0, hi: float = 6.0):
    """Set sizes log-uniform in [10^lo, 10^hi], rounded to integers."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(lo, hi, nsets)
    return [int(round(10.0 ** v)) for v in e]


def batch(nsets: int = 64, seed: int = 0, lo: float = 4.0, hi: float = 6.0):
    """Independent sets of uneven size: even k uniform cube (64 neighbours),
    odd k Plummer (100 neighbours), set k drawn with seed 1000 + k.
    Returns a list of (x, y, z, h) tuples."""
    sets = []
    for k, n in enumerate(batch_sizes(nsets, seed, lo, hi)):
        if k % 2 == 0:
            sets.append(uniform_cube(n, 1000 + k, 64.0))
        else:
            sets.append(plummer(n, 1000 + k, 100.0))
    return sets


WORKLOADS = {
    # name: (generator, kwargs, bucket size)
    "U10k": (uniform_cube, dict(n=10_000, seed=0, neighbours=64.0), 64),
    "L1M": (lattice, dict(m=100, seed=0), 128),
    "P8M": (plummer, dict(n=8_000_000, seed=0), 128),
    "P16M": (plummer, dict(n=16_000_000, seed=0), 128),
}


def make(name: str):
    """Generate one of the named single-set workloads: (x, y, z, h, s)."""
    gen, kw, s = WORKLOADS[name]
    x, y, z, h = gen(**kw)
    return x, y, z, h, s
