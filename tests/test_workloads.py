"""The seeded input generators follow the stated recipe (CPU only): shapes,
ranges, index layout, smoothing-length rules, the Plummer truncation and mass
profile, the Batch64 size mix, and determinism."""
import math

import numpy as np

from paper_1910_02639_amd import workloads as W


def test_uniform_cube_recipe():
    x, y, z, h = W.uniform_cube(10_000, 0, 64.0)
    assert x.shape == (10_000,) and x.dtype == np.float64 and x.flags["C_CONTIGUOUS"]
    for a in (x, y, z):
        assert a.min() >= 0.0 and a.max() < 1.0
    # (4/3) pi (2h)^3 n = 64  ->  2h = 0.1151765...
    assert np.all(h == h[0]) and abs(2 * h[0] - 0.1151765) < 1e-6
    assert abs((4.0 / 3.0) * math.pi * (2 * h[0]) ** 3 * 10_000 - 64.0) < 1e-9


def test_lattice_index_layout_and_jitter():
    x, y, z, h = W.lattice()
    m = 100
    assert x.shape == (m ** 3,)
    for i in (0, 1, m, m * m, 123_456, m ** 3 - 1):
        ix, iy, iz = i // (m * m), (i // m) % m, i % m
        for a, c in ((x, ix), (y, iy), (z, iz)):
            assert abs(a[i] - (c + 0.5) / m) <= 1e-4
    j = x - (np.arange(m ** 3) // (m * m) + 0.5) / m
    assert np.abs(j).max() <= 1e-4 and np.abs(j).max() > 0.9e-4
    assert abs(2 * h[0] - 0.02879412) < 1e-7


def test_plummer_truncation_profile_and_h():
    n = 200_000
    x, y, z, h = W.plummer(n, 5)
    r = np.sqrt(x * x + y * y + z * z)
    assert r.max() <= 10.0 + 1e-9
    # Mass inside r = 1 over the mass inside the truncation radius.
    f1 = (1.0 / 2.0 ** 1.5) / W.PLUMMER_MCUT
    assert abs(np.mean(r <= 1.0) - f1) < 0.005
    # Isotropy: the mean direction is near zero.
    assert abs(np.mean(z / r)) < 0.01 and abs(np.mean(x / r)) < 0.01
    assert np.allclose(h, 0.5 * (100.0 / n) ** (1 / 3) * (1 + r * r) ** (5 / 6), rtol=1e-12)
    # The 8M sphere's h range follows from the same rule: [0.0116, 0.543].
    lo, hi = W.plummer_h(8_000_000, np.array([0.0, 10.0]))
    assert abs(lo - 0.0116) < 5e-5 and abs(hi - 0.543) < 5e-4


def test_batch64_size_mix():
    sizes = W.batch_sizes(64, 0)
    assert len(sizes) == 64
    assert all(10 ** 4 <= s <= 10 ** 6 for s in sizes)
    assert sum(sizes) == 13_484_554
    e = np.log10(sizes)
    assert 4.6 < e.mean() < 5.4  # log-uniform on [4, 6]


def test_batch_kinds_and_determinism():
    sets = W.batch(6, 0, 3.0, 3.5)
    for k, (x, y, z, h) in enumerate(sets):
        if k % 2 == 0:
            assert np.all(h == h[0]) and x.min() >= 0.0 and x.max() < 1.0
        else:
            assert h.std() > 0.0
    again = W.batch(6, 0, 3.0, 3.5)
    for a, b in zip(sets, again):
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
