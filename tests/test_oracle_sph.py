"""Pins of the oracle's SPH uses of the lists: the density sum (cubic-spline
kernel, support 2h) and the adaptation of h to a target neighbour count.
Each pin is a fact that does not come from the oracle's own code: the
kernel's normalisation by quadrature, its closed-form values, hand-built
configurations, a lattice's density, and the geometry a converged h must
satisfy (checked with the brute-force counts)."""
import math

import numpy as np
import pytest

from paper_1910_02639_amd import workloads as W


def test_shape_values(oracle_mod):
    o = oracle_mod
    assert o.sph_shape(0.0, 1.0) == 1.0
    assert o.sph_shape(0.25, 1.0) == 0.71875          # q = 1/2: 1 - 3/8 + 3/32
    assert o.sph_shape(1.0, 1.0) == 0.25              # q = 1 from the outer branch
    assert abs(o.sph_shape((1.0 - 1e-12) ** 2, 1.0) - 0.25) < 1e-11  # continuous at q = 1
    assert o.sph_shape(2.25, 1.0) == 0.03125          # q = 3/2: (1/4)(1/2)^3
    assert o.sph_shape(4.0, 1.0) == 0.0               # q = 2: edge of the support
    assert o.sph_shape(9.0, 1.0) == 0.0
    assert o.sph_shape(4.0 * 0.36, 0.6) == 0.0        # q = 2 at another h


def test_kernel_normalised(oracle_mod):
    """W(r, h) = w(r/h) / (pi h^3) integrates to 1 over space."""
    from scipy.integrate import quad
    for h in (1.0, 0.37):
        f = lambda r: 4.0 * math.pi * r * r * oracle_mod.sph_shape(r * r, h) / (math.pi * h ** 3)
        v1, _ = quad(f, 0.0, h, epsabs=1e-14, epsrel=1e-13)
        v2, _ = quad(f, h, 2.0 * h, epsabs=1e-14, epsrel=1e-13)
        assert abs(v1 + v2 - 1.0) < 1e-11


def test_density_closed_forms(oracle_mod):
    o = oracle_mod
    h = 0.5
    # an isolated particle: its own term only
    x, y, z = np.array([0.0, 10.0]), np.array([0.0, 0.0]), np.array([0.0, 0.0])
    rho, c = o.density(x, y, z, np.array([h, h]), mass=np.array([3.0, 1.0]))
    assert list(c) == [1, 1]
    assert rho[0] == 3.0 / (math.pi * h ** 3)
    # a centre with six neighbours on the axes at q = 1/2, and one at q = 3/2
    a = 0.5 * h
    px = [0.0, a, -a, 0, 0, 0, 0, 1.5 * h]
    py = [0.0, 0, 0, a, -a, 0, 0, 0.0]
    pz = [0.0, 0, 0, 0, 0, a, -a, 0.0]
    m = np.array([2.0, 1, 1, 1, 1, 1, 1, 4.0])
    hh = np.full(8, h)
    hh[1:] = 0.01  # the others see only themselves
    rho, c = o.density(px, py, pz, hh, mass=m)
    want = (2.0 + 6 * 0.71875 + 4.0 * 0.03125) / (math.pi * h ** 3)
    assert c[0] == 8 and abs(rho[0] - want) <= 4e-16 * want
    rho, c = o.density(px, py, pz, hh, mass=m, exclude_self=True)
    want = (6 * 0.71875 + 4.0 * 0.03125) / (math.pi * h ** 3)
    assert c[0] == 7 and abs(rho[0] - want) <= 4e-16 * want
    assert c[1] == 0 and rho[1] == 0.0
    # h = 0: empty row, density 0
    rho, c = o.density(px, py, pz, np.zeros(8))
    assert not c.any() and not rho.any()


def test_density_of_a_lattice(oracle_mod):
    """Unit masses on a lattice of spacing a: interior densities are the
    number density 1/a^3 within the SPH summation error (about 1 % at
    2h = 2.88 spacings)."""
    m = 24
    x, y, z, h = W.lattice(m, 0, jitter=0.0)
    rho, c = oracle_mod.density(x, y, z, h)
    i = np.arange(m ** 3)
    ix, iy, iz = i // (m * m), (i // m) % m, i % m
    inner = (np.minimum.reduce([ix, iy, iz, m - 1 - ix, m - 1 - iy, m - 1 - iz]) >= 3)
    dens = m ** 3
    assert np.all(np.abs(rho[inner] / dens - 1.0) < 0.02)
    assert np.ptp(rho[inner]) < 1e-9 * dens  # every interior particle sees the same shells


def test_density_rows_match_brute_force(oracle_mod):
    """The density's rows (cell list) are the brute-force rows: same counts."""
    x, y, z, h = W.plummer(3000, 9)
    rho, c = oracle_mod.density(x, y, z, h)
    assert np.array_equal(c, oracle_mod.counts(x, y, z, h))


def test_adapt_h_chain(oracle_mod):
    """Five particles one apart on a line, target 3 neighbours (self
    included), tol 0: an interior particle needs 1 < 2h <= 2, an end one
    2 < 2h <= 3 (and the middle one too: 1 < 2h <= 2)."""
    x = np.arange(5, dtype=np.float64)
    zero = np.zeros(5)
    h, c, it = oracle_mod.adapt_h(x, zero, zero, np.full(5, 0.2), 3, 0, 100)
    assert list(c) == [3] * 5 and 0 < it < 100
    assert np.all(oracle_mod.counts(x, zero, zero, h) == 3)
    R = 2 * h
    assert np.all((R[1:4] > 1) & (R[1:4] <= 2))
    assert (R[0] > 2) & (R[0] <= 3) and (R[4] > 2) & (R[4] <= 3)


@pytest.mark.parametrize("gen,T,tol,scale", [("cube", 64, 2, 0.5), ("cube", 100, 0, 1.3),
                                            ("plummer", 100, 3, 0.7), ("lattice", 100, 0, 0.5)])
def test_adapt_h_converges(oracle_mod, gen, T, tol, scale):
    if gen == "cube":
        x, y, z, h = W.uniform_cube(8000, 3, 64.0)
    elif gen == "plummer":
        x, y, z, h = W.plummer(8000, 4)
    else:
        x, y, z, h = W.lattice(20, 0)
    h0 = h * scale
    hf, c, it = oracle_mod.adapt_h(x, y, z, h0, T, tol, 60)
    assert it < 60
    bc = oracle_mod.counts(x, y, z, hf)
    assert np.array_equal(bc, c)
    assert np.all(np.abs(bc - T) <= tol)
    # a second call starts converged: no round, h unchanged
    h2, c2, it2 = oracle_mod.adapt_h(x, y, z, hf, T, tol, 60)
    assert it2 == 0 and np.array_equal(h2, hf)


def test_adapt_h_zero_h_stays(oracle_mod):
    x, y, z, h = W.uniform_cube(500, 5, 20.0)
    h = h.copy()
    h[::10] = 0.0
    hf, c, it = oracle_mod.adapt_h(x, y, z, h, 20, 2, 60)
    assert np.all(hf[::10] == 0.0) and np.all(c[::10] == 0)
    assert it < 60
