"""Pins for the atom-centred product grid (Sec. 2.2, eq. num_int; Table 2)."""
import math

import numpy as np
import pytest

import oracle
from workloads import lebedev_table


def _dfact(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


@pytest.mark.parametrize("n_ang,degree", [(302, 29), (590, 41), (974, 53)])
def test_lebedev_moment_exactness(n_ang, degree):
    """A Lebedev rule of degree L integrates x^a y^b z^c over the sphere
    exactly for a+b+c <= L: 4 pi (a-1)!!(b-1)!!(c-1)!!/(a+b+c+1)!! for even
    a, b, c and 0 otherwise."""
    t = lebedev_table(n_ang)
    x, y, z, w = t.T
    assert np.allclose(x * x + y * y + z * z, 1.0, atol=1e-15)
    for a in range(degree + 1):
        for b in range(degree + 1 - a):
            for c in range(0, degree + 1 - a - b, 3 if (a + b) > 20 else 1):
                got = float((w * x ** a * y ** b * z ** c).sum())
                if a % 2 or b % 2 or c % 2:
                    exp = 0.0
                else:
                    exp = (4 * math.pi * _dfact(a - 1) * _dfact(b - 1)
                           * _dfact(c - 1) / _dfact(a + b + c + 1))
                assert abs(got - exp) <= 2e-14 * 4 * math.pi, (a, b, c, got, exp)


@pytest.mark.parametrize("n_rad,n_ang,count", [(75, 302, 22650), (99, 590, 58410),
                                               (100, 590, 59000), (175, 974, 170450)])
def test_point_counts(n_rad, n_ang, count):
    """Table 2: N_g^A = N_rad x N_ang (no pruning)."""
    pts, w = oracle.atomic_grid(np.zeros(3), n_rad, 5.0, lebedev_table(n_ang))
    assert pts.shape == (count, 3) and w.shape == (count,)


def test_mura_knowles_gaussian_moments_converge():
    """int_0^inf r^2 exp(-a r^2) dr = sqrt(pi) / (4 a^(3/2)); the MK rule
    converges to it for exponents spanning the basis range."""
    prev = None
    for n in (50, 75, 100, 150):
        r, w = oracle.mura_knowles(n, 5.0)
        errs = np.array([abs((w * np.exp(-a * r * r)).sum()
                             / (math.sqrt(math.pi) / (4 * a ** 1.5)) - 1)
                         for a in (0.04, 0.1, 1.0, 100.0, 5000.0)])
        if prev is not None:
            assert errs.max() <= prev.max() * 1.01
        prev = errs
    assert prev.max() < 1e-7


def test_mura_knowles_nodes():
    """r_k = -alpha ln(1 - x_k^3) on midpoint nodes: strictly increasing,
    positive, with the weights positive."""
    r, w = oracle.mura_knowles(75, 5.0)
    assert np.all(np.diff(r) > 0) and r[0] > 0 and np.all(w > 0)
    x = (np.arange(75) + 0.5) / 75
    assert np.allclose(np.exp(-r / 5.0), 1 - x ** 3, rtol=1e-14)


def test_single_atom_grid_integrates_gaussian():
    """Product grid of one atom: int exp(-a |r|^2) d^3r = (pi/a)^(3/2)."""
    pts, w = oracle.atomic_grid(np.array([0.3, -0.2, 1.0]), 99, 5.0,
                                lebedev_table(590))
    d2 = ((pts - np.array([0.3, -0.2, 1.0])) ** 2).sum(1)
    for a in (0.1, 1.0, 30.0):
        got = (w * np.exp(-a * d2)).sum()
        assert abs(got / (math.pi / a) ** 1.5 - 1) < 1e-9
