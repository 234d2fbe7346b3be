"""Pins for the Stratmann-Scuseria-Frisch partition (Sec. 2.2,
eq. atomic_partition and eq. num_int)."""
import math

import numpy as np

import oracle
from workloads import lebedev_table, water_cluster, water


def test_cell_function_shape():
    """g is odd, reaches -1 and +1 at mu = -a and a with zero slope there,
    and s = (1 - g)/2 decreases from 1 to 0 with s(0) = 1/2."""
    a = 0.64
    mu = np.linspace(-1, 1, 2001)
    s = oracle.ssf_cell(mu, a)
    assert np.all(np.diff(s) <= 1e-16)
    assert s[0] == 1.0 and s[-1] == 0.0 and abs(s[1000] - 0.5) < 1e-15
    assert np.allclose(s + oracle.ssf_cell(-mu, a), 1.0, atol=1e-15)
    h = 1e-6
    for edge in (-a, a):
        inner = edge - math.copysign(h, edge)
        assert abs(oracle.ssf_cell(np.array([inner]), a)[0]
                   - oracle.ssf_cell(np.array([edge]), a)[0]) < 1e-12
    # continuity just inside the edges: 1 - g ~ (1 - z)^4
    z = 1 - 1e-3
    assert oracle.ssf_cell(np.array([a * z]), a)[0] < 1e-9


def test_partition_of_unity_and_nuclei():
    mol = water_cluster(4, box=9.0, min_oo=4.5, seed=3)
    rng = np.random.default_rng(0)
    pts = rng.uniform(-2, 11, size=(500, 3))
    p = oracle.ssf_partition(pts, mol.coords)
    assert np.allclose(p.sum(1), 1.0, atol=1e-14)
    assert np.all(p >= 0)
    pn = oracle.ssf_partition(mol.coords, mol.coords)
    assert np.allclose(pn, np.eye(mol.natoms), atol=1e-15)


def test_nearest_neighbour_shortcut_region():
    """Inside |r - R_A| < (1-a)/2 min_B R_AB the partition of A is exactly 1."""
    mol = water()
    a = 0.64
    X = mol.coords
    R = np.linalg.norm(X[:, None] - X[None], axis=2)
    np.fill_diagonal(R, np.inf)
    rng = np.random.default_rng(1)
    for A in range(mol.natoms):
        rad = 0.5 * (1 - a) * R[A].min()
        d = rng.normal(size=(200, 3))
        d *= (rng.uniform(0, 0.999, size=200) * rad / np.linalg.norm(d, axis=1))[:, None]
        p = oracle.ssf_partition(X[A] + d, X, a)
        assert np.all(p[:, A] == 1.0)


def test_two_atom_midplane():
    X = np.array([[0.0, 0, 0], [2.0, 0, 0]])
    pts = np.array([[1.0, y, z] for y in (-1, 0, 3) for z in (0, 2)])
    p = oracle.ssf_partition(pts, X)
    assert np.allclose(p, 0.5, atol=1e-15)


def test_partitioned_grid_integrates_molecular_function():
    """sum_i w_i f(r_i) with SSF weights reproduces the integral of a
    smooth molecular function: int sum_A exp(-|r - R_A|^2) = N_A pi^(3/2).
    A wrong sign or index in mu_AB breaks the partition and this sum."""
    mol = water()
    pts, wq, par = oracle.molecular_grid(mol.coords, np.full(3, 5.0), 75,
                                         lebedev_table(302))
    w = oracle.ssf_weights(pts, wq, par, mol.coords)
    f = sum(np.exp(-((pts - c) ** 2).sum(1)) for c in mol.coords)
    assert abs((w * f).sum() / (3 * math.pi ** 1.5) - 1) < 2e-6
    # the unpartitioned grids triple count
    assert abs((wq * f).sum() / (3 * math.pi ** 1.5) - 1) > 0.1


# --- Becke's partition (Sec. 2.2 lists it among the possible choices) ---
def test_becke_cell_function_shape():
    """s(nu) = (1 - p(p(p(nu))))/2 falls from 1 at nu = -1 to 0 at +1, is
    1/2 at 0, satisfies s(nu) + s(-nu) = 1, and is flat at both ends
    (p'(+-1) = 0)."""
    nu = np.linspace(-1, 1, 2001)
    s = oracle.becke_cell(nu)
    assert s[0] == 1.0 and s[-1] == 0.0 and abs(s[1000] - 0.5) < 1e-15
    assert np.all(np.diff(s) <= 1e-16)
    assert np.allclose(s + oracle.becke_cell(-nu), 1.0, atol=1e-15)
    h = 1e-3
    assert oracle.becke_cell(np.array([1 - h]))[0] < 1e-15
    assert 1.0 - oracle.becke_cell(np.array([-1 + h]))[0] < 1e-15


def test_becke_size_adjustment_antisymmetric_and_bounded():
    r = np.array([0.35, 0.60, 0.70, 0.65, 2.0])
    a = oracle.becke_size_adjustment(r)
    assert np.allclose(a, -a.T, atol=0) and np.all(np.abs(a) <= 0.5)
    assert np.all(np.diag(a) == 0.0)
    assert oracle.becke_size_adjustment(None) is None


def test_becke_partition_of_unity_and_nuclei():
    mol = water_cluster(4, box=9.0, min_oo=4.5, seed=3)
    radii = np.where(mol.Z == 1, 0.35, 0.60)
    rng = np.random.default_rng(5)
    pts = rng.uniform(-2, 11, size=(400, 3))
    for rad in (None, radii):
        p = oracle.becke_partition(pts, mol.coords, rad)
        assert np.allclose(p.sum(1), 1.0, atol=1e-14) and np.all(p >= 0)
        pn = oracle.becke_partition(mol.coords, mol.coords, rad)
        assert np.allclose(pn, np.eye(mol.natoms), atol=1e-15)


def test_becke_two_atom_boundaries():
    """Equal radii: the mid-plane splits 1/2 : 1/2. Radii R_O, R_H: on the
    O-H axis the split falls where r_O / r_H = R_O / R_H (the point of the
    size adjustment), provided |a| < 1/2."""
    X = np.array([[0.0, 0, 0], [2.0, 0, 0]])
    pts = np.array([[1.0, y, z] for y in (-1, 0, 3) for z in (0, 2)])
    assert np.allclose(oracle.becke_partition(pts, X), 0.5, atol=1e-15)
    rO, rH = 0.60, 0.35
    a = oracle.becke_size_adjustment(np.array([rO, rH]))
    assert abs(a[0, 1]) < 0.5
    x = 2.0 * rO / (rO + rH)            # r_O / r_H = rO / rH on the axis
    p = oracle.becke_partition(np.array([[x, 0.0, 0.0]]), X, np.array([rO, rH]))
    assert np.allclose(p, 0.5, atol=1e-14)
    # and without the adjustment the same point belongs mostly to H
    p0 = oracle.becke_partition(np.array([[x, 0.0, 0.0]]), X)
    assert p0[0, 1] > 0.6


def test_becke_grid_integrates_molecular_function():
    mol = water()
    radii = np.where(mol.Z == 1, 0.35, 0.60)
    pts, wq, par = oracle.molecular_grid(mol.coords, np.full(3, 5.0), 75,
                                         lebedev_table(302))
    w = oracle.becke_weights(pts, wq, par, mol.coords, radii)
    f = sum(np.exp(-((pts - c) ** 2).sum(1)) for c in mol.coords)
    assert abs((w * f).sum() / (3 * math.pi ** 1.5) - 1) < 2e-6
