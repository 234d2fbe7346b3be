"""The seeded input generators produce the stated shapes."""
import numpy as np

from workloads import (cfg_water, cfg_water_cluster, peptide_chain,
                       cfg_serving_request, water_cluster)
from workloads.basis import make_basis


def test_water_shape():
    w = cfg_water()
    assert w.natoms == 3 and w.nbf == 25
    assert w.n_points_nominal == 3 * 75 * 302 == 67950
    assert abs(np.trace(w.P @ w.S) - 10) < 1e-12
    assert np.all(np.linalg.eigvalsh(w.P) > -1e-12)
    assert np.array_equal(w.P, w.P.T)


def test_cluster_geometry_and_basis_count():
    m = water_cluster(64, box=25.0, seed=2)
    O = m.coords[m.Z == 8]
    D = np.linalg.norm(O[:, None] - O[None], axis=2)
    np.fill_diagonal(D, np.inf)
    assert D.min() >= 5.0 and O.min() >= 0 and O.max() < 25.0
    assert make_basis(m.Z).nbf == 1600
    # rigid waters: O-H distances preserved
    H = m.coords.reshape(64, 3, 3)
    assert np.allclose(np.linalg.norm(H[:, 1] - H[:, 0], axis=1), np.hypot(1.43, 1.11))


def test_chain_composition():
    m = peptide_chain(600, seed=4)
    counts = np.bincount(m.Z, minlength=9)
    assert (counts[6], counts[7], counts[8], counts[1]) == (134, 67, 67, 332)
    D = np.linalg.norm(m.coords[:, None] - m.coords[None], axis=2)
    np.fill_diagonal(D, np.inf)
    assert D.min() >= 1.89
    b = make_basis(m.Z, diffuse=0.04)
    assert b.nbf == 268 * 16 + 332 * 6


def test_serving_request_is_seeded():
    w1, d1 = cfg_serving_request(3)
    w2, d2 = cfg_serving_request(3)
    assert w1.name == w2.name and len(d1) == len(d2) and 6 <= len(d1) <= 12
    assert np.array_equal(d1[0], d2[0])
    assert abs(np.linalg.norm(d1[0] - w1.P) - 1e-3) < 1e-12
