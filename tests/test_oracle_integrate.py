"""Whole-integration pins for the oracle (Sec. 2.1 eq. vxc_exact,
eq. zvec_r; Sec. 2.2 eq. exc_batch, eq. vxc_batch, eq. z_mat)."""
import math

import numpy as np
import pytest

import oracle
from workloads import cfg_water, lebedev_table
from workloads.basis import BasisSet, make_basis, overlap_matrix
from workloads.density import random_density

CX = 0.75 * (3 / math.pi) ** (1 / 3)


@pytest.mark.parametrize("alpha", [0.1, 1.0, 30.0])
def test_slater_single_gaussian_closed_form(alpha):
    """One normalised s Gaussian with P = [[c]] on one atom (partition = 1):
    E_x = -C_x c^(4/3) (2a/pi)^2 (3 pi / (8 a))^(3/2)."""
    c = 1.7
    d = (2 * alpha / math.pi) ** 0.75
    b = BasisSet(np.array([0], np.int32), np.array([0], np.int32),
                 np.array([1], np.int32), np.array([alpha]), np.array([d]))
    X = np.array([[0.2, -0.1, 0.4]])
    E, N, V = oracle.integrate(X, np.array([5.0]), b, np.array([[c]]), "slater",
                               150, lebedev_table(302), screen_eta=0.0,
                               rho_thresh=0.0)
    exact = -CX * c ** (4 / 3) * (2 * alpha / math.pi) ** 2 * (
        3 * math.pi / (8 * alpha)) ** 1.5
    assert abs(E / exact - 1) < 1e-10
    assert abs(N / c - 1) < 1e-10
    # V = dE/dP for a 1x1 density: (4/3) E / c
    assert abs(V[0, 0] / (4 / 3 * exact / c) - 1) < 1e-10


def test_slater_golden_values():
    """Closed-form E_x for c = 1 at alpha = 0.1 and 1 (tests/golden)."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "slater_gaussian.json")))
    for row in g["values"]:
        a = row["alpha"]
        exact = -CX * (2 * a / math.pi) ** 2 * (3 * math.pi / (8 * a)) ** 1.5
        assert abs(exact - row["E_x"]) < 1e-14
        if a <= 1.0:
            d = (2 * a / math.pi) ** 0.75
            b = BasisSet(np.array([0], np.int32), np.array([0], np.int32),
                         np.array([1], np.int32), np.array([a]), np.array([d]))
            E, _, _ = oracle.integrate(np.zeros((1, 3)), np.array([5.0]), b,
                                       np.array([[1.0]]), "slater", 150,
                                       lebedev_table(302), screen_eta=0.0)
            assert abs(E - row["E_x"]) < 1e-10


def test_slater_homogeneity():
    """E_x[c P] = c^(4/3) E_x[P] on the discrete grid (threshold off)."""
    w = cfg_water(n_rad=40, n_ang=110)
    E1, _, _ = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, "slater",
                                w.n_rad, w.ang, rho_thresh=0.0)
    E2, _, _ = oracle.integrate(w.coords, w.mk_alpha, w.basis, 2.5 * w.P,
                                "slater", w.n_rad, w.ang, rho_thresh=0.0)
    assert abs(E2 / (2.5 ** (4 / 3) * E1) - 1) < 1e-13


def _h2():
    Z = np.array([1, 1])
    X = np.array([[0.0, 0.0, 0.0], [0.3, 0.2, 1.4]])
    b = make_basis(Z)
    S = overlap_matrix(b, X)
    return X, b, random_density(S, 1, seed=9)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
@pytest.mark.parametrize("system", ["h2", "water"])
def test_potential_is_energy_derivative(functional, system):
    """V = dE/dP: central differences along symmetric unit directions give
    2 V_mn (m != n) and V_mm. Pins the factors 1/2 and 2 of eq. z_mat and
    the reading gamma = |grad rho|^2."""
    if system == "h2":
        X, b, P = _h2()
        alpha = np.full(2, 5.0)
        n_rad, ang = 40, lebedev_table(110)
    else:
        w = cfg_water(n_rad=30, n_ang=110)
        X, b, P, alpha, n_rad, ang = w.coords, w.basis, w.P, w.mk_alpha, w.n_rad, w.ang
    run = lambda Pm: oracle.integrate(X, alpha, b, Pm, functional, n_rad, ang,
                                      rho_thresh=1e-20)
    # keep P positive definite under the +-h steps so that rho stays > 0
    # (a rank-deficient P - hD has negative-density regions)
    P = P + 0.05 * np.eye(P.shape[0])
    E0, _, V = run(P)
    nb = P.shape[0]
    rng = np.random.default_rng(4)
    pairs = [(0, 0), (nb - 1, 0), (1, 2)] + [tuple(rng.integers(0, nb, 2)) for _ in range(3)]
    h = 1e-4
    for m, n in pairs:
        D = np.zeros_like(P)
        D[m, n] += 1.0
        if m != n:
            D[n, m] += 1.0
        Ep, _, _ = run(P + h * D)
        Em, _, _ = run(P - h * D)
        fd = (Ep - Em) / (2 * h)
        an = V[m, n] * (2.0 if m != n else 1.0)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (m, n, fd, an)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_symmetry_translation_and_mask_additivity(functional):
    w = cfg_water(n_rad=40, n_ang=146)
    E, N, V = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, functional,
                               w.n_rad, w.ang)
    assert np.abs(V - V.T).max() <= 1e-13 * np.abs(V).max()
    shift = np.array([0.37, -1.1, 2.3])
    E2, N2, V2 = oracle.integrate(w.coords + shift, w.mk_alpha, w.basis, w.P,
                                  functional, w.n_rad, w.ang)
    assert abs(E2 - E) <= 1e-12 * abs(E) and abs(N2 - N) <= 1e-12 * N
    assert np.abs(V2 - V).max() <= 1e-11 * np.abs(V).max()
    m = np.array([True, False, True])
    Ea, Na, Va = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, functional,
                                  w.n_rad, w.ang, atom_mask=m)
    Eb, Nb, Vb = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, functional,
                                  w.n_rad, w.ang, atom_mask=~m)
    assert abs(Ea + Eb - E) <= 1e-13 * abs(E)
    assert np.abs(Va + Vb - V).max() <= 1e-13 * np.abs(V).max()


def test_screening_changes_little():
    """The eta = 1e-10 truncation moves E_xc by a small amount only."""
    w = cfg_water(n_rad=50, n_ang=146)
    E, _, _ = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, "lda",
                               w.n_rad, w.ang)
    E0, _, _ = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, "lda",
                                w.n_rad, w.ang, screen_eta=0.0)
    assert abs(E - E0) < 1e-8


def test_golden_water_regression():
    """Stored oracle values for one water (written by tests/golden/make_golden.py)."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "oracle_water.json")))
    w = cfg_water()
    for f in ("lda", "pbe"):
        E, N, V = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, f,
                                   w.n_rad, w.ang)
        ref = g[f]
        assert abs(E - ref["E_xc"]) < 1e-11
        assert abs(N - ref["N_e"]) < 1e-11
        assert abs(np.trace(V) - ref["trace_V"]) < 1e-10
        assert abs(np.linalg.norm(V) - ref["fro_V"]) < 1e-10
