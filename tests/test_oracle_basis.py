"""Pins for the collocation of eq. gau_cart and the cutoff of eq. rcut."""
import math

import numpy as np
import pytest

import oracle
from workloads import cfg_water, lebedev_table, make_basis, overlap_matrix
from workloads.basis import BasisSet


def test_cartesian_order_and_count():
    assert oracle.cart_exponents(2) == [(2, 0, 0), (1, 1, 0), (1, 0, 1),
                                       (0, 2, 0), (0, 1, 1), (0, 0, 2)]
    for L in range(4):
        assert len(oracle.cart_exponents(L)) == (L + 1) * (L + 2) // 2


def test_rcut_definition():
    """At r_cut the primitive that sets it has sqrt(alpha) exp(-alpha r^2) = eta."""
    alpha = np.array([5000.0, 13.6, 0.1])
    eta = 1e-10
    rc = oracle.shell_rcut(alpha, eta)
    vals = np.sqrt(alpha) * np.exp(-alpha * rc * rc)
    assert abs(vals.max() / eta - 1) < 1e-12
    assert np.isinf(oracle.shell_rcut(alpha, 0.0))


@pytest.mark.parametrize("polarisation", [False, True])
def test_collocation_gradient_matches_finite_difference(polarisation):
    w = cfg_water(polarisation=polarisation)
    rng = np.random.default_rng(2)
    pts = rng.normal(scale=1.5, size=(40, 3))
    phi, dphi = oracle.collocation(pts, w.coords, w.basis, 0.0)
    h = 1e-5
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fp, _ = oracle.collocation(pts + e, w.coords, w.basis, 0.0, grad=False)
        fm, _ = oracle.collocation(pts - e, w.coords, w.basis, 0.0, grad=False)
        fd = (fp - fm) / (2 * h)
        scale = np.abs(dphi[d]).max()
        assert np.abs(fd - dphi[d]).max() < 1e-6 * scale


def test_collocation_truncation():
    w = cfg_water()
    rng = np.random.default_rng(3)
    pts = rng.normal(scale=6.0, size=(3000, 3))
    full, _ = oracle.collocation(pts, w.coords, w.basis, 0.0, grad=False)
    trunc, _ = oracle.collocation(pts, w.coords, w.basis, 1e-10, grad=False)
    ff = w.basis.first_func
    for s in range(w.basis.nshells):
        atom, L, alpha, d = w.basis.shell(s)
        rc = oracle.shell_rcut(alpha, 1e-10)
        inside = ((pts - w.coords[atom]) ** 2).sum(1) <= rc * rc
        blk = slice(ff[s], ff[s + 1])
        assert np.array_equal(trunc[inside, blk], full[inside, blk])
        assert np.all(trunc[~inside, blk] == 0.0)


@pytest.mark.parametrize("polarisation", [False, True])
def test_grid_overlap_matches_analytic(polarisation):
    """sum_i w_i phi_mu phi_nu on the SSF grid reproduces the analytic
    overlap S (independent Gaussian-product formula), so every power,
    exponent and coefficient of the collocation is pinned; with
    polarisation the basis holds f (L = 3) and d shells."""
    w = cfg_water(n_rad=100, n_ang=590, polarisation=polarisation)
    pts, wts, _ = oracle.grid_and_weights(
        w.coords, w.mk_alpha, 100, w.ang)
    phi, _ = oracle.collocation(pts, w.coords, w.basis, 0.0, grad=False)
    S_grid = phi.T @ (phi * wts[:, None])
    assert np.abs(S_grid - w.S).max() < 2e-5
    # diagonal x^L components are unit-normalised by construction
    ff = w.basis.first_func
    for s in range(w.basis.nshells):
        assert abs(w.S[ff[s], ff[s]] - 1) < 1e-12


def test_electron_count_recovered():
    """N_e = sum_i w_i rho_i approaches tr(P S) = 2 n_occ (no truncation)."""
    w = cfg_water()
    E, N, V = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, "lda",
                               w.n_rad, w.ang, screen_eta=0.0)
    assert abs(np.trace(w.P @ w.S) - 10.0) < 1e-12
    assert abs(N - 10.0) < 1e-5


def test_analytic_overlap_two_centre_brute_force():
    """The generator's two-centre overlap against a dense Cartesian sum."""
    b = BasisSet(np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                 np.array([1, 1], np.int32), np.array([0.7, 0.4]),
                 np.array([1.0, 1.0]))
    X = np.array([[0.0, 0.0, 0.0], [0.6, -0.3, 0.4]])
    S = overlap_matrix(b, X)
    g = np.linspace(-9, 9, 181)
    hgrid = g[1] - g[0]
    G = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    phi, _ = oracle.collocation(G, X, b, 0.0, grad=False)
    S_num = phi.T @ phi * hgrid ** 3
    assert np.abs(S_num - S).max() < 1e-8
