"""Pins of the oracle's spherical shells (Sec. 2.1: spherical-harmonic
combinations of a shell's Cartesian functions, as in the paper's cc-pVDZ
runs) against facts that do not depend on its closed form: every real solid
harmonic is a harmonic polynomial, they are orthogonal on the sphere with
the Racah norm 4 pi / (2L+1) (Lebedev quadrature, exact to degree 41), the
d table of the textbooks, and spherical shells built from Cartesian shells
normalised for x^L are orthonormal under the analytic Cartesian overlap."""
import numpy as np
import pytest

import oracle
from oracle.basis import cart_exponents, solid_harmonics
from workloads import cfg_water, lebedev_table, make_basis, overlap_matrix
from workloads.molecules import water


def _laplacian_coeffs(L, coef):
    """Coefficients (over the degree L-2 monomials) of the Laplacian of the
    polynomial sum_c coef[c] x^l y^m z^n."""
    out = {}
    for c, (l, m, n) in enumerate(cart_exponents(L)):
        for k, (a, b, d) in ((0, (l, m, n)), (1, (m, l, n)), (2, (n, l, m))):
            if a >= 2:
                e = [l, m, n]
                e[k] -= 2
                out[tuple(e)] = out.get(tuple(e), 0.0) + coef[c] * a * (a - 1)
    return out


@pytest.mark.parametrize("L", range(0, 6))
def test_solid_harmonics_are_harmonic(L):
    T = solid_harmonics(L)
    assert T.shape == (2 * L + 1, (L + 1) * (L + 2) // 2)
    for row in T:
        lap = _laplacian_coeffs(L, row)
        assert max((abs(v) for v in lap.values()), default=0.0) <= 1e-12


@pytest.mark.parametrize("L", range(0, 6))
def test_sphere_orthogonality_and_racah_norm(L):
    ang = lebedev_table(590)           # exact for polynomials up to degree 41
    x, y, z, w = ang.T
    mono = np.stack([x ** l * y ** m * z ** n for (l, m, n) in cart_exponents(L)])
    S = solid_harmonics(L) @ mono      # (2L+1, npts)
    G = (S * w) @ S.T
    assert np.allclose(G, np.eye(2 * L + 1) * 4 * np.pi / (2 * L + 1), atol=1e-12)
    # the same norm as the x^L component
    assert abs((w * x ** (2 * L)).sum() - 4 * np.pi / (2 * L + 1)) <= 1e-12


def test_d_table():
    r3 = np.sqrt(3.0)
    # xx xy xz yy yz zz; m = -2 .. 2: sqrt3 xy, sqrt3 yz, z^2 - (x^2+y^2)/2,
    # sqrt3 xz, sqrt3/2 (x^2 - y^2)
    ref = np.array([[0, r3, 0, 0, 0, 0], [0, 0, 0, 0, r3, 0], [-0.5, 0, 0, -0.5, 0, 1],
                    [0, 0, r3, 0, 0, 0], [r3 / 2, 0, 0, -r3 / 2, 0, 0]])
    assert np.allclose(solid_harmonics(2), ref, atol=1e-15)


def test_p_and_s_are_the_cartesian_functions():
    assert np.allclose(solid_harmonics(0), [[1.0]])
    # m = -1, 0, 1 are y, z, x
    assert np.allclose(solid_harmonics(1), [[0, 1, 0], [0, 0, 1], [1, 0, 0]])


def test_spherical_shells_orthonormal_under_cartesian_overlap():
    """Each d and f shell of the polarised basis is normalised for its x^L
    component; T S_shell T^T with the analytic Cartesian overlap block must
    be the identity."""
    b = make_basis(water().Z, polarisation=True)
    S = overlap_matrix(b, water().coords)
    ff = b.first_func
    seen = set()
    for s in range(b.nshells):
        L = int(b.shell_L[s])
        if L < 2:
            continue
        T = solid_harmonics(L)
        blk = S[ff[s]:ff[s + 1], ff[s]:ff[s + 1]]
        assert np.allclose(T @ blk @ T.T, np.eye(2 * L + 1), atol=1e-12), (s, L)
        seen.add(L)
    assert seen == {2, 3}


def _spherical_overlap(w):
    """S of the spherical basis from the analytic Cartesian overlap and the
    oracle's transform, block by block."""
    cb = w.basis.cartesian()
    Sc = overlap_matrix(cb, w.coords)
    rows = []
    for s in range(w.basis.nshells):
        L = int(w.basis.shell_L[s])
        n = (L + 1) * (L + 2) // 2
        rows.append(solid_harmonics(L) if w.basis.is_pure(s) else np.eye(n))
    from scipy.linalg import block_diag
    T = block_diag(*rows)
    return T @ Sc @ T.T


def test_spherical_basis_electron_count():
    """N_e of a spherical-basis water (f on O, d on H) recovers tr(P S) with
    S the spherical overlap, to quadrature accuracy (75 x 302)."""
    w = cfg_water(polarisation=True, pure=True)
    assert w.nbf == 41
    S = _spherical_overlap(w)
    E, N, V = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, "lda", w.n_rad, w.ang,
                               screen_eta=0.0)
    ref = float(np.sum(w.P * S))
    assert abs(N - ref) <= 2e-5 * ref, (N, ref)


@pytest.mark.parametrize("functional", ["lda", "pbe"])
def test_spherical_potential_is_energy_derivative(functional):
    w = cfg_water(polarisation=True, pure=True, n_rad=24, n_ang=86)
    P = w.P + 0.05 * np.eye(w.nbf)
    run = lambda Pm: oracle.integrate(w.coords, w.mk_alpha, w.basis, Pm, functional,
                                      w.n_rad, w.ang, rho_thresh=1e-20)
    E0, _, V = run(P)
    f_shell = int(w.basis.first_func[6])        # the O f shell (7 functions)
    h = 1e-4
    for m, n in [(f_shell, f_shell), (f_shell + 3, f_shell + 1), (w.nbf - 1, f_shell + 6),
                 (0, w.nbf - 2)]:
        D = np.zeros_like(P)
        D[m, n] += 1.0
        if m != n:
            D[n, m] += 1.0
        fd = (run(P + h * D)[0] - run(P - h * D)[0]) / (2 * h)
        an = V[m, n] * (2.0 if m != n else 1.0)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (m, n, fd, an)
