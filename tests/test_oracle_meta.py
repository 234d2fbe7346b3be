"""Pins of the oracle's meta-GGA integration (oracle/meta.py, TPSS): the
hydrogen atom's exchange energy (TPSS reproduces the exact -5/16 Eh by
construction; the local-density value -0.2680 Eh is checked beside it), the
uniform-gas limit (Slater + PW92 from the separately written unpolarised
module), the z -> 0 limit of the correlation (PBE), the fully polarised PBE
correlation against the spin-unrestricted module, complex-step derivatives
against central differences, and V = dE/dP by central differences,
including the kinetic-energy-density term."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.functionals import pbe_c, pbe_x, pw92, slater
from oracle.meta import (_pbe_eps_c, energy_density, evaluate_mgga, integrate_mgga,
                         tpss_parts)
from oracle.spin import _PW_1, energy_density as spin_energy_density
from workloads import cfg_water

K_F2 = np.cbrt(3.0 * math.pi ** 2) ** 2


def _hydrogen_exchange(functional_parts):
    """E_x of the hydrogen 1s density n = exp(-2r)/pi (one spin): by spin
    scaling, half the unpolarised exchange of the doubled density, whose
    sigma is 16 n^2 and whose tau is n (twice tau_up = |grad psi|^2/2 = n/2)."""
    def f(r):
        n = math.exp(-2.0 * r) / math.pi
        ex = functional_parts(np.array([2.0 * n], complex), np.array([16.0 * n * n], complex),
                              np.array([n], complex))
        return 0.5 * ex[0].real * 4.0 * math.pi * r * r
    with np.errstate(all="ignore"):     # the correlation part, unused, underflows far out
        return quad(f, 0.0, 40.0, limit=400, epsabs=1e-14, epsrel=1e-13)[0]


def test_hydrogen_atom_exchange_is_exact():
    ex = _hydrogen_exchange(lambda r, s, t: tpss_parts(r, s, t)[0])
    assert abs(ex - (-0.3125)) < 2e-7, ex
    lsd = _hydrogen_exchange(lambda r, s, t: -0.75 * np.cbrt(3 / math.pi) * r ** (4 / 3))
    assert abs(lsd - (-0.26804)) < 1e-5, lsd


def test_uniform_gas_limit():
    rho = 10 ** np.linspace(-6, 2, 40)
    tau = 0.3 * K_F2 * rho ** (5 / 3)
    ex, ec = tpss_parts(rho.astype(complex), 0 * rho + 0j, tau.astype(complex))
    ref_x = slater(rho)[0]
    ref_c = rho * pw92(np.cbrt(3 / (4 * math.pi * rho)))[0]
    assert np.allclose(ex.real, ref_x, rtol=1e-14, atol=0)
    assert np.allclose(ec.real, ref_c, rtol=1e-13, atol=0)


def test_correlation_tends_to_pbe_as_z_vanishes():
    rng = np.random.default_rng(3)
    rho = 10 ** rng.uniform(-4, 1, 30)
    sig = rho ** (8 / 3) * 10 ** rng.uniform(-2, 1, 30)
    tau = 1e9 * (sig / (8 * rho) + 0.3 * K_F2 * rho ** (5 / 3))   # z ~ 1e-9
    ec = tpss_parts(rho.astype(complex), sig.astype(complex), tau.astype(complex))[1].real
    assert np.allclose(ec, pbe_c(rho, sig)[0], rtol=1e-8, atol=0)


def test_fully_polarised_pbe_correlation_matches_spin_module():
    """eps_PBE of the density n with zeta = 1 against the spin-unrestricted
    module at n_a = n, n_b = 0 (whose zeta is held at 1 - 1e-10), with
    that module's exchange removed."""
    rng = np.random.default_rng(4)
    n = 10 ** rng.uniform(-4, 1, 30)
    s = n ** (8 / 3) * 10 ** rng.uniform(-2, 1.5, 30)
    eps = _pbe_eps_c(n.astype(complex), s.astype(complex), _PW_1, 2 ** (-1 / 3)).real
    tot = spin_energy_density("pbe", n, 0 * n, s, 0 * n, 0 * n).real
    ex = 0.5 * pbe_x(2 * n, 4 * s)[0]
    assert np.allclose(n * eps, tot - ex, rtol=1e-6, atol=0)


def test_clamped_and_open_roots_agree_at_the_boundary():
    """At tau = tau_W (1 + 1e-12) the open branch's z is 1 - 1e-12: both
    branches give the same energy to rounding."""
    rho = np.array([0.2, 1.3, 0.01])
    sig = np.array([0.05, 2.0, 1e-4])
    tw = sig / (8 * rho)
    a = energy_density(rho, sig, tw * (1 + 1e-12)).real
    b = energy_density(rho, sig, tw).real
    assert np.allclose(a, b, rtol=1e-10, atol=0)


def test_complex_step_matches_central_differences():
    rng = np.random.default_rng(5)
    rho = 10 ** rng.uniform(-3, 1, 25)
    sig = rho ** (8 / 3) * 10 ** rng.uniform(-1, 1, 25)
    tau = sig / (8 * rho) * (1.0 + 10 ** rng.uniform(-1, 1, 25))
    x = [rho, sig, tau]
    ders = evaluate_mgga(*x)[1:]
    for k in range(3):
        def shifted(d):
            y = [v.copy() for v in x]
            y[k] = y[k] + d
            return energy_density(*y).real
        h = 1e-3 * np.abs(x[k])
        fd = (-shifted(2 * h) + 8 * shifted(h) - 8 * shifted(-h) + shifted(-2 * h)) / (12 * h)
        assert np.allclose(ders[k], fd, rtol=1e-6, atol=1e-10 * np.abs(fd).max()), k


def test_sigma_derivative_finite_at_zero_gradient():
    rho = np.array([0.5, 0.05])
    tau = 0.3 * K_F2 * rho ** (5 / 3) * 1.5
    e, vr, vs, vt = evaluate_mgga(rho, 0 * rho, tau)
    assert np.all(np.isfinite(vs)) and np.all(np.isfinite(vr)) and np.all(np.isfinite(vt))
    h = 1e-9
    fd = (energy_density(rho, 0 * rho + h, tau).real - e) / h
    assert np.allclose(vs, fd, rtol=1e-4)


def test_potential_is_energy_derivative():
    w = cfg_water(n_rad=24, n_ang=86)
    P = w.P + 0.02 * np.eye(w.nbf)
    run = lambda Pm: integrate_mgga(w.coords, w.mk_alpha, w.basis, Pm, w.n_rad, w.ang,
                                    rho_thresh=1e-20)
    E0, N0, V = run(P)
    assert np.array_equal(V, V.T) or np.abs(V - V.T).max() <= 1e-13 * np.abs(V).max()
    h = 1e-4
    for m, n in [(0, 0), (w.nbf - 1, 2), (3, 7), (10, 4)]:
        D = np.zeros_like(P)
        D[m, n] += 1.0
        if m != n:
            D[n, m] += 1.0
        fd = (run(P + h * D)[0] - run(P - h * D)[0]) / (2 * h)
        an = V[m, n] * (2.0 if m != n else 1.0)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (m, n, fd, an)


def test_tau_is_at_least_the_weizsaecker_value():
    """For a positive semidefinite P, tau >= tau_W = sigma/(8 rho) at every
    point (Cauchy-Schwarz on the natural orbitals)."""
    w = cfg_water(n_rad=20, n_ang=50)
    E, N, V, (rho, sig, tau) = integrate_mgga(w.coords, w.mk_alpha, w.basis, w.P, w.n_rad,
                                              w.ang, details=True)
    keep = rho > 1e-10
    assert np.all(tau[keep] >= sig[keep] / (8 * rho[keep]) * (1 - 1e-10))
    assert abs(N - 10.0) < 2e-2     # coarse 20 x 50 grid
