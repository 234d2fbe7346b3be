"""Pins for the functional kernels of the oracle.

Derivatives are checked against symbolic differentiation (sympy) evaluated
at 50 digits; the energies against limits and special cases that the
published forms fix (Slater constant, high-density limit, PBE at zero
gradient, large- and small-gradient limits), and VWN5 against PW92 (two
independent fits of the same correlation energy)."""
import math

import mpmath
import numpy as np
import pytest
import sympy as sp

import oracle
from oracle.functionals import pw92

PI = math.pi


def _sym_functionals():
    r, s = sp.symbols("rho sigma", positive=True)
    pi = sp.pi
    rs = (3 / (4 * pi * r)) ** sp.Rational(1, 3)
    ex = -sp.Rational(3, 4) * (3 / pi) ** sp.Rational(1, 3) * r ** sp.Rational(4, 3)
    A, b, c, x0 = (sp.Float("0.0310907", 30), sp.Float("3.72744", 30),
                   sp.Float("12.9352", 30), sp.Float("-0.10498", 30))
    x = sp.sqrt(rs)
    X = lambda t: t * t + b * t + c
    Q = sp.sqrt(4 * c - b * b)
    eps_vwn = A * (sp.log(x ** 2 / X(x)) + 2 * b / Q * sp.atan(Q / (2 * x + b))
                   - b * x0 / X(x0) * (sp.log((x - x0) ** 2 / X(x))
                                       + 2 * (b + 2 * x0) / Q * sp.atan(Q / (2 * x + b))))
    kappa, mu = sp.Float("0.804", 30), sp.Float("0.2195149727645171", 30)
    s2 = s / (4 * (3 * pi ** 2) ** sp.Rational(2, 3) * r ** sp.Rational(8, 3))
    Fx = 1 + kappa - kappa / (1 + mu * s2 / kappa)
    Ap = sp.Float("0.0310907", 30)
    a1, b1, b2, b3, b4 = [sp.Float(v, 30) for v in
                          ("0.21370", "7.5957", "3.5876", "1.6382", "0.49294")]
    eps_pw = -2 * Ap * (1 + a1 * rs) * sp.log(
        1 + 1 / (2 * Ap * (b1 * sp.sqrt(rs) + b2 * rs + b3 * rs ** sp.Rational(3, 2)
                           + b4 * rs ** 2)))
    beta = sp.Float("0.06672455060314922", 30)
    gamma = (1 - sp.log(2)) / pi ** 2
    kF = (3 * pi ** 2 * r) ** sp.Rational(1, 3)
    ks = sp.sqrt(4 * kF / pi)
    t2 = s / (4 * ks ** 2 * r ** 2)
    Ac = beta / gamma / (sp.exp(-eps_pw / gamma) - 1)
    H = gamma * sp.log(1 + beta / gamma * t2 * (1 + Ac * t2)
                       / (1 + Ac * t2 + Ac ** 2 * t2 ** 2))
    return r, s, {"slater": ex, "vwn5": r * eps_vwn, "pbe_x": ex * Fx,
                  "pbe_c": r * (eps_pw + H)}


SYM = _sym_functionals()


def _mp_eval(expr, rv, sv):
    r, s, _ = SYM
    f = sp.lambdify((r, s), expr, modules="mpmath")
    with mpmath.workdps(50):
        return float(f(mpmath.mpf(rv), mpmath.mpf(sv)))


def _sigma_from_s(rho, sred):
    return sred ** 2 * 4 * (3 * PI ** 2) ** (2 / 3) * rho ** (8 / 3)


RHOS = [1e-10, 1e-6, 1e-3, 0.1, 1.0, 30.0, 1e4]
SRED = [0.0, 0.05, 0.7, 3.0, 20.0]


@pytest.mark.parametrize("name", ["slater", "vwn5", "pbe_x", "pbe_c"])
def test_derivatives_match_symbolic(name):
    r, s, ex = SYM
    e_sym = ex[name]
    dr = sp.diff(e_sym, r)
    ds = sp.diff(e_sym, s)
    for rho in RHOS:
        for sred in (SRED if name.startswith("pbe") else [0.0]):
            sig = _sigma_from_s(rho, sred)
            a = np.array([rho])
            if name == "slater":
                e, v = oracle.slater(a)
                w = None
            elif name == "vwn5":
                e, v = oracle.vwn5(a)
                w = None
            elif name == "pbe_x":
                e, v, w = oracle.pbe_x(a, np.array([sig]))
            else:
                e, v, w = oracle.pbe_c(a, np.array([sig]))
            ref_e = _mp_eval(e_sym, rho, sig)
            ref_v = _mp_eval(dr, rho, sig)
            # pbe_c at large gradient is a difference of nearly equal parts
            # (eps_c + H -> 0); scale the tolerance by the zero-gradient part
            se = max(abs(ref_e), abs(_mp_eval(e_sym, rho, 0.0)))
            sv = max(abs(ref_v), abs(_mp_eval(dr, rho, 0.0)))
            assert abs(e[0] - ref_e) <= 1e-12 * se + 1e-300, (rho, sred)
            assert abs(v[0] - ref_v) <= 1e-11 * sv + 1e-300, (rho, sred)
            if w is not None and sig > 0:
                ref_w = _mp_eval(ds, rho, sig)
                assert abs(w[0] - ref_w) <= 1e-10 * abs(ref_w) + 1e-300, (rho, sred)


def test_slater_uniform_gas_constant():
    """eps_x = -(3/(4 pi)) (9 pi/4)^(1/3) / r_s = -0.4581652932831429 / r_s."""
    for rs in (0.5, 1.0, 4.0):
        rho = 3 / (4 * PI * rs ** 3)
        e, _ = oracle.slater(np.array([rho]))
        assert abs(e[0] / rho * rs + 0.4581652932831429) < 1e-15


def test_high_density_limit_slope():
    """Both correlation fits follow eps_c ~ A ln r_s with the
    Gell-Mann-Brueckner coefficient A = (1 - ln 2)/pi^2 as r_s -> 0."""
    A = (1 - math.log(2)) / PI ** 2
    r0, h = 1e-8, 1e-3
    r1, r2 = r0 * math.exp(-h), r0 * math.exp(h)
    rho = lambda q: 3 / (4 * PI * q ** 3)
    sv = (oracle.vwn5(np.array([rho(r2)]))[0][0] / rho(r2)
          - oracle.vwn5(np.array([rho(r1)]))[0][0] / rho(r1)) / (2 * h)
    sp_ = (pw92(np.array([r2]))[0][0] - pw92(np.array([r1]))[0][0]) / (2 * h)
    assert abs(sv / A - 1) < 1e-4 and abs(sp_ / A - 1) < 1e-4


def test_vwn5_and_pw92_agree():
    """Two independent fits of the same correlation energy agree to < 1 mHa
    over metallic densities."""
    rs = np.geomspace(0.1, 50, 40)
    rho = 3 / (4 * PI * rs ** 3)
    e, _ = oracle.vwn5(rho)
    assert np.abs(e / rho - pw92(rs)[0]).max() < 1e-3


def test_pbe_reduces_to_lda_parts_at_zero_gradient():
    rho = np.geomspace(1e-8, 1e3, 30)
    z = np.zeros_like(rho)
    ex, vx, _ = oracle.pbe_x(rho, z)
    es, vs = oracle.slater(rho)
    assert np.allclose(ex, es, rtol=1e-15) and np.allclose(vx, vs, rtol=1e-15)
    ec, vc, _ = oracle.pbe_c(rho, z)
    rs = np.cbrt(3 / (4 * PI * rho))
    assert np.allclose(ec, rho * pw92(rs)[0], rtol=1e-14)


def test_pbe_exchange_limits():
    rho = np.array([0.3])
    es, _ = oracle.slater(rho)
    big = np.array([_sigma_from_s(0.3, 1e7)])
    ex, _, _ = oracle.pbe_x(rho, big)
    assert abs(ex[0] / es[0] - 1.804) < 1e-10
    small = np.array([_sigma_from_s(0.3, 1e-4)])
    ex, _, _ = oracle.pbe_x(rho, small)
    assert abs((ex[0] / es[0] - 1) / 1e-8 - 0.2195149727645171) < 1e-6


def test_pbe_correlation_limits():
    """H -> -eps_c for t -> inf (correlation vanishes) and H ~ beta t^2 for
    small t (gradient expansion)."""
    rho = np.array([0.05])
    kF = (3 * PI ** 2 * 0.05) ** (1 / 3)
    ks2 = 4 * kF / PI
    to_sigma = lambda t2: t2 * 4 * ks2 * 0.05 ** 2
    ec, _, _ = oracle.pbe_c(rho, np.array([to_sigma(1e12)]))
    assert abs(ec[0]) < 1e-9 * 0.05
    e0, _, _ = oracle.pbe_c(rho, np.array([0.0]))
    t2 = 1e-7
    e1, _, _ = oracle.pbe_c(rho, np.array([to_sigma(t2)]))
    assert abs((e1[0] - e0[0]) / 0.05 / t2 / 0.06672455060314922 - 1) < 1e-5


def test_threshold_zeroes_low_density():
    e, v, w = oracle.evaluate("pbe", np.array([1e-16, 1.0]), np.array([1e-30, 0.1]),
                              1e-15)
    assert e[0] == 0 and v[0] == 0 and w[0] == 0 and e[1] != 0
