"""Spin-unrestricted Kohn-Sham XC integration (the extension Sec. 2.1 notes
needs only a few more intermediates): two density matrices P^a, P^b give
rho_a, rho_b and their gradients, the functional depends on
(rho_a, rho_b, sigma_aa, sigma_ab, sigma_bb) with sigma_st = grad rho_s .
grad rho_t, and

    E_xc   = sum_i w_i e(rho_a, rho_b, sigma_aa, sigma_ab, sigma_bb)
    V^a_mn = sum_i w_i [ v_rho_a phi_m phi_n
                         + (2 v_sigma_aa grad rho_a + v_sigma_ab grad rho_b)
                           . (phi_m grad phi_n + grad phi_m phi_n) ]

and V^b likewise with a and b exchanged (the unrestricted form of Sec. 2.1
eq. vxc_exact and eq. zvec_r; V^s = dE/dP^s).

Functionals, in the same reading as the unpolarised ones (oracle/functionals):
  exchange by spin scaling, E_x[rho_a, rho_b] = (E_x[2 rho_a] + E_x[2 rho_b])/2
    (Slater; PBE with sigma -> 4 sigma_ss), a spin's term counted only where
    rho_s >= rho_thresh;
  VWN5 correlation (Vosko, Wilk, Nusair 1980) with its spin interpolation
    eps = eps_P + alpha_c f(zeta)/f''(0) (1 - zeta^4) + (eps_F - eps_P) f(zeta) zeta^4,
    f(zeta) = ((1+zeta)^(4/3) + (1-zeta)^(4/3) - 2)/(2^(4/3) - 2), from its
    paramagnetic, ferromagnetic and spin-stiffness fits;
  PBE correlation on the spin-interpolated PW92 (Perdew and Wang 1992,
    the same interpolation with its three fits; -alpha_c is the fitted one)
    with H = gamma phi^3 ln(1 + (beta/gamma) t^2 (1 + A t^2)/(1 + A t^2 + A^2 t^4)),
    A = (beta/gamma)/(exp(-eps/(gamma phi^3)) - 1),
    t^2 = sigma/(4 phi^2 k_s^2 rho^2), phi = ((1+zeta)^(2/3) + (1-zeta)^(2/3))/2,
    sigma = sigma_aa + 2 sigma_ab + sigma_bb;
  points with rho_a + rho_b < rho_thresh add nothing (N_e counts them);
  zeta is held within [-1 + 1e-10, 1 - 1e-10] (a reading: the paper is silent;
    it keeps phi's zeta derivative finite).

The potentials are the partial derivatives of e, taken here by the complex
step (Im e(x + i h)/h with h = 1e-30: no subtraction, exact to rounding for
these analytic formulas), so they share nothing with a hand derivation.
"""
import math

import numpy as np

from .basis import collocation
from .partition import becke_weights, ssf_weights
from .quadrature import molecular_grid

PI = np.pi
ZETA_CLAMP = 1.0 - 1e-10
_H = 1e-30

# VWN fits (A, b, c, x0): paramagnetic, ferromagnetic, spin stiffness
_VWN_P = (0.0310907, 3.72744, 12.9352, -0.10498)
_VWN_F = (0.01554535, 7.06042, 18.0578, -0.32500)
_VWN_A = (-1.0 / (6.0 * PI ** 2), 1.13107, 13.0045, -0.0047584)
# PW92 fits (A, alpha1, beta1..4): eps(rs, 0), eps(rs, 1), -alpha_c(rs)
_PW_0 = (0.0310907, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294)
_PW_1 = (0.01554535, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517)
_PW_A = (0.0168869, 0.11125, 10.357, 3.6231, 0.88026, 0.49671)


def _p(x, a):
    return np.power(x, a)


def _vwn_fit(x, A, b, c, x0):
    X = x * x + b * x + c
    X0 = x0 * x0 + b * x0 + c
    Q = math.sqrt(4.0 * c - b * b)
    at = np.arctan(Q / (2.0 * x + b))
    return A * (np.log(x * x / X) + 2.0 * b / Q * at
                - b * x0 / X0 * (np.log((x - x0) ** 2 / X) + 2.0 * (b + 2.0 * x0) / Q * at))


def _pw_fit(rs, A, a1, b1, b2, b3, b4):
    sr = np.sqrt(rs)
    return -2.0 * A * (1.0 + a1 * rs) * np.log1p(
        1.0 / (2.0 * A * (b1 * sr + b2 * rs + b3 * rs * sr + b4 * rs * rs)))


def _fzeta(z):
    return (_p(1.0 + z, 4.0 / 3.0) + _p(1.0 - z, 4.0 / 3.0) - 2.0) / (2.0 ** (4.0 / 3.0) - 2.0)


FPP0 = 4.0 / (9.0 * (2.0 ** (1.0 / 3.0) - 1.0))   # f''(0)


def _interp(e0, e1, ac, z):
    f = _fzeta(z)
    z4 = z ** 4
    return e0 + ac * f / FPP0 * (1.0 - z4) + (e1 - e0) * f * z4


def _zeta(ra, rb):
    rho = ra + rb
    z = (ra - rb) / rho
    z = np.where(z.real > ZETA_CLAMP, ZETA_CLAMP + 0j, z)
    return np.where(z.real < -ZETA_CLAMP, -ZETA_CLAMP + 0j, z)


def _slater_u(rho):
    return -0.75 * np.cbrt(3.0 / PI) * _p(rho, 4.0 / 3.0)


def _pbe_x_u(rho, sigma):
    kappa, mu = 0.804, 0.2195149727645171
    s2 = sigma / (4.0 * np.cbrt(3.0 * PI * PI) ** 2 * _p(rho, 8.0 / 3.0))
    return _slater_u(rho) * (1.0 + kappa - kappa / (1.0 + mu * s2 / kappa))


def energy_density(functional, ra, rb, saa, sab, sbb, rho_thresh=1e-15):
    """e(rho_a, rho_b, sigma_aa, sigma_ab, sigma_bb) elementwise (complex
    arguments allowed). Points below the thresholds give 0."""
    ra = np.asarray(ra, dtype=complex)
    rb = np.asarray(rb, dtype=complex)
    keep = (ra + rb).real >= rho_thresh
    ka, kb = keep & (ra.real >= rho_thresh), keep & (rb.real >= rho_thresh)
    one = np.ones_like(ra)
    ra_s, rb_s = np.where(ka, ra, one), np.where(kb, rb, one)
    rho = np.where(keep, ra + rb, 2.0 * one)
    ra_c = np.where(keep, ra, one)
    rb_c = np.where(keep, rb, one)
    z = _zeta(ra_c, rb_c)
    rs = np.cbrt(3.0 / (4.0 * PI)) * _p(rho, -1.0 / 3.0)
    if functional == "lda":
        ex = 0.5 * (np.where(ka, _slater_u(2.0 * ra_s), 0.0)
                    + np.where(kb, _slater_u(2.0 * rb_s), 0.0))
        x = np.sqrt(rs)
        eps = _interp(_vwn_fit(x, *_VWN_P), _vwn_fit(x, *_VWN_F), _vwn_fit(x, *_VWN_A), z)
        ec = rho * eps
    elif functional == "pbe":
        saa = np.asarray(saa, dtype=complex)
        sbb = np.asarray(sbb, dtype=complex)
        sab = np.asarray(sab, dtype=complex)
        ex = 0.5 * (np.where(ka, _pbe_x_u(2.0 * ra_s, 4.0 * np.where(ka, saa, 0.0)), 0.0)
                    + np.where(kb, _pbe_x_u(2.0 * rb_s, 4.0 * np.where(kb, sbb, 0.0)), 0.0))
        beta = 0.06672455060314922
        gamma = (1.0 - math.log(2.0)) / PI ** 2
        eps = _interp(_pw_fit(rs, *_PW_0), _pw_fit(rs, *_PW_1), -_pw_fit(rs, *_PW_A), z)
        phi = 0.5 * (_p(1.0 + z, 2.0 / 3.0) + _p(1.0 - z, 2.0 / 3.0))
        sig = np.where(keep, saa + 2.0 * sab + sbb, 0.0)
        kF = np.cbrt(3.0 * PI * PI) * _p(rho, 1.0 / 3.0)
        ks2 = 4.0 * kF / PI
        t2 = sig / (4.0 * phi * phi * ks2 * rho * rho)
        g3 = gamma * phi ** 3
        A = (beta / gamma) / np.expm1(-eps / g3)
        At2 = A * t2
        H = g3 * np.log1p((beta / gamma) * t2 * (1.0 + At2) / (1.0 + At2 + At2 * At2))
        ec = rho * (eps + H)
    else:
        raise ValueError(f"unknown functional {functional!r}")
    return np.where(keep, ex + ec, 0.0)


def evaluate_spin(functional, ra, rb, saa=None, sab=None, sbb=None, rho_thresh=1e-15):
    """e and its partial derivatives (v_rho_a, v_rho_b, v_sigma_aa,
    v_sigma_ab, v_sigma_bb) by the complex step; real arrays."""
    args = [np.asarray(a, dtype=np.float64) for a in (ra, rb)]
    if functional == "pbe":
        args += [np.asarray(a, dtype=np.float64) for a in (saa, sab, sbb)]
    else:
        zero = np.zeros_like(args[0])
        args += [zero, zero, zero]
    e = energy_density(functional, *args, rho_thresh=rho_thresh).real
    ders = []
    nvar = 5 if functional == "pbe" else 2
    for k in range(5):
        if k >= nvar:
            ders.append(np.zeros_like(e))
            continue
        a = [x.astype(complex) for x in args]
        a[k] = a[k] + 1j * _H
        ders.append(energy_density(functional, *a, rho_thresh=rho_thresh).imag / _H)
    return (e, *ders)


def integrate_uks(coords, mk_alpha, basis, Pa, Pb, functional, n_rad, ang, ssf_a=0.64,
                  screen_eta=1e-10, rho_thresh=1e-15, atom_mask=None, chunk=None,
                  partition="ssf", becke_radius=None):
    """Return (E_xc, N_e, V^a, V^b) by direct quadrature over all points."""
    coords = np.asarray(coords, dtype=np.float64)
    gga = functional == "pbe"
    pts, wq, parent = molecular_grid(coords, mk_alpha, n_rad, ang, atom_mask)
    if partition == "becke":
        w = becke_weights(pts, wq, parent, coords, becke_radius)
    else:
        w = ssf_weights(pts, wq, parent, coords, ssf_a)
    nbf = basis.nbf
    if chunk is None:
        chunk = max(256, min(8192, int(2e7 // max(nbf, 1))))
    Va, Vb = np.zeros((nbf, nbf)), np.zeros((nbf, nbf))
    e_terms, n_terms = [], []
    for c0 in range(0, pts.shape[0], chunk):
        p, wc = pts[c0:c0 + chunk], w[c0:c0 + chunk]
        phi, dphi = collocation(p, coords, basis, screen_eta, grad=gga)
        Xa, Xb = phi @ Pa, phi @ Pb
        ra, rb = (phi * Xa).sum(1), (phi * Xb).sum(1)
        if gga:
            ga = 2.0 * (dphi * Xa[None]).sum(2)
            gb = 2.0 * (dphi * Xb[None]).sum(2)
            saa, sab, sbb = (ga * ga).sum(0), (ga * gb).sum(0), (gb * gb).sum(0)
        else:
            saa = sab = sbb = None
        e, vra, vrb, vsaa, vsab, vsbb = evaluate_spin(functional, ra, rb, saa, sab, sbb,
                                                      rho_thresh)
        e_terms.append(wc * e)
        n_terms.append(wc * (ra + rb))
        for V, vr, mine, other, vss in ((Va, vra, ga if gga else None, gb if gga else None,
                                         vsaa),
                                        (Vb, vrb, gb if gga else None, ga if gga else None,
                                         vsbb)):
            V += phi.T @ (phi * (wc * vr)[:, None])
            if gga:
                for d in range(3):
                    cfac = wc * (2.0 * vss * mine[d] + vsab * other[d])
                    V += phi.T @ (dphi[d] * cfac[:, None])
                    V += dphi[d].T @ (phi * cfac[:, None])
    E = math.fsum(np.concatenate(e_terms)) if e_terms else 0.0
    N = math.fsum(np.concatenate(n_terms)) if n_terms else 0.0
    return E, N, Va, Vb
