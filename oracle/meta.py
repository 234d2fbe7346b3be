"""Meta-GGA XC integration (the kinetic-energy-density extension Sec. 2.1
notes needs only a few more intermediates), spin-unpolarised. Besides rho and
sigma the functional depends on the kinetic energy density

    tau_i = 1/2 sum_mn P_mn grad phi_m(r_i) . grad phi_n(r_i),

and since d tau/d P_mn = grad phi_m . grad phi_n / 2,

    V_mn = sum_i w_i [ v_rho phi_m phi_n
                       + 2 v_sigma grad rho . (phi_m grad phi_n + grad phi_m phi_n)
                       + 1/2 v_tau grad phi_m . grad phi_n ].

Functional: TPSS (Tao, Perdew, Staroverov, Scuseria, Phys. Rev. Lett. 91,
146401 (2003)), written from its published definition:

  exchange  e_x = e_x^LDA(rho) F_x(p, z), F_x = 1 + kappa - kappa/(1 + x/kappa),
    p = sigma/(4 (3 pi^2)^(2/3) rho^(8/3)), tau_W = sigma/(8 rho), z = tau_W/tau,
    alpha = (tau - tau_W)/tau_unif, tau_unif = (3/10)(3 pi^2)^(2/3) rho^(5/3),
    q_b = (9/20)(alpha - 1)/sqrt(1 + b alpha (alpha - 1)) + 2p/3,
    x = { [10/81 + c z^2/(1 + z^2)^2] p + (146/2025) q_b^2
          - (73/405) q_b sqrt((3z/5)^2/2 + p^2/2) + (10/81)^2 p^2/kappa
          + 2 sqrt(e) (10/81)(3z/5)^2 + e mu p^3 } / (1 + sqrt(e) p)^2,
    kappa = 0.804, b = 0.40, c = 1.59096, e = 1.537, mu = 0.21951;
  correlation  e_c = rho eps_TPSS, eps_TPSS = eps_rev (1 + d eps_rev z^3), d = 2.8,
    eps_rev = eps_PBE(rho, sigma)(1 + C z^2) - (1 + C) z^2 eps~,
    eps~ = max(eps_PBE(rho/2, 0; sigma/4), eps_PBE(rho, sigma)), C = C(0, 0) = 0.53
    (closed shell: zeta = 0 and grad zeta = 0, both spins alike), where
    eps_PBE(rho/2, 0; sigma/4) is the PBE correlation of the fully polarised
    density rho/2 with |grad|^2 = sigma/4 (PW92's ferromagnetic fit and
    phi = 2^(-1/3)).

Readings (the paper names no meta-GGA):
  * z is held at 1 where tau < tau_W (tau is then taken as tau_W: the
    inequality tau >= tau_W holds for every density of a positive
    semidefinite P, so only rounding or an indefinite P reach it);
  * sqrt((3z/5)^2/2 + p^2/2) is formed, where z < 1, as
    sigma sqrt((3/(5 * 8 rho tau))^2/2 + (p/sigma)^2/2) (the same number for
    sigma >= 0, with no 0/0 in its sigma derivative at sigma = 0);
  * the point threshold is the same as for the other functionals
    (rho < rho_thresh adds nothing; N_e counts every point).

The potentials are partial derivatives taken by the complex step (as in
oracle/spin); the max() and the clamp compare real parts.
"""
import math

import numpy as np

from .basis import collocation
from .partition import becke_weights, ssf_weights
from .quadrature import molecular_grid
from .spin import _PW_0, _PW_1, _pw_fit

PI = np.pi
_H = 1e-30

KAPPA, B_TPSS, C_TPSS, E_TPSS, MU_TPSS = 0.804, 0.40, 1.59096, 1.537, 0.21951
C00, D_TPSS = 0.53, 2.8
BETA = 0.06672455060314922
GAMMA = (1.0 - math.log(2.0)) / PI ** 2
K_F = np.cbrt(3.0 * PI * PI)          # k_F = K_F rho^(1/3)


def _p(x, a):
    return np.power(x, a)


def _pbe_eps_c(n, sig, fit, phi):
    """PBE correlation energy per particle of a density n with |grad n|^2 =
    sig, for the spin state whose PW92 fit is `fit` and whose spin-scaling
    factor is phi (1: unpolarised; 2^(-1/3): fully polarised)."""
    rs = np.cbrt(3.0 / (4.0 * PI)) * _p(n, -1.0 / 3.0)
    eps = _pw_fit(rs, *fit)
    ks2 = 4.0 * K_F * _p(n, 1.0 / 3.0) / PI
    t2 = sig / (4.0 * phi * phi * ks2 * n * n)
    g3 = GAMMA * phi ** 3
    A = (BETA / GAMMA) / np.expm1(-eps / g3)
    At2 = A * t2
    H = g3 * np.log1p((BETA / GAMMA) * t2 * (1.0 + At2) / (1.0 + At2 + At2 * At2))
    return eps + H


def _cmax(a, b):
    return np.where(a.real >= b.real, a, b)


def tpss_parts(rho, sigma, tau):
    """(e_x, e_c) of TPSS per unit volume; complex arguments allowed."""
    tau_w = sigma / (8.0 * rho)
    clamp = tau.real <= tau_w.real           # z = 1 there
    tau_e = np.where(clamp, tau_w, tau)
    one = np.ones_like(rho)
    z = np.where(clamp, one, tau_w / np.where(clamp, one, tau))
    p = sigma / (4.0 * K_F * K_F * _p(rho, 8.0 / 3.0))
    tau_unif = 0.3 * K_F * K_F * _p(rho, 5.0 / 3.0)
    alpha = (tau_e - tau_w) / tau_unif
    qb = 0.45 * (alpha - 1.0) / np.sqrt(1.0 + B_TPSS * alpha * (alpha - 1.0)) + 2.0 * p / 3.0
    p_over_s = 1.0 / (4.0 * K_F * K_F * _p(rho, 8.0 / 3.0))
    root_open = sigma * np.sqrt(0.5 * (0.6 / (8.0 * rho * np.where(clamp, one, tau))) ** 2
                                + 0.5 * p_over_s ** 2)
    root_clamp = np.sqrt(0.5 * 0.36 + 0.5 * p * p)
    root = np.where(clamp, root_clamp, root_open)
    se = math.sqrt(E_TPSS)
    z2 = z * z
    num = ((10.0 / 81.0 + C_TPSS * z2 / (1.0 + z2) ** 2) * p
           + (146.0 / 2025.0) * qb * qb
           - (73.0 / 405.0) * qb * root
           + (10.0 / 81.0) ** 2 * p * p / KAPPA
           + 2.0 * se * (10.0 / 81.0) * 0.36 * z2
           + E_TPSS * MU_TPSS * p ** 3)
    x = num / (1.0 + se * p) ** 2
    fx = 1.0 + KAPPA - KAPPA / (1.0 + x / KAPPA)
    ex = -0.75 * np.cbrt(3.0 / PI) * _p(rho, 4.0 / 3.0) * fx
    eps_pbe = _pbe_eps_c(rho, sigma, _PW_0, 1.0)
    eps_pol = _pbe_eps_c(0.5 * rho, 0.25 * sigma, _PW_1, 2.0 ** (-1.0 / 3.0))
    eps_t = _cmax(eps_pol, eps_pbe)
    eps_rev = eps_pbe * (1.0 + C00 * z2) - (1.0 + C00) * z2 * eps_t
    ec = rho * eps_rev * (1.0 + D_TPSS * eps_rev * z2 * z)
    return ex, ec


def energy_density(rho, sigma, tau, rho_thresh=1e-15):
    """e(rho, sigma, tau) of TPSS elementwise; 0 below the threshold."""
    rho = np.asarray(rho, dtype=complex)
    sigma = np.asarray(sigma, dtype=complex)
    tau = np.asarray(tau, dtype=complex)
    keep = rho.real >= rho_thresh
    one = np.ones_like(rho)
    r = np.where(keep, rho, one)
    s = np.where(keep, sigma, 0.0 * one)
    t = np.where(keep, tau, one)
    ex, ec = tpss_parts(r, s, t)
    return np.where(keep, ex + ec, 0.0)


def evaluate_mgga(rho, sigma, tau, rho_thresh=1e-15):
    """e, v_rho, v_sigma, v_tau by the complex step; real arrays."""
    args = [np.asarray(a, dtype=np.float64) for a in (rho, sigma, tau)]
    e = energy_density(*args, rho_thresh=rho_thresh).real
    ders = []
    for k in range(3):
        a = [x.astype(complex) for x in args]
        a[k] = a[k] + 1j * _H
        ders.append(energy_density(*a, rho_thresh=rho_thresh).imag / _H)
    return (e, *ders)


def integrate_mgga(coords, mk_alpha, basis, P, n_rad, ang, ssf_a=0.64, screen_eta=1e-10,
                   rho_thresh=1e-15, atom_mask=None, chunk=None, partition="ssf",
                   becke_radius=None, details=False):
    """Return (E_xc, N_e, V_xc) of TPSS by direct quadrature over all points
    [and per-point rho, sigma, tau when details]."""
    coords = np.asarray(coords, dtype=np.float64)
    pts, wq, parent = molecular_grid(coords, mk_alpha, n_rad, ang, atom_mask)
    if partition == "becke":
        w = becke_weights(pts, wq, parent, coords, becke_radius)
    else:
        w = ssf_weights(pts, wq, parent, coords, ssf_a)
    nbf = basis.nbf
    if chunk is None:
        chunk = max(256, min(8192, int(2e7 // max(nbf, 1))))
    V = np.zeros((nbf, nbf))
    e_terms, n_terms, det = [], [], []
    for c0 in range(0, pts.shape[0], chunk):
        p, wc = pts[c0:c0 + chunk], w[c0:c0 + chunk]
        phi, dphi = collocation(p, coords, basis, screen_eta, grad=True)
        X = phi @ P
        rho = (phi * X).sum(1)
        g = 2.0 * (dphi * X[None]).sum(2)
        sigma = (g * g).sum(0)
        tau = 0.5 * sum(((dphi[d] @ P) * dphi[d]).sum(1) for d in range(3))
        e, vr, vs, vt = evaluate_mgga(rho, sigma, tau, rho_thresh)
        e_terms.append(wc * e)
        n_terms.append(wc * rho)
        V += phi.T @ (phi * (wc * vr)[:, None])
        for d in range(3):
            c = 2.0 * wc * vs * g[d]
            V += phi.T @ (dphi[d] * c[:, None])
            V += dphi[d].T @ (phi * c[:, None])
            V += dphi[d].T @ (dphi[d] * (0.5 * wc * vt)[:, None])
        if details:
            det.append((rho, sigma, tau))
    E = math.fsum(np.concatenate(e_terms)) if e_terms else 0.0
    N = math.fsum(np.concatenate(n_terms)) if n_terms else 0.0
    if details:
        return E, N, V, [np.concatenate(x) for x in zip(*det)]
    return E, N, V
