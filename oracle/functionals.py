"""Spin-unpolarised exchange-correlation functionals in Hartree atomic units.

Each function returns (e, v_rho[, v_sigma]) where e = rho * eps is the
energy per unit volume, v_rho = de/drho and v_sigma = de/dsigma with
sigma = |grad rho|^2. This is the reading of the paper's U-variables
(Sec. 2.1, eq. exc_vvar and eq. zvec_r): gamma is taken as sigma (the only
reading under which the factor 2 of eq. zvec_r gives V = dE/dP), and the
derivatives are those of the volumetric density e.

Formulas (the paper names the functionals only through its test
configuration; the constants are the published ones):
  Slater exchange: e = -(3/4)(3/pi)^(1/3) rho^(4/3)
  VWN5 correlation (paramagnetic fit): A = 0.0310907, b = 3.72744,
      c = 12.9352, x0 = -0.10498, x = sqrt(rs)
  PBE exchange: F_x(s) = 1 + kappa - kappa / (1 + mu s^2 / kappa),
      kappa = 0.804, mu = 0.2195149727645171
  PBE correlation: PW92 (A = 0.0310907, alpha1 = 0.21370, beta1..4 =
      7.5957, 3.5876, 1.6382, 0.49294) plus
      H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2)/(1 + A t^2 + A^2 t^4)),
      beta = 0.06672455060314922, gamma = (1 - ln 2)/pi^2.
"""
import numpy as np

PI = np.pi


def _rs(rho):
    return np.cbrt(3.0 / (4.0 * PI * rho))


def slater(rho):
    cx = 0.75 * np.cbrt(3.0 / PI)
    r13 = np.cbrt(rho)
    e = -cx * rho * r13
    v = -(4.0 / 3.0) * cx * r13
    return e, v


def vwn5(rho):
    A, b, c, x0 = 0.0310907, 3.72744, 12.9352, -0.10498
    x = np.sqrt(_rs(rho))
    X = x * x + b * x + c
    X0 = x0 * x0 + b * x0 + c
    Q = np.sqrt(4.0 * c - b * b)
    at = np.arctan(Q / (2.0 * x + b))
    k = b * x0 / X0
    eps = A * (np.log(x * x / X) + 2.0 * b / Q * at
               - k * (np.log((x - x0) ** 2 / X) + 2.0 * (b + 2.0 * x0) / Q * at))
    # d/dx of (2b/Q) atan(Q/(2x+b)) is -b/X because (2x+b)^2 + Q^2 = 4X
    deps_dx = A * (2.0 / x - (2.0 * x + b) / X - b / X
                   - k * (2.0 / (x - x0) - (2.0 * x + b) / X - (b + 2.0 * x0) / X))
    e = rho * eps
    # rho d(eps)/d(rho) = -(rs/3) d(eps)/d(rs) = -(x/6) d(eps)/dx
    v = eps - x / 6.0 * deps_dx
    return e, v


def pbe_x(rho, sigma):
    kappa, mu = 0.804, 0.2195149727645171
    ex, vx = slater(rho)
    k = 1.0 / (4.0 * np.cbrt(3.0 * PI * PI) ** 2)
    r83 = rho ** (8.0 / 3.0)
    s2 = k * sigma / r83
    den = 1.0 + mu * s2 / kappa
    Fx = 1.0 + kappa - kappa / den
    dF = mu / den ** 2                      # dF_x / d(s^2)
    e = ex * Fx
    vrho = vx * Fx + ex * dF * (-8.0 / 3.0) * s2 / rho
    vsigma = ex * dF * k / r83
    return e, vrho, vsigma


def pw92(rs):
    """PW92 correlation energy per particle (unpolarised) and d/d rs."""
    A, a1, b1, b2, b3, b4 = 0.0310907, 0.21370, 7.5957, 3.5876, 1.6382, 0.49294
    srs = np.sqrt(rs)
    Q0 = -2.0 * A * (1.0 + a1 * rs)
    Q1 = 2.0 * A * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs)
    Q1p = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs)
    L = np.log1p(1.0 / Q1)
    eps = Q0 * L
    deps = -2.0 * A * a1 * L - Q0 * Q1p / (Q1 * Q1 + Q1)
    return eps, deps


def pbe_c(rho, sigma):
    beta = 0.06672455060314922
    gamma = (1.0 - np.log(2.0)) / PI ** 2
    c = beta / gamma
    rs = _rs(rho)
    eps, deps_drs = pw92(rs)
    deps_drho = deps_drs * (-rs / (3.0 * rho))
    kF = np.cbrt(3.0 * PI * PI * rho)
    ks2 = 4.0 * kF / PI
    dt2_dsigma = 1.0 / (4.0 * ks2 * rho * rho)
    y = sigma * dt2_dsigma                  # t^2
    Em1 = np.expm1(-eps / gamma)
    A = c / Em1
    N = 1.0 + A * y
    D = 1.0 + A * y + A * A * y * y
    F = c * y * N / D
    H = gamma * np.log1p(F)
    F_y = c * (N * D + y * (A * D - N * (A + 2.0 * A * A * y))) / (D * D)
    F_A = c * y * y * (D - N * (1.0 + 2.0 * A * y)) / (D * D)
    H_y = gamma * F_y / (1.0 + F)
    H_A = gamma * F_A / (1.0 + F)
    dA_deps = c * (Em1 + 1.0) / (gamma * Em1 * Em1)
    dt2_drho = -(7.0 / 3.0) * y / rho
    e = rho * (eps + H)
    vrho = eps + H + rho * (deps_drho + H_y * dt2_drho + H_A * dA_deps * deps_drho)
    vsigma = rho * H_y * dt2_dsigma
    return e, vrho, vsigma


def evaluate(functional, rho, sigma=None, rho_thresh=0.0):
    """e, v_rho, v_sigma on all points; zero where rho < rho_thresh."""
    rho = np.asarray(rho, dtype=np.float64)
    keep = rho >= rho_thresh
    r = np.where(keep, rho, 1.0)
    e = np.zeros_like(rho)
    vr = np.zeros_like(rho)
    vs = np.zeros_like(rho)
    if functional == "slater":
        e1, v1 = slater(r)
        e[:] = np.where(keep, e1, 0.0)
        vr[:] = np.where(keep, v1, 0.0)
    elif functional == "lda":
        e1, v1 = slater(r)
        e2, v2 = vwn5(r)
        e[:] = np.where(keep, e1 + e2, 0.0)
        vr[:] = np.where(keep, v1 + v2, 0.0)
    elif functional == "pbe":
        s = np.where(keep, np.asarray(sigma, dtype=np.float64), 0.0)
        e1, v1, w1 = pbe_x(r, s)
        e2, v2, w2 = pbe_c(r, s)
        e[:] = np.where(keep, e1 + e2, 0.0)
        vr[:] = np.where(keep, v1 + v2, 0.0)
        vs[:] = np.where(keep, w1 + w2, 0.0)
    else:
        raise ValueError(f"unknown functional {functional!r}")
    return e, vr, vs
