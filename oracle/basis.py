"""Cartesian Gaussian collocation with the shell cutoff radius (Sec. 2.1
eq. gau_cart; Sec. 2.2 eq. rcut).

phi_mu(r) = (x-Rx)^l (y-Ry)^m (z-Rz)^n sum_xi d_xi exp(-alpha_xi |r-R|^2)

A shell has (L+1)(L+2)/2 Cartesian functions (the paper's "L(L+1)" is read as
a misprint), ordered lexicographically (xx, xy, xz, yy, yz, zz for L = 2).
The contraction coefficients are used as given.

Spherical shells (Sec. 2.1: the Cartesian functions of a shell may be
replaced by spherical-harmonic combinations of them; the paper's cc-pVDZ
runs do so): a shell flagged pure with L >= 2 holds the 2L+1 real solid
harmonics S_{L,m}(x-Rx, y-Ry, z-Rz) times the same radial factor, m = -L..L,
each a fixed combination of the shell's Cartesian functions. Shells with
L <= 1 stay Cartesian (x, y, z order). The solid harmonics follow the
closed form of Helgaker, Jorgensen and Olsen, Molecular Electronic-Structure
Theory (Wiley, 2000), Sec. 6.4.2, with Racah normalisation: the integral of
S_{L,m}^2 over the unit sphere is 4 pi / (2L+1), the same as that of x^L, so
a shell normalised for its x^L component gives normalised spherical
functions.

Truncated function (the compact-support approximation of Sec. 2.2):
phi~_mu(r) = phi_mu(r) if |r - R_mu| <= r_cut of its shell, else 0, with
r_cut = max_xi sqrt((ln(alpha_xi)/2 - ln(eta)) / alpha_xi); eta = 0 means
no truncation.
"""
import numpy as np


def cart_exponents(L):
    out = []
    for l in range(L, -1, -1):
        for m in range(L - l, -1, -1):
            out.append((l, m, L - l - m))
    return out


def solid_harmonics(L):
    """T (2L+1, (L+1)(L+2)/2) with S_{L,m} = sum_c T[m + L, c] x^l y^m z^n
    over the Cartesian components c in cart_exponents(L) order, m = -L..L.

    S_{L,m} = N sum_{t, u, v} C_{tuv} x^(2t+|m|-2(u+v)) y^(2(u+v)) z^(L-2t-|m|)
    with t = 0..floor((L-|m|)/2), u = 0..t, v = v_m, v_m + 1, ..,
    floor(|m|/2 - v_m) + v_m (v_m = 0 for m >= 0, 1/2 for m < 0),
    C_{tuv} = (-1)^(t+v-v_m) (1/4)^t binom(L, t) binom(L-t, |m|+t) binom(t, u)
              binom(|m|, 2v),
    N = sqrt(2 (L+|m|)! (L-|m|)! / 2^[m = 0]) / (2^|m| L!)."""
    from math import comb, factorial, floor, sqrt
    idx = {e: k for k, e in enumerate(cart_exponents(L))}
    T = np.zeros((2 * L + 1, len(idx)))
    for m in range(-L, L + 1):
        am = abs(m)
        two_vm = 0 if m >= 0 else 1                      # 2 v_m
        norm = sqrt(2.0 * factorial(L + am) * factorial(L - am)
                    / (2.0 if m == 0 else 1.0)) / (2 ** am * factorial(L))
        v_top2 = 2 * floor(am / 2.0 - two_vm / 2.0) + two_vm   # 2 x (largest v)
        for t in range((L - am) // 2 + 1):
            for u in range(t + 1):
                for two_v in range(two_vm, v_top2 + 1, 2):
                    sign = -1.0 if ((2 * t + two_v - two_vm) // 2) % 2 else 1.0
                    c = (sign * 0.25 ** t * comb(L, t) * comb(L - t, am + t) * comb(t, u)
                         * comb(am, two_v))
                    ex = (2 * t + am - 2 * u - two_v, 2 * u + two_v, L - 2 * t - am)
                    T[m + L, idx[ex]] += norm * c
    return T


def shell_rcut(alpha, eta):
    """Cutoff radius of one shell (eq. rcut); inf when eta <= 0."""
    if eta <= 0.0:
        return np.inf
    arg = (np.log(alpha) / 2.0 - np.log(eta)) / alpha
    return float(np.sqrt(np.maximum(arg, 0.0)).max())


def _pow(x, n):
    return np.ones_like(x) if n == 0 else x ** n


def _is_pure(basis, s):
    flags = getattr(basis, "shell_pure", None)
    return flags is not None and bool(flags[s]) and int(basis.shell_L[s]) >= 2


def collocation(points, coords, basis, eta, grad=True):
    """phi~ (npts, nbf) and, if grad, its gradient (3, npts, nbf)."""
    npts = points.shape[0]
    nbf = basis.nbf
    phi = np.zeros((npts, nbf))
    dphi = np.zeros((3, npts, nbf)) if grad else None
    f = 0
    for s in range(basis.nshells):
        atom, L, alpha, d = basis.shell(s)
        if _is_pure(basis, s):
            # the shell's Cartesian functions, then their solid-harmonic
            # combinations
            T = solid_harmonics(L)
            one = _one_shell(points, coords, atom, L, alpha, d, eta, grad)
            phi[:, f:f + 2 * L + 1] = one[0] @ T.T
            if grad:
                for ax in range(3):
                    dphi[ax, :, f:f + 2 * L + 1] = one[1][ax] @ T.T
            f += 2 * L + 1
            continue
        rc = shell_rcut(alpha, eta)
        dx = points - coords[atom][None, :]
        r2 = (dx ** 2).sum(axis=1)
        inside = r2 <= rc * rc if np.isfinite(rc) else np.ones(npts, bool)
        ex = np.exp(-np.outer(r2, alpha))           # (npts, nprim)
        rad = ex @ d                                 # sum d exp
        drad = ex @ (-2.0 * alpha * d)               # d(rad)/d(r^2) * 2
        x, y, z = dx[:, 0], dx[:, 1], dx[:, 2]
        for (l, m, n) in cart_exponents(L):
            ang = _pow(x, l) * _pow(y, m) * _pow(z, n)
            phi[:, f] = np.where(inside, ang * rad, 0.0)
            if grad:
                gx = (l * _pow(x, l - 1) * _pow(y, m) * _pow(z, n) if l else 0.0)
                gy = (m * _pow(x, l) * _pow(y, m - 1) * _pow(z, n) if m else 0.0)
                gz = (n * _pow(x, l) * _pow(y, m) * _pow(z, n - 1) if n else 0.0)
                dphi[0, :, f] = np.where(inside, gx * rad + ang * drad * x, 0.0)
                dphi[1, :, f] = np.where(inside, gy * rad + ang * drad * y, 0.0)
                dphi[2, :, f] = np.where(inside, gz * rad + ang * drad * z, 0.0)
            f += 1
    return phi, dphi


def _one_shell(points, coords, atom, L, alpha, d, eta, grad):
    """Cartesian phi~ (npts, ncart) of one shell and its gradient."""
    from types import SimpleNamespace
    one = SimpleNamespace(nshells=1, nbf=(L + 1) * (L + 2) // 2,
                          shell=lambda s: (0, L, alpha, d), shell_L=np.array([L]),
                          shell_pure=None)
    return collocation(points, coords[atom:atom + 1], one, eta, grad=grad)
