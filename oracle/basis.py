"""Cartesian Gaussian collocation with the shell cutoff radius (Sec. 2.1
eq. gau_cart; Sec. 2.2 eq. rcut).

phi_mu(r) = (x-Rx)^l (y-Ry)^m (z-Rz)^n sum_xi d_xi exp(-alpha_xi |r-R|^2)

A shell has (L+1)(L+2)/2 Cartesian functions (the paper's "L(L+1)" is read as
a misprint), ordered lexicographically (xx, xy, xz, yy, yz, zz for L = 2).
The contraction coefficients are used as given.

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


def shell_rcut(alpha, eta):
    """Cutoff radius of one shell (eq. rcut); inf when eta <= 0."""
    if eta <= 0.0:
        return np.inf
    arg = (np.log(alpha) / 2.0 - np.log(eta)) / alpha
    return float(np.sqrt(np.maximum(arg, 0.0)).max())


def _pow(x, n):
    return np.ones_like(x) if n == 0 else x ** n


def collocation(points, coords, basis, eta, grad=True):
    """phi~ (npts, nbf) and, if grad, its gradient (3, npts, nbf)."""
    npts = points.shape[0]
    nbf = basis.nbf
    phi = np.zeros((npts, nbf))
    dphi = np.zeros((3, npts, nbf)) if grad else None
    f = 0
    for s in range(basis.nshells):
        atom, L, alpha, d = basis.shell(s)
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
