"""Atom-centred product quadrature (Sec. 2.2, eq. num_int; Table 2).

Radial part: Mura-Knowles "log3" rule, r = -alpha ln(1 - x^3) on midpoint
nodes x_k = (k - 1/2)/N_rad, with the r^2 Jacobian folded into the weight.
The paper cites the rule without printing it; this is the reading used.
Angular part: a Lebedev-Laikov table passed in as (x, y, z, w) rows.
Point order inside one atom: radial index outer, angular index inner.
"""
import numpy as np


def mura_knowles(n_rad, alpha):
    """Radial nodes r_k and weights w_k (including r^2) of the MK rule."""
    k = np.arange(1, n_rad + 1, dtype=np.float64)
    x = (k - 0.5) / n_rad
    one_minus = 1.0 - x ** 3
    r = -alpha * np.log(one_minus)
    dr_dx = 3.0 * alpha * x ** 2 / one_minus
    w = dr_dx / n_rad * r ** 2
    return r, w


def atomic_grid(center, n_rad, alpha, ang):
    """Points and unscaled weights w^q of one atom's product grid.

    ang: (n_ang, 4) unit vectors and weights (sum 4 pi)."""
    r, wr = mura_knowles(n_rad, alpha)
    pts = center[None, None, :] + r[:, None, None] * ang[None, :, :3]
    w = wr[:, None] * ang[None, :, 3]
    return pts.reshape(-1, 3), w.reshape(-1)


def molecular_grid(coords, mk_alpha, n_rad, ang, atom_mask=None):
    """Concatenated atomic grids of the parent atoms selected by atom_mask
    (all atoms when None). Returns points, unscaled weights, parent index."""
    P, W, A = [], [], []
    for a in range(coords.shape[0]):
        if atom_mask is not None and not atom_mask[a]:
            continue
        p, w = atomic_grid(coords[a], n_rad, mk_alpha[a], ang)
        P.append(p)
        W.append(w)
        A.append(np.full(w.shape[0], a, dtype=np.int64))
    if not P:
        return np.zeros((0, 3)), np.zeros(0), np.zeros(0, dtype=np.int64)
    return np.concatenate(P), np.concatenate(W), np.concatenate(A)
