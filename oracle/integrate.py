"""E_xc, N_e and V_xc by direct quadrature over all grid points (Sec. 2.1
eq. vxc_exact and eq. zvec_r; Sec. 2.2 eq. exc_batch, eq. vxc_inc,
eq. vxc_batch and eq. z_mat summed over every batch).

Points are processed in chunks only to bound memory; there is no batching,
screening or compression. E_xc and N_e are exactly-rounded sums
(math.fsum) of the per-point terms.
"""
import math

import numpy as np

from .basis import collocation
from .functionals import evaluate
from .partition import becke_weights, ssf_weights
from .quadrature import molecular_grid


def density_on_points(points, coords, basis, P, eta, grad=True):
    """rho (npts,), grad rho (3, npts) or None, and the collocation used."""
    phi, dphi = collocation(points, coords, basis, eta, grad=grad)
    X = phi @ P
    rho = (phi * X).sum(axis=1)
    g = 2.0 * (dphi * X[None]).sum(axis=2) if grad else None
    return rho, g, phi, dphi


def grid_and_weights(coords, mk_alpha, n_rad, ang, ssf_a=0.64, atom_mask=None,
                     progress=None, point_slice=None, partition="ssf", becke_radius=None):
    pts, wq, parent = molecular_grid(coords, mk_alpha, n_rad, ang, atom_mask)
    if point_slice is not None:
        pts, wq, parent = pts[point_slice], wq[point_slice], parent[point_slice]
    if partition == "becke":
        w = becke_weights(pts, wq, parent, coords, becke_radius, progress=progress)
    elif partition == "ssf":
        w = ssf_weights(pts, wq, parent, coords, ssf_a, progress=progress)
    else:
        raise ValueError(f"unknown partition {partition}")
    return pts, w, parent


def integrate(coords, mk_alpha, basis, P, functional, n_rad, ang,
              ssf_a=0.64, screen_eta=1e-10, rho_thresh=1e-15, atom_mask=None,
              chunk=None, details=False, progress=None, point_slice=None,
              partition="ssf", becke_radius=None):
    """Return (E_xc, N_e, V_xc) [and per-point details when asked].
    progress(stage, done, total), if given, is called after every chunk;
    point_slice, if given, restricts the sums to that slice of the grid
    points (a sample of the work); partition "ssf" (default) or "becke"
    (with becke_radius, the atomic radii of the size adjustment, or None)."""
    coords = np.asarray(coords, dtype=np.float64)
    gga = functional == "pbe"
    pts, w, parent = grid_and_weights(coords, mk_alpha, n_rad, ang, ssf_a,
                                      atom_mask, progress, point_slice, partition,
                                      becke_radius)
    nbf = basis.nbf
    if chunk is None:
        chunk = max(256, min(8192, int(2e7 // max(nbf, 1))))
    V = np.zeros((nbf, nbf))
    e_terms, n_terms = [], []
    rho_all, sig_all = [], []
    for c0 in range(0, pts.shape[0], chunk):
        p = pts[c0:c0 + chunk]
        wc = w[c0:c0 + chunk]
        rho, g, phi, dphi = density_on_points(p, coords, basis, P, screen_eta,
                                              grad=gga)
        sigma = (g * g).sum(axis=0) if gga else None
        e, vr, vs = evaluate(functional, rho, sigma, rho_thresh)
        e_terms.append(wc * e)
        n_terms.append(wc * rho)
        V += phi.T @ (phi * (wc * vr)[:, None])
        if gga:
            for d in range(3):
                c = 2.0 * wc * vs * g[d]
                V += phi.T @ (dphi[d] * c[:, None])
                V += dphi[d].T @ (phi * c[:, None])
        if progress is not None:
            progress("integrate", min(c0 + chunk, pts.shape[0]), pts.shape[0])
        if details:
            rho_all.append(rho)
            sig_all.append(sigma if gga else np.zeros_like(rho))
    E = math.fsum(np.concatenate(e_terms)) if e_terms else 0.0
    N = math.fsum(np.concatenate(n_terms)) if n_terms else 0.0
    if details:
        return E, N, V, dict(points=pts, weights=w, parent=parent,
                             rho=np.concatenate(rho_all) if rho_all else np.zeros(0),
                             sigma=np.concatenate(sig_all) if sig_all else np.zeros(0))
    return E, N, V
