"""Stratmann-Scuseria-Frisch atomic partition (Sec. 2.2, eq. atomic_partition
and eq. num_int).

The paper names the scheme without printing it. Reading used here:
    mu_AB = (|r - R_A| - |r - R_B|) / R_AB
    g(mu) = (35 z - 35 z^3 + 21 z^5 - 5 z^7) / 16 with z = mu / a, |mu| < a
    g(mu) = -1 for mu <= -a,  +1 for mu >= a          (a = 0.64)
    s(mu) = (1 - g(mu)) / 2
    P_A(r) = prod_{B != A} s(mu_AB),   p_A(r) = P_A(r) / sum_B P_B(r)
No atomic-size adjustment. The full product is always formed here (the
nearest-neighbour shortcut is not used), so the oracle is the plain
definition.
"""
import numpy as np


def ssf_cell(mu, a=0.64):
    """s(mu) of the SSF scheme, elementwise."""
    z = mu / a
    z2 = z * z
    z3 = z2 * z
    z5 = z3 * z2
    z7 = z5 * z2
    g = (35.0 * z - 35.0 * z3 + 21.0 * z5 - 5.0 * z7) / 16.0
    g = np.where(mu <= -a, -1.0, np.where(mu >= a, 1.0, g))
    return 0.5 * (1.0 - g)


def ssf_partition(points, coords, a=0.64):
    """p_A(r_i) for every atom A and point i; returns (npts, natoms)."""
    n_at = coords.shape[0]
    d = np.linalg.norm(points[:, None, :] - coords[None, :, :], axis=2)
    R = np.linalg.norm(coords[:, None, :] - coords[None, :, :], axis=2)
    Pm = np.ones((points.shape[0], n_at))
    for A in range(n_at):
        others = np.arange(n_at) != A
        mu = (d[:, A:A + 1] - d[:, others]) / R[A, others][None, :]
        Pm[:, A] = np.prod(ssf_cell(mu, a), axis=1)
    return Pm / Pm.sum(axis=1, keepdims=True)


def ssf_weights(points, w_q, parent, coords, a=0.64, chunk=2048, progress=None):
    """Scaled weights w_i = p_{A(i)}(r_i) w^q_i (eq. num_int)."""
    out = np.empty_like(w_q)
    if coords.shape[0] == 1:
        out[:] = w_q
        return out
    for c0 in range(0, points.shape[0], chunk):
        sl = slice(c0, c0 + chunk)
        p = ssf_partition(points[sl], coords, a)
        out[sl] = w_q[sl] * p[np.arange(p.shape[0]), parent[sl]]
        if progress is not None:
            progress("ssf", min(c0 + chunk, points.shape[0]), points.shape[0])
    return out
