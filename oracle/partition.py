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

The alternative partition the paper lists among the possible choices
(Sec. 2.2, after eq. num_int) is Becke's (J. Chem. Phys. 88, 2547 (1988)),
with his atomic-size adjustment:
    nu_AB = mu_AB + a_AB (1 - mu_AB^2),  chi = R_A / R_B (atomic radii),
    u = (chi - 1) / (chi + 1),  a_AB = u / (u^2 - 1) clipped to [-1/2, 1/2]
    p(x) = 3x/2 - x^3/2,  s(nu) = (1 - p(p(p(nu)))) / 2
    P_A(r) = prod_{B != A} s(nu_AB),   p_A(r) = P_A(r) / sum_B P_B(r)
(radii None: a_AB = 0, the unadjusted scheme).
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


def becke_cell(nu):
    """s(nu) of Becke's scheme: three iterations of p(x) = 3x/2 - x^3/2."""
    f = nu
    for _ in range(3):
        f = 1.5 * f - 0.5 * f ** 3
    return 0.5 * (1.0 - f)


def becke_size_adjustment(radii):
    """a_AB (natoms x natoms) from the atomic radii; zeros when radii is None."""
    if radii is None:
        return None
    r = np.asarray(radii, dtype=np.float64)
    chi = r[:, None] / r[None, :]
    u = (chi - 1.0) / (chi + 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = u / (u * u - 1.0)
    a = np.where(np.abs(u) < 1.0, a, 0.0)
    return np.clip(a, -0.5, 0.5)


def becke_partition(points, coords, radii=None):
    """p_A(r_i) of Becke's partition for every atom A and point i;
    returns (npts, natoms)."""
    n_at = coords.shape[0]
    d = np.linalg.norm(points[:, None, :] - coords[None, :, :], axis=2)
    R = np.linalg.norm(coords[:, None, :] - coords[None, :, :], axis=2)
    adj = becke_size_adjustment(radii)
    Pm = np.ones((points.shape[0], n_at))
    for A in range(n_at):
        others = np.arange(n_at) != A
        mu = (d[:, A:A + 1] - d[:, others]) / R[A, others][None, :]
        nu = mu if adj is None else mu + adj[A, others][None, :] * (1.0 - mu * mu)
        Pm[:, A] = np.prod(becke_cell(nu), axis=1)
    return Pm / Pm.sum(axis=1, keepdims=True)


def becke_weights(points, w_q, parent, coords, radii=None, chunk=2048, progress=None):
    """Scaled weights w_i = p_{A(i)}(r_i) w^q_i (eq. num_int) with Becke's
    partition."""
    out = np.empty_like(w_q)
    if coords.shape[0] == 1:
        out[:] = w_q
        return out
    for c0 in range(0, points.shape[0], chunk):
        sl = slice(c0, c0 + chunk)
        p = becke_partition(points[sl], coords, radii)
        out[sl] = w_q[sl] * p[np.arange(p.shape[0]), parent[sl]]
        if progress is not None:
            progress("becke", min(c0 + chunk, points.shape[0]), points.shape[0])
    return out
