"""Seeded density matrices.

P = 2 C C^T with C the S-orthonormalised random orbitals, so that P is
symmetric positive semidefinite and tr(P S) = 2 n_occ. Perturbed copies
P_k = P_0 + delta_k (symmetric delta_k of a given Frobenius norm) stand in
for successive SCF iterations.
"""
import numpy as np


def random_density(S, n_occ, seed=0):
    rng = np.random.default_rng([seed, 1])
    nb = S.shape[0]
    C = rng.normal(size=(nb, n_occ))
    M = C.T @ S @ C
    ev, U = np.linalg.eigh(M)
    C = C @ (U / np.sqrt(ev)) @ U.T
    P = 2.0 * C @ C.T
    return np.ascontiguousarray(0.5 * (P + P.T))


def open_shell_densities(S, n_alpha, n_beta, seed=0):
    """P^a = C C^T over n_alpha S-orthonormalised random orbitals and P^b over
    their first n_beta (n_beta <= n_alpha): both positive semidefinite,
    tr(P^a S) = n_alpha, tr(P^b S) = n_beta."""
    rng = np.random.default_rng([seed, 4])
    nb = S.shape[0]
    C = rng.normal(size=(nb, n_alpha))
    M = C.T @ S @ C
    ev, U = np.linalg.eigh(M)
    C = C @ (U / np.sqrt(ev)) @ U.T
    Pa = C @ C.T
    Pb = C[:, :n_beta] @ C[:, :n_beta].T
    return (np.ascontiguousarray(0.5 * (Pa + Pa.T)), np.ascontiguousarray(0.5 * (Pb + Pb.T)))


def perturbed_density(P0, norm, seed):
    rng = np.random.default_rng([seed, 2])
    d = rng.normal(size=P0.shape)
    d = 0.5 * (d + d.T)
    d *= norm / np.linalg.norm(d)
    return np.ascontiguousarray(P0 + d)


def random_psd_density(nbf, n_occ, seed=0):
    """P = 2 C C^T / nbf with C (nbf x n_occ) standard normal: symmetric
    positive semidefinite, without reference to an overlap matrix (for bases
    whose overlap the generators do not form)."""
    rng = np.random.default_rng([seed, 3])
    C = rng.normal(size=(nbf, n_occ))
    P = 2.0 * C @ C.T / nbf
    return np.ascontiguousarray(0.5 * (P + P.T))
