"""Seeded synthetic molecular geometries (bohr).

Stand-ins for the paper's test molecules (Table 1), whose geometries are not
available: a single water, a cluster of rigid waters at random orientations,
and a polypeptide-like chain with C:N:O:H = 2:1:1:5.
"""
from dataclasses import dataclass

import numpy as np

# Water shape: O at the origin, H at (+-1.43, 1.11, 0) bohr.
WATER_SHAPE = np.array([[0.0, 0.0, 0.0], [1.43, 1.11, 0.0], [-1.43, 1.11, 0.0]])
WATER_Z = np.array([8, 1, 1], dtype=np.int32)


@dataclass
class Molecule:
    Z: np.ndarray        # int32 [natoms]
    coords: np.ndarray   # float64 [natoms, 3], bohr

    @property
    def natoms(self):
        return int(self.Z.shape[0])

    @property
    def n_electrons(self):
        return int(self.Z.sum())


def water():
    return Molecule(WATER_Z.copy(), WATER_SHAPE.copy())


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def water_cluster(n_waters, box=25.0, min_oo=5.0, seed=0, max_tries=200000):
    """n rigid waters, O uniform in [0, box)^3 with rejection until every O-O
    distance is at least min_oo, each at a uniform random orientation."""
    rng = np.random.default_rng([seed, 64])
    O = []
    tries = 0
    while len(O) < n_waters:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("water_cluster: box too small for min_oo")
        p = rng.uniform(0.0, box, size=3)
        if all(np.linalg.norm(p - q) >= min_oo for q in O):
            O.append(p)
    Z, X = [], []
    for p in O:
        R = _random_rotation(rng)
        X.append(p + WATER_SHAPE @ R.T)
        Z.append(WATER_Z)
    return Molecule(np.concatenate(Z).astype(np.int32), np.concatenate(X))


def _place(a, b, c, bond, angle, torsion):
    """Position of d bonded to c with |cd| = bond, angle(b,c,d) = angle and
    dihedral(a,b,c,d) = torsion (natural extension reference frame)."""
    bc = c - b
    bc /= np.linalg.norm(bc)
    n = np.cross(b - a, bc)
    nn = np.linalg.norm(n)
    if nn < 1e-8:
        n = np.cross(bc, [1.0, 0.0, 0.0])
        if np.linalg.norm(n) < 1e-8:
            n = np.cross(bc, [0.0, 1.0, 0.0])
        nn = np.linalg.norm(n)
    n /= nn
    m = np.cross(n, bc)
    d2 = np.array([-bond * np.cos(angle),
                   bond * np.sin(angle) * np.cos(torsion),
                   bond * np.sin(angle) * np.sin(torsion)])
    return c + d2[0] * bc + d2[1] * m + d2[2] * n


def peptide_chain(n_atoms=600, seed=0):
    """Self-avoiding chain shaped like a polypeptide backbone.

    Units of {N, C, C, O, H x5}: N-C-C form the chain (heavy-heavy bonds
    U(2.5, 2.9) bohr, angles U(110, 120) degrees, random torsions, at least
    3 bohr between non-bonded backbone atoms). Then O hangs off the second C
    (bond U(2.3, 2.4)) and five H atoms (bonds U(1.9, 2.1)) hang off N,
    C(alpha) twice, C and O, each in a random direction at least 1.9 bohr
    (2.3 for O) from every other atom. The atom list is truncated to
    n_atoms; inside a unit the heavy atoms come first, so truncation removes
    H atoms."""
    rng = np.random.default_rng([seed, 600])
    n_units = -(-n_atoms // 9)
    nb = 3 * n_units
    B = np.zeros((nb, 3))
    B[1] = [2.7, 0.0, 0.0]
    ang = np.deg2rad(115.0)
    B[2] = B[1] + 2.7 * np.array([-np.cos(ang), np.sin(ang), 0.0])
    for k in range(3, nb):
        for _ in range(20000):
            p = _place(B[k - 3], B[k - 2], B[k - 1], rng.uniform(2.5, 2.9),
                       np.deg2rad(rng.uniform(110, 120)),
                       rng.uniform(-np.pi, np.pi))
            if np.linalg.norm(B[:k - 1] - p, axis=1).min() >= 3.0:
                B[k] = p
                break
        else:
            raise RuntimeError("peptide_chain: could not place a backbone atom")
    X = [B[k] for k in range(nb)]
    Z = [7 if k % 3 == 0 else 6 for k in range(nb)]

    def branch(parent, z, lo, hi, r_min):
        c = X[parent]
        for _ in range(20000):
            d = rng.normal(size=3)
            p = c + rng.uniform(lo, hi) * d / np.linalg.norm(d)
            dist = np.linalg.norm(np.asarray(X) - p, axis=1)
            dist[parent] = np.inf
            if dist.min() >= r_min:
                X.append(p)
                Z.append(z)
                return len(X) - 1
        raise RuntimeError("peptide_chain: could not place a side atom")

    order = []
    for u in range(n_units):
        n_i, ca, cc = 3 * u, 3 * u + 1, 3 * u + 2
        o = branch(cc, 8, 2.3, 2.4, 2.3)
        hs = [branch(n_i, 1, 1.9, 2.1, 1.9), branch(ca, 1, 1.9, 2.1, 1.9),
              branch(ca, 1, 1.9, 2.1, 1.9), branch(cc, 1, 1.9, 2.1, 1.9),
              branch(o, 1, 1.9, 2.1, 1.9)]
        order.extend([n_i, ca, cc, o] + hs)
    order = order[:n_atoms]
    return Molecule(np.array([Z[k] for k in order], dtype=np.int32),
                    np.array([X[k] for k in order]))
