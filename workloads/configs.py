"""The workload shapes the library is exercised and measured on.

Each builder returns a Workload with every input of one XC integration:
atoms (coordinates and Mura-Knowles radial scale), basis, density matrix and
grid parameters. Grid sizes follow the paper's Table 2 shapes (75 x 302,
99 x 590) plus 100 x 590 for the water cluster; screening tolerance 1e-10 and
batches of at most 512 points follow Sec. 2.2.
"""
from dataclasses import dataclass, field

import numpy as np

from .angular import lebedev_table
from .basis import BasisSet, make_basis, overlap_matrix
from .density import random_density, perturbed_density, random_psd_density
from .molecules import Molecule, water, water_cluster, peptide_chain

# Mura-Knowles radial scale per element (5.0 for H, C, N, O).
MK_ALPHA = {1: 5.0, 6: 5.0, 7: 5.0, 8: 5.0}
# Atomic radii for the size adjustment of Becke's partition: Bragg-Slater
# radii in angstrom (Slater, J. Chem. Phys. 41, 3199 (1964)), with 0.35 for
# hydrogen as Becke chose; only their ratios matter.
BECKE_RADIUS = {1: 0.35, 6: 0.70, 7: 0.65, 8: 0.60}


@dataclass
class Workload:
    name: str
    mol: Molecule
    basis: BasisSet
    P: np.ndarray
    n_occ: int
    n_rad: int
    n_ang: int
    functional: str                 # "lda" (Slater + VWN5) or "pbe"
    S: np.ndarray = None
    ssf_a: float = 0.64
    screen_eta: float = 1e-10
    batch_max: int = 512
    rho_thresh: float = 1e-15
    ang: np.ndarray = field(default=None, repr=False)

    def __post_init__(self):
        if self.ang is None:
            self.ang = lebedev_table(self.n_ang)

    @property
    def coords(self):
        return self.mol.coords

    @property
    def mk_alpha(self):
        return np.array([MK_ALPHA[int(z)] for z in self.mol.Z])

    @property
    def becke_radius(self):
        return np.array([BECKE_RADIUS[int(z)] for z in self.mol.Z])

    @property
    def natoms(self):
        return self.mol.natoms

    @property
    def nbf(self):
        return self.basis.nbf

    @property
    def n_points_nominal(self):
        return self.natoms * self.n_rad * self.n_ang


def grid_spec_dict(w, atom_mask=None, **over):
    d = dict(n_rad=w.n_rad, n_ang=w.n_ang, ang=w.ang, ssf_a=w.ssf_a,
             screen_eta=w.screen_eta, batch_max=w.batch_max,
             rho_thresh=w.rho_thresh, atom_mask=atom_mask)
    d.update(over)
    return d


def _finish(name, mol, n_occ, n_rad, n_ang, functional, seed, diffuse=None,
            with_S=True, polarisation=False, pure=False):
    basis = make_basis(mol.Z, seed=2007, diffuse=diffuse, polarisation=polarisation,
                       pure=pure)
    if pure:
        # the generators form Cartesian overlaps only: a plain PSD density
        P = random_psd_density(basis.nbf, n_occ, seed=seed)
        return Workload(name, mol, basis, P, n_occ, n_rad, n_ang, functional)
    S = overlap_matrix(basis, mol.coords)
    P = random_density(S, n_occ, seed=seed)
    return Workload(name, mol, basis, P, n_occ, n_rad, n_ang, functional,
                    S=S if with_S else None)


def cfg_water(functional="lda", n_rad=75, n_ang=302, seed=1, polarisation=False,
              pure=False):
    """One water, ~25 functions, 5 occupied orbitals (tr PS = 10),
    75 x 302 grid per atom (67,950 points). polarisation=True adds an f
    shell on O and a d shell on each H (47 functions); pure=True makes the
    d and f shells spherical (41 functions with polarisation)."""
    name = "water_fd" if polarisation else "water"
    return _finish(name + ("_sph" if pure else ""), water(), 5, n_rad, n_ang,
                   functional, seed, polarisation=polarisation, pure=pure)


def cfg_water_cluster(n_waters=64, functional="pbe", n_rad=100, n_ang=590,
                      seed=2, n_occ=None, box=None, polarisation=False, pure=False):
    """n_waters rigid waters in a box (25 bohr for 64, scaled with the cube
    root of the count otherwise), minimum O-O distance 5 bohr. polarisation
    and pure as for cfg_water (f on O, d on H; spherical d and f shells)."""
    if box is None:
        box = 25.0 * (n_waters / 64.0) ** (1.0 / 3.0)
    if n_occ is None:
        n_occ = 4 * n_waters
    mol = water_cluster(n_waters, box=box, seed=seed)
    name = f"water{n_waters}" + ("_fd" if polarisation else "") + ("_sph" if pure else "")
    return _finish(name, mol, n_occ, n_rad, n_ang, functional, seed,
                   polarisation=polarisation, pure=pure)


def cfg_chain(n_atoms=600, functional="pbe", n_rad=99, n_ang=590, seed=4):
    """Polypeptide-like chain with one extra diffuse s shell (exponent 0.04)
    per atom."""
    mol = peptide_chain(n_atoms, seed=seed)
    n_occ = mol.n_electrons // 2
    return _finish(f"chain{n_atoms}", mol, n_occ, n_rad, n_ang, functional,
                   seed, diffuse=0.04)


def cfg_serving_request(index, seed=5, n_rad=75, n_ang=302):
    """One request of the serving stream: a water cluster of 1-100 waters
    (log-uniform), LDA or PBE (50/50), and 6-12 SCF densities
    P_k = P_0 + delta_k with |delta_k|_F = 1e-3."""
    rng = np.random.default_rng([seed, index])
    n_w = int(np.clip(np.round(np.exp(rng.uniform(0.0, np.log(100.0)))), 1, 100))
    func = "lda" if rng.uniform() < 0.5 else "pbe"
    n_iter = int(rng.integers(6, 13))
    w = cfg_water_cluster(n_w, functional=func, n_rad=n_rad, n_ang=n_ang,
                          seed=seed * 100003 + index, n_occ=5 * n_w)
    w.name = f"req{index}_water{n_w}"
    dens = [perturbed_density(w.P, 1e-3, seed=seed * 7919 + index * 31 + k)
            for k in range(n_iter)]
    return w, dens


def serving_stream(n_requests, seed=5, n_rad=75, n_ang=302, max_waters=100):
    """Request mix of the serving stream: water clusters of 1..max_waters
    waters (log-uniform), LDA or PBE (50/50), 6-12 SCF iterations each.
    Returns (workload, n_iter, density_seed) per request; densities are made
    on the device by the serving loop from density_seed."""
    out = []
    ang = lebedev_table(n_ang)
    for i in range(n_requests):
        rng = np.random.default_rng([seed, i])
        n_w = int(np.clip(np.round(np.exp(rng.uniform(0.0, np.log(max_waters)))), 1,
                          max_waters))
        func = "lda" if rng.uniform() < 0.5 else "pbe"
        n_iter = int(rng.integers(6, 13))
        box = 25.0 * (n_w / 64.0) ** (1.0 / 3.0)
        mol = water_cluster(n_w, box=max(box, 5.0), seed=seed * 100003 + i)
        basis = make_basis(mol.Z, seed=2007)
        w = Workload(f"req{i}_water{n_w}", mol, basis, None, 5 * n_w, n_rad, n_ang,
                     func, ang=ang)
        out.append((w, n_iter, seed * 7919 + i))
    return out
