"""Writes tests/golden/cluster64_ext_atoms.json: oracle values of the
spin-unrestricted (PBE) and meta-GGA (TPSS) integrations for single parent
atoms of the seeded 64-water cluster (192 atoms, 1600 functions, 100 x 590
grid, the partition over all atoms, eta = 1e-10).

Densities: the cluster's restricted P for TPSS; for the unrestricted run
P^a over 256 and P^b over the first 250 of 256 S-orthonormal random orbitals
(workloads.density.open_shell_densities, seed 2). For each sampled atom and
integration: E_xc, N_e, every row sum of each V, and each V on a seeded
sample of entries (lower triangle and diagonal). Calls only the oracle and
the input generators. Run from the repository root (takes several minutes):

    python tests/golden/make_cluster64_ext_golden.py [atom ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.meta import integrate_mgga  # noqa: E402
from oracle.spin import integrate_uks  # noqa: E402
from workloads import cfg_water_cluster  # noqa: E402
from workloads.density import open_shell_densities  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "cluster64_ext_atoms.json")
N_SAMPLE = 4000
SAMPLE_SEED = 64
N_ALPHA, N_BETA, DENS_SEED = 256, 250, 2


def sample_entries(nbf, n, seed):
    """Seeded (row, col) pairs with row >= col, distinct."""
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, nbf, size=3 * n)
    cols = rng.integers(0, nbf, size=3 * n)
    r, c = np.maximum(rows, cols), np.minimum(rows, cols)
    key = r.astype(np.int64) * nbf + c
    _, first = np.unique(key, return_index=True)
    first = np.sort(first)[:n]
    return r[first], c[first]


def v_record(V, r, c):
    return {"row_sums": V.sum(axis=1).tolist(), "sample_values": V[r, c].tolist(),
            "max_abs_V": float(np.abs(V).max())}


def atom_values(w, Pa, Pb, atom):
    mask = np.zeros(w.natoms, np.uint8)
    mask[atom] = 1
    kw = dict(ssf_a=w.ssf_a, screen_eta=w.screen_eta, rho_thresh=w.rho_thresh, atom_mask=mask)
    r, c = sample_entries(w.nbf, N_SAMPLE, SAMPLE_SEED + atom)
    t = time.time()
    Eu, Nu, Va, Vb = integrate_uks(w.coords, w.mk_alpha, w.basis, Pa, Pb, "pbe", w.n_rad,
                                   w.ang, **kw)
    print(f"  uks {time.time() - t:.0f} s", flush=True)
    t = time.time()
    Et, Nt, Vt = integrate_mgga(w.coords, w.mk_alpha, w.basis, w.P, w.n_rad, w.ang, **kw)
    print(f"  tpss {time.time() - t:.0f} s", flush=True)
    return {"atom": int(atom), "Z": int(w.mol.Z[atom]),
            "sample_rows": r.tolist(), "sample_cols": c.tolist(),
            "uks_pbe": {"E_xc": Eu, "N_e": Nu, "Va": v_record(Va, r, c),
                        "Vb": v_record(Vb, r, c)},
            "tpss": {"E_xc": Et, "N_e": Nt, "V": v_record(Vt, r, c)}}


def main(atoms):
    w = cfg_water_cluster()
    Pa, Pb = open_shell_densities(w.S, N_ALPHA, N_BETA, seed=DENS_SEED)
    out = {"citation": "Oracle values of the spin-unrestricted and meta-GGA extensions "
                       "(Sec. 2.1) summed over all batches of one parent atom (Sec. 2.2 "
                       "eq. exc_batch, eq. vxc_inc) of the seeded 64-water cluster, "
                       "100 x 590 grid, eta = 1e-10; written by this script from "
                       "oracle/ and workloads/ only.",
           "n_rad": w.n_rad, "n_ang": w.n_ang, "nbf": w.nbf,
           "open_shell": {"n_alpha": N_ALPHA, "n_beta": N_BETA, "seed": DENS_SEED},
           "atoms": []}
    for a in atoms:
        print(f"atom {a} (Z = {w.mol.Z[a]})", flush=True)
        out["atoms"].append(atom_values(w, Pa, Pb, a))
        json.dump(out, open(OUT, "w"))
    print(f"written {OUT}")


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [0, 100])
