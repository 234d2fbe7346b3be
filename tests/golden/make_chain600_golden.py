"""Writes tests/golden/chain600_atoms.json: oracle values for single parent
atoms of the 600-atom polypeptide-like chain at its full grid (99 radial x
590 angular points, the partition over all 600 atoms, 6280 functions with
the diffuse shell), PBE, eta = 1e-10.

For each sampled atom: E_xc, N_e, every row sum of V_xc, and V_xc on a seeded
sample of entries (lower triangle and diagonal). Calls only the oracle and the
input generators. Run from the repository root (takes tens of minutes):

    python tests/golden/make_chain600_golden.py [atom ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import cfg_chain  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "chain600_atoms.json")
N_SAMPLE = 12000
SAMPLE_SEED = 600


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


def atom_values(w, atom):
    mask = np.zeros(w.natoms, np.uint8)
    mask[atom] = 1
    t = time.time()

    def progress(stage, done, total):
        print(f"  atom {atom} {stage} {done}/{total} ({time.time() - t:.0f} s)", flush=True)

    E, N, V = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, "pbe", w.n_rad, w.ang,
                               ssf_a=w.ssf_a, screen_eta=w.screen_eta,
                               rho_thresh=w.rho_thresh, atom_mask=mask, progress=progress)
    r, c = sample_entries(w.nbf, N_SAMPLE, SAMPLE_SEED + atom)
    return {"atom": int(atom), "Z": int(w.mol.Z[atom]), "E_xc": E, "N_e": N,
            "row_sums": V.sum(axis=1).tolist(),
            "sample_rows": r.tolist(), "sample_cols": c.tolist(),
            "sample_values": V[r, c].tolist(),
            "max_abs_V": float(np.abs(V).max()),
            "oracle_seconds": round(time.time() - t, 1)}


def main(atoms):
    w = cfg_chain()
    out = {"citation": "Oracle values (Sec. 2.2 eq. exc_batch, eq. vxc_inc and "
                       "eq. vxc_batch summed over all batches of one parent atom) for "
                       "single parent atoms of the seeded 600-atom polypeptide-like "
                       "chain, 99 x 590 grid (the UFG shape of Table 2), PBE, "
                       "eta = 1e-10 (eq. rcut); written by this script from oracle/ "
                       "and workloads/ only.",
           "n_rad": w.n_rad, "n_ang": w.n_ang, "nbf": w.nbf, "atoms": []}
    for a in atoms:
        print(f"atom {a} (Z = {w.mol.Z[a]})", flush=True)
        out["atoms"].append(atom_values(w, a))
        json.dump(out, open(OUT, "w"))
    print(f"written {OUT}")


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [361, 368])
