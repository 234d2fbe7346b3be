"""Writes the stored expected values under tests/golden/.

Calls only the oracle and the input generators. Run from the repository
root: python tests/golden/make_golden.py
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import cfg_water  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def slater_gaussian():
    cx = 0.75 * (3 / math.pi) ** (1 / 3)
    vals = []
    for a in (0.1, 1.0, 5000.0):
        vals.append({"alpha": a, "E_x": -cx * (2 * a / math.pi) ** 2
                     * (3 * math.pi / (8 * a)) ** 1.5})
    return {"citation": "Slater exchange (Sec. 2.1 eq. exc_vvar with the LDA "
                        "exchange energy density) of one normalised s Gaussian, "
                        "P = [[1]]: E_x = -C_x (2a/pi)^2 (3 pi/(8 a))^(3/2), "
                        "C_x = (3/4)(3/pi)^(1/3); closed form, not a paper "
                        "table.",
            "values": vals}


def oracle_water():
    w = cfg_water()
    out = {"citation": "Oracle regression values for one water (O at origin, "
                       "H at (+-1.43, 1.11, 0) bohr), seeded basis and density, "
                       "75 x 302 grid (Table 2 FG shape), eta = 1e-10 (eq. "
                       "rcut), written by this script from oracle/ only."}
    for f in ("lda", "pbe"):
        E, N, V = oracle.integrate(w.coords, w.mk_alpha, w.basis, w.P, f,
                                   w.n_rad, w.ang)
        out[f] = {"E_xc": E, "N_e": N, "trace_V": float(np.trace(V)),
                  "fro_V": float(np.linalg.norm(V))}
    return out


if __name__ == "__main__":
    json.dump(slater_gaussian(), open(os.path.join(HERE, "slater_gaussian.json"), "w"),
              indent=1)
    json.dump(oracle_water(), open(os.path.join(HERE, "oracle_water.json"), "w"),
              indent=1)
    print("written")
