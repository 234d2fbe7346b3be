"""Lebedev-Laikov angular tables, taken from SciPy at run time.

The paper uses Lebedev-Laikov angular quadrature (Sec. 2.2, Table 2); the
tables themselves are not printed there, so they are passed into both the
oracle and the HIP path as an input array of (x, y, z, w) rows with
sum(w) = 4*pi.
"""
import numpy as np

# Lebedev point counts and the polynomial degree each rule integrates exactly.
_DEGREE_OF = {6: 3, 14: 5, 26: 7, 38: 9, 50: 11, 74: 13, 86: 15, 110: 17,
              146: 19, 170: 21, 194: 23, 230: 25, 266: 27, 302: 29, 350: 31,
              434: 35, 590: 41, 770: 47, 974: 53, 1202: 59}


def lebedev_degree(n_ang):
    if n_ang not in _DEGREE_OF:
        raise ValueError(f"no Lebedev rule with {n_ang} points")
    return _DEGREE_OF[n_ang]


def lebedev_table(n_ang):
    """Return an (n_ang, 4) float64 array of unit vectors and weights (sum 4*pi)."""
    from scipy.integrate import lebedev_rule
    x, w = lebedev_rule(lebedev_degree(n_ang))
    if x.shape[1] != n_ang:
        raise RuntimeError(f"scipy returned {x.shape[1]} points for n_ang={n_ang}")
    tab = np.empty((n_ang, 4), dtype=np.float64)
    tab[:, :3] = x.T
    tab[:, 3] = w
    return np.ascontiguousarray(tab)
