"""Basis-shell screening of a point batch by cuboid-sphere intersection
(Sec. 2.2, Alg. 1).

The printed algorithm has two slips that are read as follows: the upper
bound in the second branch is the maximum vertex W_p, and the function
reports an intersection when the remaining squared radius is non-negative
(d >= 0; a tangent sphere counts as intersecting), which is the closed-ball
test matching the truncation |r - R| <= r_cut.
"""
import numpy as np


def cuboid_sphere_intersect(center, radius, vmin, vmax):
    d = radius * radius
    for p in range(3):
        if center[p] < vmin[p]:
            d -= (center[p] - vmin[p]) ** 2
        elif center[p] > vmax[p]:
            d -= (center[p] - vmax[p]) ** 2
    return d >= 0.0


def screen_batch(points, coords, basis, eta):
    """Shells whose cutoff sphere meets the bounding box of points."""
    from .basis import shell_rcut
    vmin = points.min(axis=0)
    vmax = points.max(axis=0)
    keep = []
    for s in range(basis.nshells):
        atom, L, alpha, d = basis.shell(s)
        rc = shell_rcut(alpha, eta)
        if not np.isfinite(rc) or cuboid_sphere_intersect(coords[atom], rc, vmin, vmax):
            keep.append(s)
    return keep
