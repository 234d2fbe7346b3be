"""Alg. 1 (cuboid-sphere intersection) against brute force."""
import numpy as np

import oracle


def test_alg1_matches_closest_point_distance():
    rng = np.random.default_rng(7)
    n_checked = 0
    for _ in range(20000):
        lo = rng.uniform(-5, 5, 3)
        hi = lo + rng.uniform(0, 4, 3)
        c = rng.uniform(-10, 10, 3)
        r = rng.uniform(0, 8)
        closest = np.clip(c, lo, hi)
        dist = np.linalg.norm(c - closest)
        if abs(dist - r) < 1e-9:
            continue
        assert oracle.cuboid_sphere_intersect(c, r, lo, hi) == (dist <= r)
        n_checked += 1
    assert n_checked > 19000


def test_alg1_centre_inside_box_always_intersects():
    lo, hi = np.zeros(3), np.ones(3)
    assert oracle.cuboid_sphere_intersect(np.array([0.5, 0.5, 0.5]), 0.0, lo, hi)


def test_alg1_tangent_counts():
    lo, hi = np.zeros(3), np.ones(3)
    assert oracle.cuboid_sphere_intersect(np.array([3.0, 0.5, 0.5]), 2.0, lo, hi)
    assert not oracle.cuboid_sphere_intersect(np.array([3.0, 0.5, 0.5]), 1.999, lo, hi)


def _rcut_by_bisection(alpha, eta):
    """Largest r at which some primitive's sqrt(alpha) e^{-alpha r^2} still
    reaches eta (the condition eq. rcut solves in closed form), found by
    bisection on that condition directly."""
    alpha = np.asarray(alpha, float)
    f = lambda r: np.max(np.sqrt(alpha) * np.exp(-alpha * r * r)) - eta
    if f(0.0) < 0.0:
        return 0.0
    lo, hi = 0.0, 1.0
    while f(hi) >= 0.0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) >= 0.0:
            lo = mid
        else:
            hi = mid
    return lo


def test_screen_batch_lists_exactly_the_shells_reaching_the_box():
    """screen_batch (Alg. 1 over every shell, with the eq. rcut radius)
    against brute force: a shell is listed exactly when the distance from
    its centre to the closest point of the batch's bounding box is at most
    its cutoff radius, the radius coming from bisection on the defining
    condition. Near-ties are skipped. Every shell left out is exactly zero
    (truncated) at every point of the batch."""
    from workloads.basis import BasisSet
    rng = np.random.default_rng(2007)
    eta = 1e-10
    n_cases = n_checked = 0
    for case in range(60):
        n_at = int(rng.integers(1, 6))
        coords = rng.uniform(-12, 12, (n_at, 3))
        ns = int(rng.integers(3, 9))
        atom = rng.integers(0, n_at, ns).astype(np.int32)
        L = rng.integers(0, 4, ns).astype(np.int32)
        nprim = rng.integers(1, 5, ns).astype(np.int32)
        alpha = np.exp(rng.uniform(np.log(0.03), np.log(5e3), int(nprim.sum())))
        coef = rng.uniform(0.1, 1.0, int(nprim.sum()))
        basis = BasisSet(atom, L, nprim, alpha, coef)
        centre = rng.uniform(-8, 8, 3)
        pts = centre + rng.uniform(-1, 1, (int(rng.integers(1, 40)), 3)) * rng.uniform(0.1, 3.0, 3)
        lo, hi = pts.min(0), pts.max(0)
        got = oracle.screen_batch(pts, coords, basis, eta)
        off = basis.prim_offset
        for s in range(ns):
            rc = _rcut_by_bisection(alpha[off[s]:off[s + 1]], eta)
            c = coords[atom[s]]
            dist = np.linalg.norm(c - np.clip(c, lo, hi))
            if abs(dist - rc) < 1e-9 * max(1.0, rc):
                continue
            assert (s in got) == (dist <= rc), (case, s, dist, rc)
            n_checked += 1
        phi, _ = oracle.collocation(pts, coords, basis, eta, grad=False)
        ff = basis.first_func
        for s in set(range(ns)) - set(got):
            assert not phi[:, ff[s]:ff[s + 1]].any()
        n_cases += 1
    assert n_checked > 250
