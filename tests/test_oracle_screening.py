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
