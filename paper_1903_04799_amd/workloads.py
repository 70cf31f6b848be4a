"""Seeded synthetic workloads (inputs only; none of the method's arithmetic).

``request_stream`` draws the serving workload: a Poisson stream of
independent squirmer simulations.  Each request is a periodic cubic box of
edge L in {48, 64, 96, 128, 192} with R in {4, 6, 8, 12}, beta uniform in
[-5, 5], B1 = 1e-3, nu = 1/6 and a fixed step count.  Half are one squirmer
at the box centre, half are pairs placed symmetrically about the centre at a
separation s uniform in [3R, min(6R, L/2 - R - 2)] along a random direction
(L and R are redrawn when that interval is empty); every orientation is
uniform on the sphere.
"""
from __future__ import annotations

import numpy as np

EDGES = (48, 64, 96, 128, 192)
RADII = (4.0, 6.0, 8.0, 12.0)


def unit_vector(rng):
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def draw_request(rng, steps=1000, B1=1e-3):
    """One request: (shape, list of body keyword dicts, steps)."""
    pair = rng.random() < 0.5
    while True:
        L = int(rng.choice(EDGES))
        R = float(rng.choice(RADII))
        if not pair:
            break
        hi = min(6.0 * R, L / 2.0 - R - 2.0)
        if hi >= 3.0 * R:
            break
    c = np.full(3, L / 2.0)
    bodies = []
    if not pair:
        bodies.append(dict(pos=tuple(c), e=tuple(unit_vector(rng)), R=R, B1=B1,
                           beta=float(rng.uniform(-5.0, 5.0))))
    else:
        s = float(rng.uniform(3.0 * R, hi))
        d = unit_vector(rng)
        for sign in (-1.0, 1.0):
            bodies.append(dict(pos=tuple(c + sign * 0.5 * s * d), e=tuple(unit_vector(rng)), R=R, B1=B1,
                               beta=float(rng.uniform(-5.0, 5.0))))
    return (L, L, L), bodies, int(steps)


def request_stream(n, seed=0, steps=1000):
    """n requests drawn with a fixed seed."""
    rng = np.random.default_rng(seed)
    return [draw_request(rng, steps) for _ in range(n)]


def poisson_arrivals(n, qps, seed=0):
    """Arrival times (seconds from 0) of a Poisson process of rate qps."""
    rng = np.random.default_rng(seed + 7919)
    return np.cumsum(rng.exponential(1.0 / qps, size=n))
