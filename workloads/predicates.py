"""Seeded query points for the geometric predicates (orient2d, incircle,
diametral circle and lens tests of Section 4.1).

Each query is a row of 4 points (8 doubles); orient2d, indiametral and the
lens test use the first three.  The families are chosen to reach every stage
of an exact predicate: generic points (decided by a floating-point filter),
small dyadic grids (exact zeros), rounded collinear points, rounded cocircular
points on small circles (coordinate differences exact, so an exact stage on
differences) and on large circles whose points span several binades
(differences rounded, so an exact stage on raw coordinates), and clusters a few
units in the last place apart.  Generation only: no predicate is evaluated
here.
"""
from __future__ import annotations

import math

import numpy as np

FAMILIES = ("uniform", "grid", "collinear", "cocircular_small", "cocircular_large", "ulp_cluster")


def predicate_corpus(seed: int, n_per_family: int) -> tuple[np.ndarray, np.ndarray]:
    """(queries (N, 4, 2) float64, family index (N,) int32) for every family."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows, fam = [], []
    for f, name in enumerate(FAMILIES):
        for _ in range(n_per_family):
            if name == "uniform":
                pts = rng.random((4, 2))
            elif name == "grid":
                pts = rng.integers(0, 4, size=(4, 2)) / 4.0
            elif name == "collinear":
                t = rng.random(4)
                x0, y0, dx, dy = rng.random(), rng.random(), rng.random(), rng.random() * 1e-3
                pts = np.stack([x0 + t * dx, y0 + t * dy], axis=1)
            elif name == "cocircular_small":
                cx, cy = 0.5 + rng.random() * 0.25, 0.5 + rng.random() * 0.25
                r = 1e-3 + rng.random() * 1e-2
                ang = np.sort(rng.random(4) * 2 * math.pi)
                pts = np.stack([cx + r * np.cos(ang), cy + r * np.sin(ang)], axis=1)
            elif name == "cocircular_large":
                cx, cy = 0.5, 0.5
                r = 0.3 + rng.random() * 0.19
                ang = np.sort(rng.random(4) * 2 * math.pi)
                pts = np.stack([cx + r * np.cos(ang), cy + r * np.sin(ang)], axis=1)
            else:
                base = rng.random(2)
                pts = base + rng.integers(-3, 4, size=(4, 2)) * 2.0 ** -50
            rows.append(np.asarray(pts, dtype=np.float64))
            fam.append(f)
    return np.stack(rows), np.asarray(fam, dtype=np.int32)
