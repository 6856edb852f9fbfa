"""Triangle quadrature (oracle).

The "7-point" rule is Radon's degree-5 rule (Radon 1948; Stroud 1971, T2:5-1):
the centroid plus two orbits of three points, weights summing to one, to be
multiplied by the triangle area.  The paper does not name the rule; degree-5
Radon is the reading taken for the 7-point product rule over triangle pairs.
"""
from __future__ import annotations

import math

import numpy as np


def radon7():
    """Barycentric coordinates (7, 3) and weights (7,) of the degree-5 rule."""
    s15 = math.sqrt(15.0)
    a1 = (9.0 - 2.0 * s15) / 21.0
    b1 = (6.0 + s15) / 21.0
    a2 = (9.0 + 2.0 * s15) / 21.0
    b2 = (6.0 - s15) / 21.0
    w0 = 9.0 / 40.0
    w1 = (155.0 + s15) / 1200.0
    w2 = (155.0 - s15) / 1200.0
    bary = np.array(
        [
            [1 / 3, 1 / 3, 1 / 3],
            [a1, b1, b1], [b1, a1, b1], [b1, b1, a1],
            [a2, b2, b2], [b2, a2, b2], [b2, b2, a2],
        ],
        dtype=np.float64,
    )
    w = np.array([w0, w1, w1, w1, w2, w2, w2], dtype=np.float64)
    return bary, w


def strang_fix3():
    """Barycentric coordinates (3, 3) and weights (3,) of the interior 3-point rule
    of degree 2 (points (2/3, 1/6, 1/6) and permutations, equal weights; Strang and
    Fix 1973, Table 4.1).  Used for well-separated triangle pairs by the
    distance-adaptive far rule, which the paper does not have."""
    a, b = 2.0 / 3.0, 1.0 / 6.0
    bary = np.array([[a, b, b], [b, a, b], [b, b, a]], dtype=np.float64)
    return bary, np.full(3, 1.0 / 3.0)


def points(tri_xyz, bary):
    """Cartesian quadrature points: tri_xyz (..., 3 vertices, 3) -> (..., npts, 3)."""
    return np.einsum("pk,...kx->...px", bary, tri_xyz)


def subdivided(bary, w, s):
    """Composite rule: the reference triangle split 4**s-fold (midpoint splits),
    the base rule applied on every sub-triangle.  Used only for convergence pins."""
    tris = [np.eye(3)]
    for _ in range(s):
        nt = []
        for t in tris:
            a, b, c = t
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nt += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, c]), np.array([ab, bc, ca])]
        tris = nt
    pts = np.concatenate([bary @ t for t in tris], axis=0)
    ws = np.concatenate([w / len(tris) for _ in tris])
    return pts, ws
