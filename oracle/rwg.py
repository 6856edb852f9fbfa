"""Mesh validation and RWG topology (oracle).

RWG functions (Rao, Wilton, Glisson, IEEE TAP 30(3), 1982).  The paper names
RWG only as an acronym; its 3-D discretisation is the reading taken here.

For the interior edge n with end vertices (a, b), a < b:
  T+ is the triangle whose counter-clockwise boundary runs a -> b,
  T- is the one that runs b -> a, and v+- are their free vertices;
  f_n(r) = l_n / (2 A+) (r - v+) on T+,   f_n(r) = l_n / (2 A-) (v- - r) on T-,
  div f_n = +l_n / A+ on T+,  -l_n / A- on T-.
Edges are numbered in lexicographic order of (a, b).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


class MeshError(ValueError):
    pass


@dataclass
class Mesh:
    xyz: np.ndarray          # (V, 3) float64
    tri: np.ndarray          # (T, 3) int32, CCW seen from outside
    edges: np.ndarray        # (N, 2) vertex ids (a < b), lexicographic
    edge_tri: np.ndarray     # (N, 2) (T+, T-)
    edge_free: np.ndarray    # (N, 2) free vertex ids (v+, v-)
    edge_len: np.ndarray     # (N,)
    tri_edge: np.ndarray     # (T, 3) RWG index of the edge opposite local vertex i
    tri_sign: np.ndarray     # (T, 3) +1 if the triangle is T+ of that RWG, else -1
    area: np.ndarray         # (T,)
    normal: np.ndarray       # (T, 3) unit outward normal
    centroid: np.ndarray     # (T, 3)
    hmax: np.ndarray         # (T,) longest edge

    @property
    def n(self):
        return len(self.edges)

    @property
    def t(self):
        return len(self.tri)

    def tri_xyz(self):
        return self.xyz[self.tri]


def build(xyz, tri):
    """Validate a closed, consistently oriented 2-manifold and build RWG tables."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    T = len(tri)
    if xyz.ndim != 2 or xyz.shape[1] != 3 or tri.ndim != 2 or tri.shape[1] != 3:
        raise MeshError("bad shapes")
    if tri.min() < 0 or tri.max() >= len(xyz):
        raise MeshError("vertex index out of range")
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(p1 - p0, p2 - p0)
    dbl = np.linalg.norm(cr, axis=1)
    if np.any(dbl <= 0.0):
        raise MeshError("degenerate triangle")
    area = 0.5 * dbl
    normal = cr / dbl[:, None]

    directed = {}
    for t in range(T):
        for i in range(3):
            a, b = int(tri[t, (i + 1) % 3]), int(tri[t, (i + 2) % 3])
            if (a, b) in directed:
                raise MeshError("edge used twice in the same direction (orientation or non-manifold)")
            directed[(a, b)] = (t, i)
    undirected = sorted({(min(a, b), max(a, b)) for (a, b) in directed})
    N = len(undirected)
    edges = np.array(undirected, dtype=np.int64).reshape(N, 2)
    edge_tri = np.zeros((N, 2), dtype=np.int64)
    edge_free = np.zeros((N, 2), dtype=np.int64)
    tri_edge = -np.ones((T, 3), dtype=np.int64)
    tri_sign = np.zeros((T, 3), dtype=np.int64)
    for n, (a, b) in enumerate(undirected):
        if (a, b) not in directed or (b, a) not in directed:
            raise MeshError("open edge")
        tp, ip = directed[(a, b)]
        tm, im = directed[(b, a)]
        edge_tri[n] = (tp, tm)
        edge_free[n] = (tri[tp, ip], tri[tm, im])
        tri_edge[tp, ip], tri_sign[tp, ip] = n, +1
        tri_edge[tm, im], tri_sign[tm, im] = n, -1
    edge_len = np.linalg.norm(xyz[edges[:, 1]] - xyz[edges[:, 0]], axis=1)
    el = np.stack([np.linalg.norm(p1 - p2, axis=1), np.linalg.norm(p2 - p0, axis=1), np.linalg.norm(p0 - p1, axis=1)], 1)
    return Mesh(
        xyz=xyz, tri=tri, edges=edges, edge_tri=edge_tri, edge_free=edge_free, edge_len=edge_len,
        tri_edge=tri_edge, tri_sign=tri_sign, area=area, normal=normal,
        centroid=(p0 + p1 + p2) / 3.0, hmax=el.max(axis=1),
    )


def basis_on_triangle(mesh, t, pts):
    """Values of the three RWG half-functions carried by triangle t at points
    pts (..., 3): returns (3, ..., 3); entry i belongs to RWG mesh.tri_edge[t, i]."""
    out = []
    for i in range(3):
        n = mesh.tri_edge[t, i]
        s = mesh.tri_sign[t, i]
        v = mesh.xyz[mesh.tri[t, i]]
        out.append(s * mesh.edge_len[n] / (2.0 * mesh.area[t]) * (pts - v))
    return np.stack(out)


def divergence_on_triangle(mesh, t):
    """Surface divergence of the three RWG half-functions on triangle t: (3,)."""
    n = mesh.tri_edge[t]
    return mesh.tri_sign[t] * mesh.edge_len[n] / mesh.area[t]
