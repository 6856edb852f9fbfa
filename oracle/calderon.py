"""Calderon preconditioner of the EFIE on barycentric refinements (oracle).

Structure from the paper (Sec. III, eq. 16 and the definition of k~ after it):
second operator at the complex wavenumber k~ = k - 0.4 j k^(1/3) a^(-2/3), times
the inverse of a Gram matrix, times the first operator at k.  In 3-D the second
operator must act on a dual basis; the reading taken (the paper is 2-D) is the
Buffa-Christiansen (BC) basis on the barycentric refinement (Buffa and
Christiansen, Math. Comp. 76, 2007; Andriulli et al., IEEE TAP 56(8), 2008):

  * barycentric refinement: each triangle (v0, v1, v2) with centroid c and edge
    midpoints m01, m12, m20 becomes (v0,m01,c), (m01,v1,c), (v1,m12,c),
    (m12,v2,c), (v2,m20,c), (m20,v0,c);
  * BC function g_n of the primal edge n = (a, b), a < b: a current on the
    barycentric triangles around a and b (the dual cells of a and b) that flows
    from cell(a) to cell(b) across the dual edge of n (flux 1/2 through each of
    its two halves), with equal charge +1/N_a on each of the N_a barycentric
    triangles of cell(a) and -1/N_b on those of cell(b), and zero flux across the
    two halves of the primal edge itself (the symmetric gauge).  It is a sum of
    unit-flux barycentric RWG functions f_e / l_e with the ring fluxes as
    coefficients: g_n = sum_e R[e, n] f_e;
  * mixed Gram matrix (G_mix)_mn = int (n x f_m) . g_n dS (f_m primal RWG), exact
    with the 7-point rule on the barycentric triangles (degree-2 integrand);
  * T_BC(k~) = R^T Z_bary(k~) R with Z_bary the EFIE matrix on the barycentric RWGs;
  * preconditioned operator M = T_BC(k~) G_mix^{-1} Z(k), right-hand side
    T_BC(k~) G_mix^{-1} V.
Equal charge per barycentric triangle and the symmetric gauge are readings: the
literature constructions differ in such details, the paper gives none.
"""
from __future__ import annotations

import math

import numpy as np

from . import efie, quadrature, rwg


def ktilde(k, a=1.0):
    """The complex wavenumber at which the paper evaluates the second operator of
    its Calderon product (Sec. III, the definition that follows eq. 16):
    k~ = k - 0.4 j k^(1/3) a^(-2/3), a an average radius of curvature of the
    scatterer (a = 1 for the unit sphere)."""
    return complex(k, -0.4 * np.cbrt(k) / np.cbrt(a) ** 2)


def barycentric_refinement(mesh):
    """(vertices, triangles) of the barycentric refinement: vertex ids
    0..V-1 original, V..V+N-1 edge midpoints (RWG order), V+N..V+N+T-1 centroids.
    Triangle 6t + k is the k-th sub-triangle of primal triangle t."""
    V, N, T = len(mesh.xyz), mesh.n, mesh.t
    mids = 0.5 * (mesh.xyz[mesh.edges[:, 0]] + mesh.xyz[mesh.edges[:, 1]])
    cents = mesh.xyz[mesh.tri].mean(axis=1)
    xyz = np.concatenate([mesh.xyz, mids, cents])
    tris = []
    for t in range(T):
        v0, v1, v2 = mesh.tri[t]
        # edge opposite local vertex i: midpoint of (v_{i+1}, v_{i+2})
        m12 = V + mesh.tri_edge[t, 0]
        m20 = V + mesh.tri_edge[t, 1]
        m01 = V + mesh.tri_edge[t, 2]
        c = V + N + t
        tris += [(v0, m01, c), (m01, v1, c), (v1, m12, c), (m12, v2, c), (v2, m20, c), (m20, v0, c)]
    return xyz, np.array(tris, dtype=np.int64)


def bc_coefficients(mesh, bary):
    """Dense (N_bary, N) matrix R with g_n = sum_e R[e, n] f_e (f_e barycentric RWG)."""
    V, N = len(mesh.xyz), mesh.n
    Nb = bary.n
    R = np.zeros((Nb, N))
    edge_index = {tuple(e): i for i, e in enumerate(bary.edges)}

    def bedge(p, q):
        return edge_index[(min(p, q), max(p, q))]

    # triangles of the refinement around each vertex, each rotated to start at it
    around = {}
    for b, (p, q, r) in enumerate(bary.tri):
        for (x, y, z) in ((p, q, r), (q, r, p), (r, p, q)):
            around.setdefault(int(x), []).append((b, int(y), int(z)))

    def flows_from(b, e):
        """+1 if barycentric triangle b is T+ of barycentric RWG e, else -1."""
        return 1.0 if bary.edge_tri[e, 0] == b else -1.0

    for n, (a, bvert) in enumerate(mesh.edges):
        mid = V + n
        for c, sigma in ((int(a), 1.0), (int(bvert), -1.0)):
            ring = around[c]                      # (triangle, X, Y) with (c, X, Y) counter-clockwise
            nxt = {X: (t, X, Y) for (t, X, Y) in ring}
            # t_1 has X = mid (the radial edge [c, mid] lies between t_N and t_1)
            order = [nxt[mid]]
            while len(order) < len(ring):
                order.append(nxt[order[-1][2]])
            Nc = len(order)
            x = 0.0
            for i, (t, X, Y) in enumerate(order):
                o = sigma / 2.0 if mid in (X, Y) else 0.0       # outflow through the dual edge
                x += sigma / Nc - o                              # flux from t_i into t_{i+1}
                if i < Nc - 1:
                    e = bedge(c, Y)
                    R[e, n] += flows_from(t, e) * x / bary.edge_len[e]
            assert abs(x) < 1e-12
            if sigma > 0:
                # the two halves of the dual edge, flux 1/2 each from cell(a) to cell(b)
                for (t, X, Y) in (order[0], order[-1]):
                    e = bedge(X, Y)
                    R[e, n] += flows_from(t, e) * 0.5 / bary.edge_len[e]
    return R


def mixed_gram(mesh, bary, R):
    """(G_mix)_mn = int (n x f_m) . g_n dS, 7-point rule on each barycentric triangle."""
    N = mesh.n
    bw, w = quadrature.radon7()
    G = np.zeros((N, N))
    for b in range(bary.t):
        t = b // 6                                    # parent primal triangle
        pts = quadrature.points(bary.tri_xyz()[b], bw)  # (7, 3)
        W = w * bary.area[b]
        fp = rwg.basis_on_triangle(mesh, t, pts)      # (3, 7, 3) primal RWGs on the parent
        nfp = np.cross(mesh.normal[t][None, None, :], fp)
        fb = rwg.basis_on_triangle(bary, b, pts)      # (3, 7, 3) barycentric RWGs on b
        # integrals of (n x f_m) . f_e over b
        I = np.einsum("a,iax,jax->ij", W, nfp, fb)    # (3 primal, 3 bary)
        for j in range(3):
            e = bary.tri_edge[b, j]
            cols = np.nonzero(R[e])[0]
            for i in range(3):
                G[mesh.tri_edge[t, i], cols] += I[i, j] * R[e, cols]
    return G


def bc_charge(mesh, bary, R):
    """Total charge int div g_n dS of every BC function: (N,)."""
    D = np.zeros((bary.t, bary.n))
    for b in range(bary.t):
        for i in range(3):
            e = bary.tri_edge[b, i]
            D[b, e] = bary.tri_sign[b, i] * bary.edge_len[e]    # int_b div f_e
    return (D @ R).sum(axis=0)


class Calderon:
    """Dense oracle of the Calderon-preconditioned EFIE for one mesh and wavenumber."""

    def __init__(self, mesh, k, ktilde, near_factor=2.0, eta=efie.ETA0, far3=None, far3_bary="primal"):
        """far3: ratio of the distance-adaptive far rule of the primal operator (None:
        off); far3_bary: that of the barycentric operator, measured in its own
        triangles' edges ("primal": the same as far3)."""
        self.mesh = mesh
        xyz, tri = barycentric_refinement(mesh)
        self.bary = rwg.build(xyz, tri)
        self.R = bc_coefficients(mesh, self.bary)
        self.G = mixed_gram(mesh, self.bary, self.R)
        self.Z = efie.assemble(mesh, k, near_factor=near_factor, eta=eta, far3=far3)
        fb = far3 if isinstance(far3_bary, str) else far3_bary
        self.Zb = efie.assemble(self.bary, ktilde, near_factor=near_factor, eta=eta, far3=fb)
        self.Tbc = self.R.T @ self.Zb @ self.R
        self.P = self.Tbc @ np.linalg.inv(self.G)      # second operator times the Gram inverse
        self.M = self.P @ self.Z

    def rhs(self, V):
        return self.P @ V
