"""Calderon-stabilized CFIE of a PEC body in 3-D (oracle).

The paper's stabilized operator (Sec. III, eq. 16) is written for the 2-D TM
problem: C_p = N_k~ G^-1 S_k + (G/2 - D*_k~) G^-1 (G/2 + D*_k), the first term
the Calderon product of the EFIE operator, the second that of the MFIE operator,
each second factor at the complex wavenumber k~.  In 3-D the readings taken are
(Andriulli et al., IEEE TAP 56(8), 2008, for the dual basis; Cools et al., IEEE
TAP 59(8), 2011, for the mixed discretization of the MFIE):

  * EFIE term: T_BC(k~) G_mix^-1 Z(k) (module `calderon`), G_mix = (n x f_m, g_n)
    with f RWG and g Buffa-Christiansen (BC) functions;
  * the magnetic operator K J = n x p.v. int grad G_k(r, r') x J(r') dS', the
    MFIE (1/2 - K) J = n x H^inc (J = n x H on the outer side of the surface);
  * every MFIE factor is tested with the rotated BC functions n x g_m and expands
    its argument in RWG functions:
      M_k[m][n]  = (n x g_m, (1/2 - K_k) f_n)  = -G_mix[n][m]/2 - K_BC(k)[m][n],
      M~[m][n]   = (n x g_m, (1/2 + K_k~) f_n) = -G_mix[n][m]/2 + K_BC(k~)[m][n],
      K_BC(k)[m][n] = (g_m, p.v. int grad G_k x f_n dS')   ((n x a) . (n x b) = a . b),
    and (1/2 - K_k) J in RWG coefficients is -G_mix^-T M_k j (its test with
    n x g_m against the RWG expansion is (n x g_m, f_n) = -G_mix[n][m]);
  * so the MFIE term is -M~ G_mix^-T M_k, with right-hand side
    -M~ G_mix^-T h, h_m = (n x g_m, n x H^inc) = (g_m, H^inc);
  * Calderon identity of the continuous operators: with T the EFIE operator
    scaled by 1/eta, (n x T)^2 = -1/4 + K^2, so (n x T~)(n x T) + (1/2 + K~)(1/2 - K)
    vanishes at k~ = k; the stabilized operator is their difference
      C_p = T_BC(k~) G_mix^-1 Z(k) / eta^2 + Q M_k,  Q = M~ G_mix^-T,
      b_p = T_BC(k~) G_mix^-1 V / eta^2 + Q h,
    close to -1/2 + 2 K~K (second kind), free of the interior resonances of the
    EFIE (zeros of j_n(ka) and of (x j_n(x))' at x = ka on the sphere) and of the
    MFIE.  The sign follows from the identity and is pinned numerically (the sum
    is small at k~ = k, the difference is not).

Discretization of K_BC: g_m = sum_e R[e, m] f_e over the RWG functions f_e of the
barycentric refinement, so K_BC = R^T K_mix with
  K_mix[e][n] = int f_e(r) . int grad G_k(r, r') x f_n(r') dS' dS,
the test triangle b of the refinement inside the primal triangle t = b // 6,
the source triangle q primal.  grad G = (r - r') g(R),
  g(R) = -(1 + j k R) exp(-j k R) / (4 pi R^3).
With f_n = c_j (r' - v_j) on q, (r - r') x f_n(r') = c_j (r - r') x (r - v_j).
  * q = t (the test triangle's own primal triangle, coplanar): zero (principal
    value; the integrand is normal to the plane and the test function tangential);
  * (t, q) near by the EFIE near rule of the primal mesh: 7-point rule on b;
    inner integral = 7-point rule of g_s(R) (r - r') with
    g_s = g + 1/(4 pi R^3) = -[(1 + jkR) exp(-jkR) - 1]/(4 pi R^3) (bounded times
    r - r'), plus the closed form -J(r)/(4 pi), J = int (r - r')/R^3 dS'
    (`singular.gradient_integral`);
  * otherwise the 7 x 7 product rule of g.
The numerator (1 + x) exp(-x) - 1, x = j k R, is summed as its Taylor series
sum_{m>=2} (-1)^(m+1) (m - 1) x^m / m! for |x| < 1/2 and evaluated directly above.
"""
from __future__ import annotations

import math

import numpy as np

from . import calderon, efie, quadrature, singular

ETA0 = efie.ETA0


def mfie_numerator(k, R):
    """(1 + j k R) exp(-j k R) - 1 (complex k, R >= 0 array)."""
    x = 1j * complex(k) * np.asarray(R, dtype=np.float64)
    small = np.abs(x) < 0.5
    out = (1.0 + x) * np.exp(-x) - 1.0
    if np.any(small):
        xs = x[small]
        acc = np.zeros(xs.shape, dtype=np.complex128)
        term = xs.copy()                     # x^m / m! built up from m = 1
        for m in range(2, 24):
            term = term * xs / m
            acc = acc + (-1) ** (m + 1) * (m - 1) * term
        out[small] = acc
    return out


def g_full(k, R):
    """g(R) = -(1 + j k R) exp(-j k R) / (4 pi R^3): grad G = (r - r') g."""
    R = np.asarray(R, dtype=np.float64)
    return -(mfie_numerator(k, R) + 1.0) / (4.0 * math.pi * R ** 3)


def g_smooth(k, R):
    """g + 1/(4 pi R^3) = -[(1 + j k R) exp(-j k R) - 1] / (4 pi R^3)."""
    R = np.asarray(R, dtype=np.float64)
    return -mfie_numerator(k, R) / (4.0 * math.pi * R ** 3)


def k_blocks(geo_t, geo_s, k, b, t, near):
    """Local 3 x 3 blocks of K_mix for test triangle b (of geo_t's mesh, inside
    primal triangle t) against every source triangle of geo_s's mesh:
    (T_s, 3 test, 3 source) complex.  near: (T_s,) near flags of the primal pair
    (t, q)."""
    ms = geo_s.mesh
    ra = geo_t.qp[b]                                        # (a, 3)
    rq = geo_s.qp                                           # (Q, c, 3)
    dv = ra[None, :, None, :] - rq[:, None, :, :]           # (Q, a, c, 3)
    R = np.linalg.norm(dv, axis=-1)
    g = np.empty(R.shape, dtype=np.complex128)
    far = ~near
    g[far] = g_full(k, R[far])
    g[near] = g_smooth(k, R[near])
    A = np.einsum("qc,qac,qacx->qax", geo_s.W, g, dv)       # (Q, a, 3) inner integrals
    idx = np.nonzero(near)[0]
    if len(idx):
        Jn = singular.gradient_integral(np.broadcast_to(ra, (len(idx),) + ra.shape), ms.xyz[ms.tri[idx]])
        A[idx] -= Jn / (4.0 * math.pi)
    fb = geo_t.basis(b)                                     # (3i, a, 3)
    arm = ra[None, None, :, :] - geo_s.free[:, :, None, :]  # (Q, 3j, a, 3): r - v_j
    cr = np.cross(A[:, None, :, :], arm)                    # (Q, 3j, a, 3)
    blk = np.einsum("a,iax,qjax->qij", geo_t.W[b], fb, cr) * geo_s.coef[:, None, :]
    blk[t] = 0.0
    return blk


def k_mixed(bary, mesh, k, near_factor=2.0):
    """K_mix (N_bary x N) for the barycentric refinement `bary` of `mesh` (the
    refinement's triangle b lies in primal triangle b // 6)."""
    geo_t = efie.Geometry(bary)
    geo_s = efie.Geometry(mesh)
    K = np.zeros((bary.n, mesh.n), dtype=np.complex128)
    for b in range(bary.t):
        t = b // 6
        near = efie.near_row(mesh, t, near_factor)
        blk = k_blocks(geo_t, geo_s, k, b, t, near)
        for i in range(3):
            e = bary.tri_edge[b, i]
            for j in range(3):
                np.add.at(K[e], mesh.tri_edge[:, j], blk[:, i, j])
    return K


class CFIE:
    """Dense oracle of the 3-D Calderon-stabilized CFIE for one mesh, k and k~."""

    def __init__(self, mesh, k, ktilde, near_factor=2.0, eta=ETA0):
        self.cal = calderon.Calderon(mesh, k, ktilde, near_factor=near_factor, eta=eta)
        self.mesh, self.k, self.kt, self.eta = mesh, k, ktilde, eta
        bary, R, G = self.cal.bary, self.cal.R, self.cal.G
        self.Kk = R.T @ k_mixed(bary, mesh, k, near_factor)
        self.Kkt = R.T @ k_mixed(bary, mesh, ktilde, near_factor)
        self.Mk = -0.5 * G.T - self.Kk
        self.Mt = -0.5 * G.T + self.Kkt
        self.Q = np.linalg.solve(G, self.Mt.T).T               # M~ G^-T
        self.efie_term = self.cal.P @ self.cal.Z / eta ** 2    # T_BC(k~) G^-1 Z(k) / eta^2
        self.mfie_term = self.Q @ self.Mk                      # -(the MFIE Calderon product)
        self.C = self.efie_term + self.mfie_term

    def h(self, khat, pol):
        """h_m = (g_m, H^inc) for plane waves E = pol exp(-j k khat . r),
        H = (khat x pol) exp(-j k khat . r) / eta: (S, N)."""
        khat = np.atleast_2d(khat)
        pol = np.atleast_2d(pol)
        Vb = efie.excitation(self.cal.bary, self.k, khat, np.cross(khat, pol)) / self.eta
        return Vb @ self.cal.R

    def rhs(self, khat, pol):
        """b_p (S, N) and the EFIE right-hand side V (S, N)."""
        V = efie.excitation(self.mesh, self.k, khat, pol)
        hm = self.h(khat, pol)
        return (self.cal.P @ V.T / self.eta ** 2 + self.Q @ hm.T).T, V
