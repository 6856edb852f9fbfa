"""RWG-discretised EFIE for PEC scatterers (oracle).

Operator (time factor e^{+j omega t}, paper Sec. II eq. 5 and the Galerkin
definition of Sec. III):
  (T_A)_mn   = int int f_m(r) . f_n(r') G_k(|r - r'|) dS' dS
  (T_Phi)_mn = int int div f_m(r) div' f_n(r') G_k(|r - r'|) dS' dS
  Z = eta (j k T_A + T_Phi / (j k)),     Z j = V,    V_m = int f_m . E_inc dS
with G_k(R) = exp(-j k R) / (4 pi R); k may be complex (Im k < 0 decays).

Integration: the 7-point rule on each triangle, the 7x7 product rule on each
triangle pair.  Optional distance-adaptive far rule (not in the paper): with
far3 = r, a far pair whose centroid distance D satisfies D^2 >= (r h)^2, h the
larger longest edge of the two triangles, takes the 3x3 product of the interior
3-point degree-2 rule instead (the squares compared in FP64, summed in x, y, z
order).  Near pairs (sharing a vertex, or centroid distance below
near_factor times the larger longest edge) split G_k = G_smooth + 1/(4 pi R):
  G_smooth(R) = (exp(-j k R) - 1)/(4 pi R), limit -j k / (4 pi) at R = 0,
  integrated by the same 7x7 rule; 1/(4 pi R) by the 7-point rule on the test
  triangle with the closed-form inner integrals of `singular`.  The singular
  block of an ordered pair (p, q) is the mean of the (p test, q source) block
  and the transpose of the (q test, p source) block, which makes Z exactly
  symmetric.  The scaling of Z, the near rule and the symmetrisation are
  readings: the paper defines none of them for the 3-D EFIE.
"""
from __future__ import annotations

import math

import numpy as np

from . import quadrature, rwg, singular

ETA0 = 376.730313668   # free-space wave impedance (ohm)


def near_pairs(mesh, near_factor=2.0):
    """Boolean (T, T) matrix of near triangle pairs, one test triangle at a time."""
    return np.stack([near_row(mesh, p, near_factor) for p in range(mesh.t)])


def near_row(mesh, p, near_factor=2.0):
    """Near flags of test triangle p against every source triangle: (T,)."""
    share = np.isin(mesh.tri, mesh.tri[p]).any(axis=1)
    d2 = ((mesh.centroid - mesh.centroid[p]) ** 2).sum(-1)
    hm = np.maximum(mesh.hmax, mesh.hmax[p])
    return share | (d2 < (near_factor * hm) ** 2)


def far3_row(mesh, p, far3):
    """Pairs (p, q) that take the 3x3 rule under the adaptive far rule with ratio
    far3 (before the near test, which takes precedence): (T,) bool."""
    if far3 is None:
        return np.zeros(mesh.t, dtype=bool)
    d = mesh.centroid - mesh.centroid[p]
    d2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    hm = np.maximum(mesh.hmax, mesh.hmax[p])
    lim = far3 * hm
    return d2 >= lim * lim


def green(k, R):
    """exp(-j k R) / (4 pi R)."""
    return np.exp(-1j * k * R) / (4.0 * math.pi * R)


def green_smooth(k, R, r_zero):
    """(exp(-j k R) - 1) / (4 pi R), with the value -j k / (4 pi) where R <= r_zero.
    exp(z) - 1 for z = -j k R = x + j y is written as
    expm1(x) cos y - 2 sin^2(y/2) + j exp(x) sin y (no cancellation for small R)."""
    k = complex(k)
    z_re = k.imag * R            # Re(-j k R)
    z_im = -k.real * R           # Im(-j k R)
    num = np.expm1(z_re) * np.cos(z_im) - 2.0 * np.sin(0.5 * z_im) ** 2 + 1j * np.exp(z_re) * np.sin(z_im)
    zero = R <= r_zero
    Rs = np.where(zero, 1.0, R)
    return np.where(zero, -1j * k / (4.0 * math.pi), num / (4.0 * math.pi * Rs))


class Geometry:
    """Per-triangle quadrature points, weights and RWG half-function data."""

    def __init__(self, mesh, rule=None):
        self.mesh = mesh
        bary, w = quadrature.radon7() if rule is None else rule
        self.w = w
        self.qp = quadrature.points(mesh.tri_xyz(), bary)          # (T, 7, 3)
        self.W = w[None, :] * mesh.area[:, None]                    # (T, 7)
        # f_i(r) = c_i (r - v_i) on triangle t: coefficient and free vertex
        self.coef = mesh.tri_sign * mesh.edge_len[mesh.tri_edge] / (2.0 * mesh.area[:, None])   # (T, 3)
        self.free = mesh.xyz[mesh.tri]                              # (T, 3, 3) vertex i is free for edge i
        self.div = mesh.tri_sign * mesh.edge_len[mesh.tri_edge] / mesh.area[:, None]             # (T, 3)

    def basis(self, t):
        """RWG half-function values at the quadrature points of triangles t: (..., 3 fn, 7 pts, 3)."""
        t = np.asarray(t)
        return self.coef[t][..., :, None, None] * (self.qp[t][..., None, :, :] - self.free[t][..., :, None, :])


def singular_blocks(geo, ps, qs):
    """Singular (1/(4 pi R)) parts of T_A and T_Phi for test triangles ps against
    source triangles qs (paired element-wise): 7-point rule over the test triangle,
    closed-form inner integrals over the source.  Returns (P, 3, 3), (P, 3, 3) real."""
    mesh = geo.mesh
    ps = np.asarray(ps)
    qs = np.asarray(qs)
    r = geo.qp[ps]                                          # (P, 7, 3)
    vq = mesh.xyz[mesh.tri[qs]]                             # (P, 3, 3)
    I0, I1 = singular.potential_integrals(r, vq)            # (P, 7), (P, 7, 3)
    nq = mesh.normal[qs][:, None, :]
    d = np.sum((r - vq[:, None, 0, :]) * nq, axis=-1)
    rho = r - d[..., None] * nq                              # (P, 7, 3)
    # int_q f_j(r') / R dS' = c_j [ I1 + (rho - v_j) I0 ]
    inner = geo.coef[qs][:, :, None, None] * (I1[:, None] + (rho[:, None] - geo.free[qs][:, :, None, :]) * I0[:, None, :, None])  # (P, 3j, 7, 3)
    fp = geo.basis(ps)                                      # (P, 3i, 7, 3)
    W = geo.W[ps]                                           # (P, 7)
    TA = np.einsum("pa,piax,pjax->pij", W, fp, inner) / (4.0 * math.pi)
    s0 = np.sum(W * I0, axis=-1) / (4.0 * math.pi)          # (P,)
    TP = geo.div[ps][:, :, None] * geo.div[qs][:, None, :] * s0[:, None, None]
    return TA, TP


def _regular_blocks(geo, k, p, qs, near):
    """T_A, T_Phi blocks of test triangle p against sources qs by the product rule of
    geo: G_k on the far pairs, G_smooth on the near ones (flags `near`)."""
    mesh = geo.mesh
    rp = geo.qp[p]                                   # (a, 3)
    rq = geo.qp[qs]                                  # (Q, b, 3)
    R = np.linalg.norm(rp[None, :, None, :] - rq[:, None, :, :], axis=-1)   # (Q, a, b)
    G = np.empty(R.shape, dtype=np.complex128)
    far = ~near
    G[far] = green(k, R[far])
    r_zero = 1e-14 * mesh.hmax[p]
    G[near] = green_smooth(k, R[near], r_zero)
    WW = geo.W[p][None, :, None] * geo.W[qs][:, None, :]                   # (Q, a, b)
    fp = geo.basis(p)                                # (3i, a, 3)
    fq = geo.basis(qs)                               # (Q, 3j, b, 3)
    dot = np.einsum("iax,qjbx->qijab", fp, fq)       # (Q, 3, 3, a, b)
    TA = np.einsum("qab,qijab->qij", WW * G, dot)
    S = np.einsum("qab->q", WW * G)
    TP = geo.div[p][None, :, None] * geo.div[qs][:, None, :] * S[:, None, None]
    return TA, TP


def pair_blocks(geo, k, p, qs, near_factor=2.0, far3=None, geo3=None):
    """T_A and T_Phi local 3x3 blocks for test triangle p against source triangles qs.
    Returns TA (len(qs), 3, 3) and TP (len(qs), 3, 3) complex.  far3: ratio of the
    distance-adaptive far rule (None: the 7x7 rule on every pair); geo3 the
    Geometry of the 3-point rule (built when not given)."""
    mesh = geo.mesh
    qs = np.atleast_1d(np.asarray(qs))
    near = near_row(mesh, p, near_factor)[qs]
    use3 = far3_row(mesh, p, far3)[qs] & ~near
    TA = np.empty((len(qs), 3, 3), dtype=np.complex128)
    TP = np.empty((len(qs), 3, 3), dtype=np.complex128)
    i7 = np.nonzero(~use3)[0]
    if len(i7):
        TA[i7], TP[i7] = _regular_blocks(geo, k, p, qs[i7], near[i7])
    i3 = np.nonzero(use3)[0]
    if len(i3):
        geo3 = geo3 or Geometry(mesh, quadrature.strang_fix3())
        TA[i3], TP[i3] = _regular_blocks(geo3, k, p, qs[i3], np.zeros(len(i3), dtype=bool))
    idx = np.nonzero(near)[0]
    if len(idx):
        qn = qs[idx]
        pn = np.full(len(idx), p)
        A1, P1 = singular_blocks(geo, pn, qn)
        A2, P2 = singular_blocks(geo, qn, pn)
        TA[idx] += 0.5 * (A1 + np.swapaxes(A2, 1, 2))
        TP[idx] += 0.5 * (P1 + np.swapaxes(P2, 1, 2))
    return TA, TP


def z_from_blocks(k, TA, TP, eta=ETA0):
    return eta * (1j * k * TA + TP / (1j * k))


def assemble(mesh, k, near_factor=2.0, eta=ETA0, parts=False, rule=None, far3=None):
    """Full N x N matrix Z (complex128); with parts=True also T_A and T_Phi
    (Z is None when k == 0).  `rule` replaces the 7-point rule (convergence pins);
    far3: ratio of the distance-adaptive far rule (None: off)."""
    geo = Geometry(mesh, rule)
    geo3 = Geometry(mesh, quadrature.strang_fix3()) if far3 is not None else None
    N, T = mesh.n, mesh.t
    TAm = np.zeros((N, N), dtype=np.complex128)
    TPm = np.zeros((N, N), dtype=np.complex128)
    allq = np.arange(T)
    rows_of = mesh.tri_edge                                    # (T, 3)
    for p in range(T):
        TA, TP = pair_blocks(geo, k, p, allq, near_factor, far3, geo3)
        for i in range(3):
            m = rows_of[p, i]
            for j in range(3):
                np.add.at(TAm[m], rows_of[:, j], TA[:, i, j])
                np.add.at(TPm[m], rows_of[:, j], TP[:, i, j])
    Z = z_from_blocks(k, TAm, TPm, eta) if k != 0 else None
    return (Z, TAm, TPm) if parts else Z


def z_rows(mesh, k, rows, near_factor=2.0, eta=ETA0, geo=None, far3=None):
    """Selected rows of Z: (len(rows), N).  Each row m sums its two test triangles."""
    geo = geo or Geometry(mesh)
    geo3 = Geometry(mesh, quadrature.strang_fix3()) if far3 is not None else None
    N, T = mesh.n, mesh.t
    out = np.zeros((len(rows), N), dtype=np.complex128)
    allq = np.arange(T)
    for r, m in enumerate(rows):
        for p in mesh.edge_tri[m]:
            i = int(np.nonzero(mesh.tri_edge[p] == m)[0][0])
            TA, TP = pair_blocks(geo, k, p, allq, near_factor, far3, geo3)
            zb = z_from_blocks(k, TA[:, i, :], TP[:, i, :], eta)  # (T, 3)
            for j in range(3):
                np.add.at(out[r], mesh.tri_edge[:, j], zb[:, j])
    return out


def z_entries(mesh, k, pairs, near_factor=2.0, eta=ETA0, geo=None, far3=None):
    """Individual entries Z_mn for (m, n) pairs, each from its four triangle pairs."""
    geo = geo or Geometry(mesh)
    geo3 = Geometry(mesh, quadrature.strang_fix3()) if far3 is not None else None
    out = np.zeros(len(pairs), dtype=np.complex128)
    for e, (m, n) in enumerate(pairs):
        acc = 0.0 + 0.0j
        for p in mesh.edge_tri[m]:
            i = int(np.nonzero(mesh.tri_edge[p] == m)[0][0])
            for q in mesh.edge_tri[n]:
                j = int(np.nonzero(mesh.tri_edge[q] == n)[0][0])
                TA, TP = pair_blocks(geo, k, p, [q], near_factor, far3, geo3)
                acc += z_from_blocks(k, TA[0, i, j], TP[0, i, j], eta)
        out[e] = acc
    return out


def excitation(mesh, k, khat, pol, e0=1.0, geo=None):
    """V_m(s) = int f_m . E0 pol_s exp(-j k khat_s . r) dS by the 7-point rule.
    khat, pol: (S, 3).  Returns V (S, N)."""
    geo = geo or Geometry(mesh)
    khat = np.atleast_2d(khat)
    pol = np.atleast_2d(pol)
    S = len(khat)
    V = np.zeros((S, mesh.n), dtype=np.complex128)
    f = geo.basis(np.arange(mesh.t))                                   # (T, 3, 7, 3)
    for s in range(S):
        ph = np.exp(-1j * k * np.einsum("tax,x->ta", geo.qp, khat[s]))  # (T, 7)
        fe = np.einsum("tiax,x->tia", f, pol[s])                         # (T, 3, 7)
        contrib = e0 * np.einsum("ta,ta,tia->ti", geo.W, ph, fe)         # (T, 3)
        for i in range(3):
            np.add.at(V[s], mesh.tri_edge[:, i], contrib[:, i])
    return V


def radiation_vectors(mesh, k, dirs, geo=None):
    """a_n(rhat) = int f_n(r') exp(j k rhat . r') dS' by the 7-point rule: (D, N, 3)."""
    geo = geo or Geometry(mesh)
    dirs = np.atleast_2d(dirs)
    out = np.zeros((len(dirs), mesh.n, 3), dtype=np.complex128)
    f = geo.basis(np.arange(mesh.t))
    for d, rh in enumerate(dirs):
        ph = np.exp(1j * k * np.einsum("tax,x->ta", geo.qp, rh))
        contrib = np.einsum("ta,ta,tiax->tix", geo.W, ph, f)            # (T, 3, 3)
        for i in range(3):
            np.add.at(out[d], mesh.tri_edge[:, i], contrib[:, i])
    return out


def sph_basis(dirs):
    """theta-hat and phi-hat for unit vectors dirs (D, 3)."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    th = np.arccos(np.clip(z, -1.0, 1.0))
    ph = np.arctan2(y, x)
    that = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], 1)
    phat = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], 1)
    return that, phat


def farfield(mesh, k, J, dirs, eta=ETA0, geo=None):
    """Far-field pattern F(rhat) = -(j k eta / 4 pi) (I - rhat rhat) . sum_n J_n a_n(rhat),
    returned as (theta, phi) components: (S, D, 2) for currents J (S, N)."""
    J = np.atleast_2d(J)
    dirs = np.atleast_2d(dirs)
    a = radiation_vectors(mesh, k, dirs, geo)                           # (D, N, 3)
    vec = np.einsum("sn,dnx->sdx", J, a)                                # (S, D, 3)
    that, phat = sph_basis(dirs)
    ft = np.einsum("sdx,dx->sd", vec, that)
    fp = np.einsum("sdx,dx->sd", vec, phat)
    c = -1j * k * eta / (4.0 * math.pi)
    return c * np.stack([ft, fp], axis=-1)


def rcs(F, e0=1.0):
    """sigma = 4 pi |F|^2 / |E0|^2 from (..., 2) far-field components."""
    return 4.0 * math.pi * np.sum(np.abs(F) ** 2, axis=-1) / abs(e0) ** 2
