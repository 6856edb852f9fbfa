"""Pins of the 3-D Calderon-stabilized CFIE oracle (oracle/cfie.py, the gradient
integral of oracle/singular.py) against closed forms, brute-force quadrature and
the mathematics of the continuous operators -- none re-types the oracle's
formulas:

  * J(r) = int (r - r')/R^3 dS' in closed form against a 28672-point composite
    rule off the triangle, its normal component tending to 2 pi (half the solid
    angle of a plane) just above the triangle, none in the plane;
  * the Taylor branch of (1 + x) exp(-x) - 1 against the direct formula where both
    are accurate, and g_s R -> -k^2/(8 pi) as R -> 0;
  * a near block of K (singularity extraction) against brute-force inner
    integration of the full kernel on an edge-adjacent, non-coplanar pair;
  * consistency of the MFIE discretization: the current of the EFIE satisfies the
    rotated-BC-tested MFIE (1/2 - K) J = n x H^inc to second order in h -- a wrong
    sign, scale or half of K, of the identity term or of H^inc breaks it;
  * the Calderon identity of the continuous operators, (n x T)^2 = -1/4 + K^2:
    at k~ = k the EFIE and MFIE products nearly cancel in difference (not in sum)
    on a smooth current, which fixes the sign of the combination;
  * the stabilized solution equals the EFIE's within discretization error, and at
    the discrete interior resonance of the L1 sphere (sigma_min(Z)/sigma_max(Z) =
    2e-7 at k = 2.8701) C_p keeps a condition number of about 3.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import synth
from oracle import calderon, cfie, efie, quadrature, rwg, singular


def test_gradient_integral_closed_form():
    v = np.array([[0.1, -0.2, 0.05], [1.0, 0.1, -0.1], [0.2, 0.9, 0.2]])
    bw, w = quadrature.radon7()
    pts, ws = quadrature.subdivided(bw, w, 6)
    area = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    rp = pts @ v
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    c = v.mean(0)
    for r in (c + 0.5 * n, c - 0.3 * n, c + np.array([2.0, 0.0, 0.0]), v[0] + np.array([0.3, -0.4, 0.2])):
        d = r[None] - rp
        R = np.linalg.norm(d, axis=1)
        ref = (ws[:, None] * d / R[:, None] ** 3).sum(0) * area
        J = singular.gradient_integral(r[None], v)[0]
        assert np.abs(J - ref).max() <= 1e-11 * np.abs(ref).max()
    assert abs(singular.gradient_integral((c + 1e-7 * n)[None], v)[0] @ n - 2.0 * math.pi) < 1e-5
    assert abs(singular.gradient_integral((c - 1e-7 * n)[None], v)[0] @ n + 2.0 * math.pi) < 1e-5
    assert abs(singular.gradient_integral(c[None], v)[0] @ n) < 1e-15


def test_mfie_kernel_series_and_limit():
    for k in (3.0, complex(7.0, -0.8)):
        R = np.linspace(0.3, 0.49, 9) / abs(k)       # |x| in [0.3, 0.49]: the series branch
        x = 1j * k * R
        direct = (1.0 + x) * np.exp(-x) - 1.0
        assert np.abs(cfie.mfie_numerator(k, R) - direct).max() <= 1e-13 * np.abs(direct).max()
        Rt = np.array([1e-6, 1e-4])
        lim = -(k * k) / (8.0 * math.pi)
        assert np.abs(cfie.g_smooth(k, Rt) * Rt - lim).max() <= 1e-3 * abs(lim)
        # continuity across the switch |x| = 1/2
        Re = np.array([0.5 - 1e-12, 0.5 + 1e-12]) / abs(k)
        a, b = cfie.g_full(k, Re)
        assert abs(a - b) <= 1e-9 * abs(a)


def test_k_near_block_against_brute_force():
    """At k h = 0.15 the 7-point rule of the smooth remainder is accurate, so the
    extracted near blocks must match brute-force inner integration of the full
    kernel (a dropped or mis-signed static term would be an O(1) error)."""
    m = rwg.build(*synth.icosphere(1))
    bary = rwg.build(*calderon.barycentric_refinement(m))
    k = 0.25
    geo_t, geo_s = efie.Geometry(bary), efie.Geometry(m)
    t = 0
    e0 = m.tri_edge[t, 0]
    q = int(m.edge_tri[e0][0] if m.edge_tri[e0][0] != t else m.edge_tri[e0][1])   # shares edge e0 with t
    near = efie.near_row(m, t)
    assert near[q] and abs(m.normal[q] @ m.normal[t]) < 1.0 - 1e-6
    bw, w = quadrature.radon7()
    pts, ws = quadrature.subdivided(bw, w, 6)
    rq = pts @ m.xyz[m.tri[q]]
    for b in range(6 * t, 6 * t + 6):
        blk = cfie.k_blocks(geo_t, geo_s, k, b, t, near)[q]
        ra = geo_t.qp[b]
        dv = ra[:, None, :] - rq[None, :, :]
        R = np.linalg.norm(dv, axis=-1)
        A = np.einsum("c,ac,acx->ax", ws * m.area[q], cfie.g_full(k, R), dv)
        fb = geo_t.basis(b)
        ref = np.zeros((3, 3), dtype=complex)
        for j in range(3):
            arm = ra - geo_s.free[q, j]
            ref[:, j] = geo_s.coef[q, j] * np.einsum("a,iax,ax->i", geo_t.W[b], fb, np.cross(A, arm))
        assert np.abs(blk - ref).max() <= 1e-4 * np.abs(ref).max()
    # the coplanar own triangle contributes nothing (principal value)
    assert np.abs(cfie.k_blocks(geo_t, geo_s, k, 6 * t, t, near)[t]).max() == 0.0


def _efie_current(c, khat, pol):
    V = efie.excitation(c.mesh, c.k, khat, pol)
    return np.linalg.solve(c.cal.Z, V[0])


@pytest.fixture(scope="module")
def l1_k2():
    m = rwg.build(*synth.icosphere(1))
    return cfie.CFIE(m, 2.0, complex(2.0))


def test_mfie_consistency_second_order(l1_k2):
    khat, pol = np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 0.0, 0.0]])
    errs = []
    for c in (l1_k2, None):
        if c is None:
            # level 2 without the barycentric EFIE (not needed here)
            m = rwg.build(*synth.icosphere(2))
            cal = calderon.Calderon.__new__(calderon.Calderon)
            cal.mesh = m
            cal.bary = rwg.build(*calderon.barycentric_refinement(m))
            cal.R = calderon.bc_coefficients(m, cal.bary)
            cal.G = calderon.mixed_gram(m, cal.bary, cal.R)
            cal.Z = efie.assemble(m, 2.0)
            c = cfie.CFIE.__new__(cfie.CFIE)
            c.cal, c.mesh, c.k, c.eta = cal, m, 2.0, efie.ETA0
            c.Kk = cal.R.T @ cfie.k_mixed(cal.bary, m, 2.0)
            c.Mk = -0.5 * cal.G.T - c.Kk
        J = _efie_current(c, khat, pol)
        hm = c.h(khat, pol)[0]
        errs.append(np.linalg.norm(c.Mk @ J - hm) / np.linalg.norm(hm))
    assert errs[1] < 4e-3 and errs[0] / errs[1] > 3.0


def test_calderon_identity_fixes_the_sign(l1_k2):
    c = l1_k2
    J = _efie_current(c, np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e, f = c.efie_term @ J, c.mfie_term @ J
    assert np.linalg.norm(e - f) <= 0.03 * np.linalg.norm(e)
    assert np.linalg.norm(e + f) >= 1.8 * np.linalg.norm(e)
    # both near the identity part +G^T/4 of -1/4 + K^2 in this testing
    assert np.linalg.norm(c.efie_term - 0.25 * c.cal.G.T) <= 0.3 * np.linalg.norm(c.efie_term)


def test_cfie_solution_and_conditioning():
    m = rwg.build(*synth.icosphere(1))
    k = 2.0
    c = cfie.CFIE(m, k, calderon.ktilde(k))
    khat, pol = np.array([[0.0, 0.0, -1.0], [1.0, 0.0, 0.0]]), np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    bp, V = c.rhs(khat, pol)
    for s in range(2):
        jc = np.linalg.solve(c.C, bp[s])
        je = np.linalg.solve(c.cal.Z, V[s])
        assert np.linalg.norm(jc - je) <= 0.012 * np.linalg.norm(je)
    assert np.linalg.cond(c.C) < 6.0


def test_cfie_resonance_free_l1():
    m = rwg.build(*synth.icosphere(1))

    def ratio(k):
        sv = np.linalg.svd(efie.assemble(m, k), compute_uv=False)
        return sv[-1] / sv[0]

    # the discrete counterpart of the first interior resonance ((x j_1(x))' = 0 at 2.7437)
    r = minimize_scalar(ratio, bracket=(2.8, 2.875, 2.95), tol=1e-10)
    assert r.fun < 1e-5
    c = cfie.CFIE(m, r.x, calderon.ktilde(r.x))
    sv = np.linalg.svd(c.efie_term, compute_uv=False)
    assert sv[-1] / sv[0] < 1e-5                     # the Calderon-EFIE inherits it
    assert np.linalg.cond(c.C) < 5.0                 # the stabilized CFIE does not
