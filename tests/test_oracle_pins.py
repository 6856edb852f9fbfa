"""Pins of the FP64 oracle against closed forms, identities and the Mie series.

None of these re-types the oracle's own formula: each value comes from the
mathematics (exact monomial integrals, closed-form potentials, brute-force
quadrature, RWG identities, reciprocity, passivity, power balance, Mie series
and its limits) or from a fixture under tests/golden/.
"""
import math
import os

import numpy as np
import pytest

import synth
from oracle import efie, krylov, mie, quadrature, rwg, singular

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def l1():
    return rwg.build(*synth.icosphere(1))


@pytest.fixture(scope="module")
def l2():
    return rwg.build(*synth.icosphere(2))


@pytest.fixture(scope="module")
def l2_system(l2):
    k = 1.0
    Z = efie.assemble(l2, k)
    kh, pol = synth.planewave_x_along_minus_z()
    V = efie.excitation(l2, k, kh, pol)[0]
    J = np.linalg.solve(Z, V)
    return k, Z, V, J


# ---------------------------------------------------------------- quadrature
def test_radon7_exact_to_degree5():
    bary, w = quadrature.radon7()
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(6):
        for b in range(6 - a):
            for c in range(6 - a - b):
                exact = 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 2)
                got = np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c)
                assert abs(got - exact) < 1e-15, (a, b, c)


def test_radon7_not_degree6():
    bary, w = quadrature.radon7()
    errs = []
    for a in range(7):
        for b in range(7 - a):
            c = 6 - a - b
            exact = 2.0 * math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(8)
            errs.append(abs(np.sum(w * bary[:, 0] ** a * bary[:, 1] ** b * bary[:, 2] ** c) - exact))
    assert max(errs) > 1e-6


# ---------------------------------------------------------------- closed-form potentials
def test_potential_centroid_golden():
    val = float(open(os.path.join(GOLDEN, "potential_centroid.txt")).read().split("\n")[2])
    v = np.array([[0, 0, 0], [1, 0, 0], [0.5, math.sqrt(3) / 2, 0]], dtype=float)
    I0, I1 = singular.potential_integrals(v.mean(0)[None], v)
    assert abs(I0[0] - val) < 1e-14
    assert np.abs(I1[0]).max() < 1e-14          # symmetric about the centroid


def _brute(obs, v, s=6):
    bary, w = quadrature.radon7()
    pts, ws = quadrature.subdivided(bary, w, s)
    P = pts @ v
    A = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    nrm = np.cross(v[1] - v[0], v[2] - v[0])
    nrm /= np.linalg.norm(nrm)
    R = np.linalg.norm(obs - P, axis=1)
    rho = obs - ((obs - v[0]) @ nrm) * nrm
    return A * np.sum(ws / R), A * np.sum(ws[:, None] * (P - rho) / R[:, None], 0)


@pytest.mark.parametrize("where", ["above", "above_outside", "in_plane_outside", "edge_line_extension", "far"])
def test_potential_vs_brute_force(where):
    v = np.array([[0.1, -0.2, 0.05], [1.1, 0.1, 0.0], [0.3, 0.9, -0.1]])
    nrm = np.cross(v[1] - v[0], v[2] - v[0])
    nrm /= np.linalg.norm(nrm)
    c = v.mean(0)
    obs = {
        "above": c + 0.3 * nrm,
        "above_outside": v[0] + 0.2 * (v[0] - v[1]) + 0.1 * nrm,
        "in_plane_outside": c + 2.0 * (v[1] - c),
        "edge_line_extension": v[1] + 0.5 * (v[1] - v[0]),
        "far": c + 40.0 * nrm + 10.0 * (v[2] - v[0]),
    }[where]
    I0, I1 = singular.potential_integrals(obs[None], v)
    b0, b1 = _brute(obs, v)
    assert abs(I0[0] - b0) <= 1e-11 * abs(b0)
    assert np.linalg.norm(I1[0] - b1) <= 1e-10 * max(np.linalg.norm(b1), 1e-300) + 1e-14


def test_potential_far_asymptote():
    v = np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.1, 0]], dtype=float)
    A = 0.005
    c = v.mean(0)
    for Rd in [10.0, 100.0]:
        obs = c + Rd * np.array([0.3, 0.4, math.sqrt(0.75)])
        I0, _ = singular.potential_integrals(obs[None], v)
        assert abs(I0[0] * Rd / A - 1.0) < 5 * (0.1 / Rd) ** 2


# ---------------------------------------------------------------- mesh / RWG
def test_mesh_counts_and_numbering(l2):
    assert (l2.t, l2.n, len(l2.xyz)) == (320, 480, 162)
    assert len(l2.xyz) - l2.n + l2.t == 2
    e = l2.edges
    assert np.all(e[:, 0] < e[:, 1])
    assert np.all(np.lexsort((e[:, 1], e[:, 0])) == np.arange(l2.n))
    for n in range(0, l2.n, 37):
        a, b = e[n]
        tp, tm = l2.edge_tri[n]
        cyc = lambda t: [(l2.tri[t, i], l2.tri[t, (i + 1) % 3]) for i in range(3)]
        assert (a, b) in cyc(tp) and (b, a) in cyc(tm)


def test_mesh_rejections():
    v, f = synth.icosphere(0)
    with pytest.raises(rwg.MeshError):
        rwg.build(v, f[:-1])                         # open
    g = f.copy()
    g[3] = g[3][[0, 2, 1]]
    with pytest.raises(rwg.MeshError):
        rwg.build(v, g)                              # one flipped face
    w = v.copy()
    w[f[0, 1]] = w[f[0, 0]]
    with pytest.raises(rwg.MeshError):
        rwg.build(w, f)                              # degenerate face
    with pytest.raises(rwg.MeshError):
        rwg.build(v, np.concatenate([f, f[:1]]))     # an edge used by three faces


def test_rwg_flux_and_charge(l2):
    geo = efie.Geometry(l2)
    for n in range(0, l2.n, 23):
        a, b = l2.xyz[l2.edges[n]]
        mid = 0.5 * (a + b)
        tp, tm = l2.edge_tri[n]
        ip = int(np.nonzero(l2.tri_edge[tp] == n)[0][0])
        im = int(np.nonzero(l2.tri_edge[tm] == n)[0][0])
        # unit normal to the edge in T+, pointing out of T+ (away from v+)
        t_ = (b - a) / np.linalg.norm(b - a)
        nu = np.cross(t_, l2.normal[tp])
        if np.dot(nu, mid - l2.xyz[l2.edge_free[n, 0]]) < 0:
            nu = -nu
        fpl = rwg.basis_on_triangle(l2, tp, mid[None])[ip, 0]
        fmi = rwg.basis_on_triangle(l2, tm, mid[None])[im, 0]
        assert abs(np.dot(fpl, nu) - 1.0) < 1e-12            # normal component 1: flux l_n
        nu_m = np.cross(t_, l2.normal[tm])
        if np.dot(nu_m, mid - l2.xyz[l2.edge_free[n, 1]]) > 0:
            nu_m = -nu_m
        assert abs(np.dot(fmi, nu_m) - 1.0) < 1e-12          # continuous normal component
        q = geo.div[tp, ip] * l2.area[tp] + geo.div[tm, im] * l2.area[tm]
        assert abs(q) < 1e-14                                # zero net charge


def test_tphi_kernel_is_loops(l1):
    _, TA, TP = efie.assemble(l1, 1.0, parts=True)
    nv = len(l1.xyz)
    # divergence matrix: charge of RWG n on triangle t
    D = np.zeros((l1.t, l1.n))
    for t in range(l1.t):
        for i in range(3):
            D[t, l1.tri_edge[t, i]] = l1.tri_sign[t, i] * l1.edge_len[l1.tri_edge[t, i]]
    ker = np.linalg.svd(D)[2][np.linalg.matrix_rank(D):].T   # divergence-free currents
    assert ker.shape[1] == nv - 1                             # dim = V - 1 (genus 0)
    assert np.abs(TP @ ker).max() < 1e-12 * np.abs(TP).max()
    s = np.linalg.svd(TP, compute_uv=False)
    assert np.sum(s > 1e-10 * s[0]) == l1.t - 1               # rank T - 1


# ---------------------------------------------------------------- operator properties
def test_symmetry_and_passivity(l1):
    for k in (1.0, 3.0):
        Z = efie.assemble(l1, k)
        assert np.abs(Z - Z.T).max() <= 1e-14 * np.abs(Z).max()
        ev = np.linalg.eigvalsh(0.5 * (Z + Z.conj().T))       # radiated power >= 0
        assert ev.min() > -1e-10 * ev.max()


def test_laplace_limits_definite(l1):
    _, TA, TP = efie.assemble(l1, 0.0, parts=True)
    assert np.abs(TA.imag).max() == 0.0 and np.abs(TP.imag).max() == 0.0
    ea = np.linalg.eigvalsh(TA.real)
    ep = np.linalg.eigvalsh(TP.real)
    assert ea.min() > 0.0                                      # SPD
    assert ep.min() > -1e-12 * ep.max()                        # SPSD


def test_entries_rows_full_agree(l1):
    k = 2.0
    Z = efie.assemble(l1, k)
    rows = [0, 17, 119]
    R = efie.z_rows(l1, k, rows)
    assert np.abs(R - Z[rows]).max() <= 1e-13 * np.abs(Z).max()
    pairs = [(0, 0), (5, 77), (119, 3), (40, 41)]
    E = efie.z_entries(l1, k, pairs)
    assert np.abs(E - np.array([Z[m, n] for m, n in pairs])).max() <= 1e-13 * np.abs(Z).max()


def test_green_smooth_small_argument():
    R = np.array([1e-9, 1e-6, 1e-3])
    for k in (2.0, 5.0 - 0.7j):
        got = efie.green_smooth(k, R, 0.0) * 4 * math.pi
        # Taylor series of (exp(-jkR) - 1)/R
        z = -1j * k * R
        ref = sum(z ** n / math.factorial(n) for n in range(1, 9)) / R
        assert np.abs(got - ref).max() <= 1e-12 * abs(k)
    assert efie.green_smooth(3.0, np.array([0.0]), 1e-20)[0] == -3j / (4 * math.pi)


def test_quadrature_convergence_tiny_mesh():
    """7x7 entries converge to the refined-rule limit (octahedron, N = 12)."""
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=float)
    f = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]])
    m = rwg.build(v, f)
    bary, w = quadrature.radon7()
    Zs = [efie.assemble(m, 1.5, rule=quadrature.subdivided(bary, w, s)) for s in range(4)]
    err = [np.abs(Zs[s] - Zs[3]).max() / np.abs(Zs[3]).max() for s in range(3)]
    assert err[0] < 3e-2                                       # near-type entries: O(h^2) outer rule
    assert err[1] < err[0] / 3 and err[2] < err[1] / 3


# ---------------------------------------------------------------- solves, power, Mie
def test_power_balance(l2_system, l2):
    k, Z, V, J = l2_system
    p_in = 0.5 * np.real(np.vdot(J, V))
    x, wx = np.polynomial.legendre.leggauss(24)
    nph = 48
    ph = 2 * math.pi * np.arange(nph) / nph
    th = np.arccos(x)
    D = np.array([[math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)] for t in th for p in ph])
    W = np.repeat(wx, nph) * 2 * math.pi / nph
    F = efie.farfield(l2, k, J[None], D)[0]
    p_rad = np.sum(W * np.sum(np.abs(F) ** 2, -1)) / (2 * efie.ETA0)
    assert abs(p_in - p_rad) <= 1e-8 * p_rad


def test_krylov_reach_lu(l2_system):
    k, Z, V, J = l2_system
    for solver in (krylov.cgs, krylov.cocg):
        x, it, conv, hist = solver(lambda y: Z @ y, V, 1e-8, 2000)
        assert conv and it < 200
        assert np.linalg.norm(Z @ x - V) <= 1.5e-8 * np.linalg.norm(V)
        assert np.linalg.norm(x - J) <= 1e-5 * np.linalg.norm(J)
    assert np.linalg.norm(Z @ J - V) <= 1e-13 * np.linalg.norm(V)


def test_mie_limits():
    for x in (0.1, 1.0, 5.0, 10.0):
        qe, qs = mie.efficiencies(x)
        assert abs(qe - qs) <= 1e-10 * qs                     # optical theorem, lossless
    s = mie.bistatic_rcs(0.01, 1.0, np.array([math.pi]), 0.0)[0] / math.pi
    assert abs(s / (9 * 0.01 ** 4) - 1) < 1e-3                # Rayleigh: 9 (ka)^4
    s = mie.bistatic_rcs(60.0, 1.0, np.array([math.pi]), 0.0)[0] / math.pi
    assert abs(s - 1.0) < 0.05                                # optical limit: pi a^2


def test_mom_converges_to_mie():
    """Bistatic RCS of the MoM sphere approaches Mie as the mesh is refined."""
    k = 1.0
    ts = np.linspace(0.0, math.pi, 13)
    errs = []
    for L in (1, 2):
        m = rwg.build(*synth.icosphere(L))
        Z = efie.assemble(m, k)
        kh, pol = synth.planewave_x_along_minus_z()
        J = np.linalg.solve(Z, efie.excitation(m, k, kh, pol)[0])
        e = 0.0
        for phi in (0.0, math.pi / 2):
            d = np.stack([np.sin(ts) * math.cos(phi), np.sin(ts) * math.sin(phi), -np.cos(ts)], 1)
            s = efie.rcs(efie.farfield(m, k, J[None], d))[0]
            sm = mie.bistatic_rcs(1.0, 1.0, ts, phi)
            e = max(e, np.max(np.abs(10 * np.log10(s / sm))))
        errs.append(e)
    assert errs[1] < 0.5 and errs[1] < errs[0] / 3


# ------------------------------------------------------------ near-pair rule
def _two_tetrahedra(shift, scale_b):
    """A regular tetrahedron A (edge 1) and a copy B scaled by scale_b and moved
    so that the centroid of B's face 0 lies `shift` from that of A's face 0."""
    a = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float) / (2.0 * math.sqrt(2.0))
    f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]])
    b = a * scale_b
    cA = a[f[0]].mean(axis=0)
    cB = b[f[0]].mean(axis=0)
    b = b + (cA - cB) + np.asarray(shift, dtype=float)
    return rwg.build(np.concatenate([a, b]), np.concatenate([f, f + 4]))


@pytest.mark.parametrize("factor,expect", [(1.99, True), (2.01, False)])
def test_near_rule_distance_threshold(factor, expect):
    """Centroid distance just below / above 2 h_max (the default near factor): the
    pair is near / far, whichever triangle is the test triangle, with h_max the
    longest edge of the larger triangle (edge 1 of A, 1/2 of B)."""
    m = _two_tetrahedra([factor, 0.0, 0.0], 0.5)
    assert abs(m.hmax[0] - 1.0) < 1e-15 and abs(m.hmax[4] - 0.5) < 1e-15
    assert abs(np.linalg.norm(m.centroid[4] - m.centroid[0]) - factor) < 1e-14
    assert bool(efie.near_row(m, 0)[4]) is expect
    assert bool(efie.near_row(m, 4)[0]) is expect        # symmetric: max of the two edges


def test_near_rule_uses_larger_edge():
    """At 1.5 h_max(A) the pair is near from both sides; a rule taking the test
    triangle's own edge would call it far from B's side (2 h_B = 1 < 1.5)."""
    m = _two_tetrahedra([0.0, 1.5, 0.0], 0.5)
    assert efie.near_row(m, 4)[0] and efie.near_row(m, 0)[4]
    # scaled by the near factor: 1.5 h < 1.6 h but not < 1.4 h
    assert efie.near_row(m, 0, 1.6)[4] and not efie.near_row(m, 0, 1.4)[4]


def test_near_rule_vertex_sharing():
    """Icosahedron with a vanishing distance factor: the near triangles of a face
    are the ten faces that share at least one vertex with it (itself, three across
    its edges, six touching one corner only), whatever their distance."""
    m = rwg.build(*synth.icosphere(0))
    far_edge = m.hmax.max()
    for p in range(m.t):
        row = efie.near_row(m, p, 1e-6)
        assert row.sum() == 10
        corner_only = [q for q in range(m.t) if len(set(m.tri[q]) & set(m.tri[p])) == 1]
        assert len(corner_only) == 6 and all(row[q] for q in corner_only)
        # a corner-only neighbour lies farther than its own longest edge times 1e-6
        assert all(np.linalg.norm(m.centroid[q] - m.centroid[p]) > 1e-6 * far_edge for q in corner_only)
