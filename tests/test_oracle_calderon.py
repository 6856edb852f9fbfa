"""Pins of the Calderon oracle: Buffa-Christiansen construction invariants, Gram
conditioning, and the Calderon identity's effect (bounded conditioning of the
preconditioned operator while that of Z grows as the mesh is refined)."""
import numpy as np
import pytest

import paper_2310_15644_amd as P
import synth
from oracle import calderon, efie, krylov, rwg


def _bc(level):
    m = rwg.build(*synth.icosphere(level))
    xyz, tri = calderon.barycentric_refinement(m)
    b = rwg.build(xyz, tri)
    R = calderon.bc_coefficients(m, b)
    return m, b, R


@pytest.mark.parametrize("level", [0, 1, 2])
def test_bc_charges(level):
    m, b, R = _bc(level)
    # charge of each BC function on each barycentric triangle
    D = np.zeros((b.t, b.n))
    for t in range(b.t):
        for i in range(3):
            e = b.tri_edge[t, i]
            D[t, e] = b.tri_sign[t, i] * b.edge_len[e]
    Q = D @ R                                       # (bary triangles, N)
    assert np.abs(Q.sum(axis=0)).max() < 1e-14      # zero net charge
    V = len(m.xyz)
    for n in range(0, m.n, max(1, m.n // 17)):
        a, c = m.edges[n]
        for vert, sign in ((a, 1.0), (c, -1.0)):
            cell = [t for t in range(b.t) if vert in b.tri[t]]
            q = Q[cell, n]
            assert np.allclose(q, sign / len(cell), atol=1e-14)   # equal charge per triangle of the cell
        others = [t for t in range(b.t) if a not in b.tri[t] and c not in b.tri[t]]
        assert np.abs(Q[others, n]).max() < 1e-15
    assert b.t == 6 * m.t and b.n == 9 * m.t and len(b.xyz) == V + m.n + m.t


def test_mixed_gram_conditioning_bounded():
    conds = []
    for level in (1, 2, 3):
        m, b, R = _bc(level)
        G = calderon.mixed_gram(m, b, R)
        s = np.linalg.svd(G, compute_uv=False)
        conds.append(s[0] / s[-1])
    assert max(conds) < 3.5 and max(conds) / min(conds) < 1.3, conds


def test_calderon_bounded_spectrum_l1():
    """kappa(M) small and iterations few, against a growing kappa(Z); also at low frequency."""
    m = rwg.build(*synth.icosphere(1))
    kh, pol = synth.planewave_x_along_minus_z()
    # (k, bound on kappa(M), minimum kappa(Z)/kappa(M), iteration cap); measured 2.3 / 7.1
    for k, cmax, ratio, itmax in ((1.0, 3.0, 10.0, 15), (0.1, 10.0, 300.0, 25)):
        C = calderon.Calderon(m, k, calderon.ktilde(k))
        cm, cz = np.linalg.cond(C.M), np.linalg.cond(C.Z)
        assert cm < cmax and cz > ratio * cm, (k, cm, cz)
        V = efie.excitation(m, k, kh, pol)[0]
        J = np.linalg.solve(C.Z, V)
        x, it, conv, _ = krylov.cgs(lambda y: C.M @ y, C.rhs(V), 1e-10, 500)
        assert conv and it <= itmax, (k, it)
        assert np.linalg.norm(x - J) <= 1e-8 * np.linalg.norm(J)


def test_host_library_matches_oracle_bc_and_gram():
    """The library's host-side construction (no GPU) against the oracle."""
    for level in (1, 2):
        v, f = synth.icosphere(level)
        c = P.Calderon(P.Mesh(v, f))
        R, G = c.host_matrices()
        m, b, Ro = _bc(level)
        assert np.abs(R - Ro).max() <= 1e-14 * np.abs(Ro).max()
        Go = calderon.mixed_gram(m, b, Ro)
        assert np.abs(G - Go).max() <= 1e-14 * np.abs(Go).max()


def test_ktilde_golden():
    """k~ of the paper's Sec. III against values evaluated by hand at exact cube roots."""
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "ktilde.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for k, a, re_, im in rows:
        kt = calderon.ktilde(float(k), float(a))
        assert abs(kt - complex(float(re_), float(im))) <= 1e-15 * float(k), (k, a, kt)
    # the damping grows as k^(1/3) and falls as a^(-2/3): exact ratios between rows
    assert calderon.ktilde(8.0).imag == 2.0 * calderon.ktilde(1.0).imag
    assert calderon.ktilde(1.0, 8.0).imag == 0.25 * calderon.ktilde(1.0).imag
