"""GPU parity of the paper's 2-D method (the library's efie_bie2d_* calls) against
the oracle (oracle/bie2d.py) on the same seeded contours and test matrices:

  * the operator matrices S_k, D*_k, N_k (real k and the complex k~), entry by
    entry on small contours (several assembly tiles and a ragged tail) and on
    sampled rows of a large one;
  * the counterpart's first column and its inverse's, C_p X, C_p^T X, G^-1 X, the
    right-hand sides e, h, b_p and the far field;
  * the fast direct solver with the oracle's test matrix: the same rank, the same
    projector U V^T and the same solution; the Woodbury identity; rank 0 for the
    circle against itself; the PEC-cylinder current of the series solution;
  * TE incidence: C_p^TE X, (C_p^TE)^T X, the TE counterpart, e_t, h_z, b_p and the
    TE far field against the oracle's System(pol="TE"); the same rank and solution
    as the oracle's fast direct solver; the TE cylinder current and echo width.
"""
import math

import numpy as np
import pytest

import synth
from oracle import bie2d as ob

from .gpu_common import flush

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2310_15644_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def _pair(N, geom="ellipse"):
    nodes = {"ellipse": synth.contour_ellipse, "airfoil": synth.contour_joukowsky,
             "circle": synth.contour_circle}[geom](N)
    return nodes, synth.contour_circle(N)


@pytest.mark.parametrize("N,k,q", [(47, 6.0, 4), (124, 10.0, 4), (61, 3.0, 6)])
def test_operators_match_oracle(dev, N, k, q):
    nodes, circ = _pair(N)
    h = P.Bie2d(nodes, circ, q=q, device=dev)
    c = ob.Contour(nodes)
    for kap in (complex(k), ob.ktilde(k)):
        flush(f"bie2d operators N={N} k={kap} q={q}")
        S, D, Nm = (t.cpu().numpy() for t in h.assemble(kap))
        So, Do, No = ob.assemble(c, kap, q)
        e = (rel(S, So), rel(D, Do), rel(Nm, No))
        flush(f"  rel max err S {e[0]:.2e} D* {e[1]:.2e} N {e[2]:.2e}")
        assert max(e) <= 1e-11
    # a window of the circle's matrices (the counterpart's first column path)
    S1, D1, N1 = (t.cpu().numpy() for t in h.assemble(k, which=1, rows=slice(0, N), cols=slice(0, 1)))
    So, Do, No = ob.assemble(ob.Contour(circ), complex(k), q)
    assert rel(S1[:, 0], So[:, 0]) <= 1e-11 and rel(D1[:, 0], Do[:, 0]) <= 1e-11 and rel(N1[:, 0], No[:, 0]) <= 1e-11


def test_operator_rows_large(dev):
    """N = 3001 (201 x 201 assembly tiles, ragged tail), k = 150 (20 nodes per
    wavelength on the airfoil of perimeter 2 pi): sampled rows against the oracle's."""
    N, k = 3001, 150.0
    nodes, circ = _pair(N, "airfoil")
    h = P.Bie2d(nodes, circ, device=dev)
    c = ob.Contour(nodes)
    rows = [0, 1, 1499, 2999, 3000]
    for kap in (complex(k), ob.ktilde(k)):
        flush(f"bie2d rows N={N} k={kap}")
        S, D, Nm = (t.cpu().numpy() for t in h.assemble(kap))
        So, Do, No = ob.assemble_rows(c, kap, rows)
        e = (rel(S[rows], So), rel(D[rows], Do), rel(Nm[rows], No))
        flush(f"  rel max err S {e[0]:.2e} D* {e[1]:.2e} N {e[2]:.2e}")
        assert max(e) <= 1e-11
        assert np.abs(S - S.T).max() <= 1e-13 * np.abs(S).max()
        assert np.abs(Nm - Nm.T).max() <= 1e-12 * np.abs(Nm).max()


@pytest.fixture(scope="module")
def ellipse180(dev):
    N, k = 180, 10.0
    nodes, circ = _pair(N)
    kt = ob.ktilde(k)
    so = ob.System(ob.Contour(nodes), k, kt)
    sc = ob.System(ob.Contour(circ), k, kt)
    h = P.Bie2d(nodes, circ, device=dev).setup(k, kt, rmax=N, block=16, nvec=64)
    return N, k, kt, h, so, sc


def test_apply_and_rhs(dev, ellipse180):
    N, k, kt, h, so, sc = ellipse180
    flush("bie2d C_p, C_p^T, G^-1, counterpart, rhs")
    Cp, Cc = so.calderon(), sc.calderon()
    g = torch.Generator(device=dev).manual_seed(3)
    X = torch.randn((7, N), dtype=torch.complex128, device=dev, generator=g)
    Xn = X.cpu().numpy()
    assert rel(h.apply("cp", X).cpu().numpy(), (Cp @ Xn.T).T) <= 1e-11
    assert rel(h.apply("cpt", X).cpu().numpy(), (Cp.T @ Xn.T).T) <= 1e-11
    assert rel(h.apply("ginv", X).cpu().numpy(), np.linalg.solve(so.G, Xn.T).T) <= 1e-13
    assert rel(h.apply("a", X).cpu().numpy(), ((Cp - Cc) @ Xn.T).T) <= 1e-10
    col, coli = (t.cpu().numpy() for t in h.counterpart())
    assert rel(col, Cc[:, 0]) <= 1e-11
    assert rel(coli, np.linalg.inv(Cc)[:, 0]) <= 1e-10
    assert rel(h.apply("ccinv", X).cpu().numpy(), np.linalg.solve(Cc, Xn.T).T) <= 1e-10
    phis = np.array([0.0, 0.7, 2.5])
    e, hv, bp = (t.cpu().numpy() for t in h.rhs(phis))
    eo, ho = ob.excitation(so.c, k, phis)
    assert rel(e, eo) <= 1e-13 and rel(hv, ho) <= 1e-13
    assert rel(bp, so.calderon_rhs(eo, ho)) <= 1e-11
    J = torch.as_tensor(np.linalg.solve(Cp, so.calderon_rhs(eo, ho).T).T, device=dev).contiguous()
    obs = np.linspace(0.0, 2.0 * math.pi, 37)
    assert rel(h.farfield(k, J, obs).cpu().numpy(), ob.farfield(so.c, k, J.cpu().numpy(), obs)) <= 1e-12


def test_fast_direct_solver_matches_oracle(dev, ellipse180):
    N, k, kt, h, so, sc = ellipse180
    Cp, Cc = so.calderon(), sc.calderon()
    om = synth.gaussian_block(N, N, seed=0)
    for tol in (1e-3, 1e-5):
        flush(f"bie2d skeleton N={N} k={k} tol={tol}")
        fo = ob.FastDirect(Cp, Cc, om, 16, tol)
        r, est, ref = h.skeleton(torch.as_tensor(om.T.copy(), device=dev), tol)
        flush(f"  rank gpu {r} oracle {fo.rank}; est/ref gpu {est / ref:.3e} oracle {fo.est / fo.ref:.3e}")
        assert r == fo.rank
        assert abs(ref - fo.ref) <= 1e-11 * fo.ref
        U, Vt = (t.cpu().numpy() for t in h.factors())
        Uf = U.T                                     # columns
        assert np.abs(Uf.conj().T @ Uf - np.eye(r)).max() <= 1e-12
        # same projector U U^H and same skeleton U V^T (the bases differ by a unitary)
        assert rel(Uf @ Uf.conj().T, fo.Q @ fo.Q.conj().T) <= 1e-9
        assert rel(Uf @ Vt, fo.Q @ fo.Vt) <= 1e-9
        e, hv, bp = h.rhs([0.0, 1.2, 2.9])
        X = h.solve(bp).cpu().numpy()
        Xo = fo.solve(bp.cpu().numpy().T).T
        flush(f"  Woodbury solution vs oracle: {rel(X, Xo):.2e}")
        assert rel(X, Xo) <= 1e-9
        # the Woodbury formula inverts C_c + U V^T
        lhs = (Cc @ X.T).T + ((Uf @ Vt) @ X.T).T
        assert rel(lhs, bp.cpu().numpy()) <= 1e-11
        xd = np.linalg.solve(Cp, bp.cpu().numpy().T).T
        assert rel(X, xd) <= 10 * tol * np.linalg.cond(Cp)


def test_circle_rank_zero_and_cylinder_current(dev):
    """The circle against its own counterpart has nothing to compress: rank 0, and
    the solution is the circulant solve, which reproduces the series current."""
    N, k = 400, 12.0
    circ = synth.contour_circle(N)
    h = P.Bie2d(circ, circ, device=dev).setup(k, rmax=64, block=16, nvec=16)
    om = synth.gaussian_block(N, 32, seed=1)
    r, est, ref = h.skeleton(torch.as_tensor(om.T.copy(), device=dev), 1e-6)
    assert r == 0
    e, hv, bp = h.rhs([0.4])
    J = h.solve(bp).cpu().numpy()[0]
    ja = ob.cylinder_current(k, 1.0, 2.0 * math.pi * np.arange(N) / N, 0.4)
    err = np.linalg.norm(J - ja) / np.linalg.norm(ja)
    flush(f"bie2d circle N={N} k={k}: current vs series {err:.2e}")
    assert err <= 3e-3


def test_bie2d_errors(dev):
    nodes, circ = _pair(40)
    with pytest.raises(P.EfieError):
        P.Bie2d(nodes[::-1].copy(), circ, device=dev)        # clockwise
    h = P.Bie2d(nodes, circ, device=dev)
    with pytest.raises(P.EfieError):
        h.apply("cp", torch.zeros((1, 40), dtype=torch.complex128, device=dev))   # no setup yet
    with pytest.raises(P.EfieError):
        h.setup(5.0, rmax=16, block=65, nvec=65)             # blocks of at most 64 columns
    with pytest.raises(ValueError):
        h.setup(5.0, rmax=16, block=16, nvec=16, pol="TEM")
    h.setup(5.0, rmax=16, block=16, nvec=16)
    om = synth.gaussian_block(40, 40, seed=0)
    with pytest.raises(P.EfieError):
        h.skeleton(torch.as_tensor(om.T.copy(), device=dev), 1e-12)   # rank would exceed rmax


@pytest.fixture(scope="module")
def airfoil_te(dev):
    N, k = 160, 8.0
    nodes, circ = _pair(N, "airfoil")
    kt = ob.ktilde(k)
    so = ob.System(ob.Contour(nodes), k, kt, pol="TE")
    sc = ob.System(ob.Contour(circ), k, kt, pol="TE")
    h = P.Bie2d(nodes, circ, device=dev).setup(k, kt, rmax=N, block=16, nvec=64, pol="TE")
    return N, k, kt, h, so, sc


def test_te_apply_rhs_farfield(dev, airfoil_te):
    N, k, kt, h, so, sc = airfoil_te
    flush("bie2d TE: C_p, C_p^T, counterpart, rhs, far field")
    Cp, Cc = so.calderon(), sc.calderon()
    g = torch.Generator(device=dev).manual_seed(5)
    X = torch.randn((5, N), dtype=torch.complex128, device=dev, generator=g)
    Xn = X.cpu().numpy()
    e = (rel(h.apply("cp", X).cpu().numpy(), (Cp @ Xn.T).T), rel(h.apply("cpt", X).cpu().numpy(), (Cp.T @ Xn.T).T),
         rel(h.apply("a", X).cpu().numpy(), ((Cp - Cc) @ Xn.T).T))
    flush(f"  rel err C_p {e[0]:.2e} C_p^T {e[1]:.2e} C_p - C_c {e[2]:.2e}")
    assert e[0] <= 1e-11 and e[1] <= 1e-11 and e[2] <= 1e-10
    col, coli = (t.cpu().numpy() for t in h.counterpart())
    assert rel(col, Cc[:, 0]) <= 1e-11 and rel(coli, np.linalg.inv(Cc)[:, 0]) <= 1e-10
    phis = np.array([0.2, 1.9, 4.0])
    et, hz, bp = (t.cpu().numpy() for t in h.rhs(phis))
    eo, ho = ob.excitation_te(so.c, k, phis)
    assert rel(et, eo) <= 1e-13 and rel(hz, ho) <= 1e-13
    assert rel(bp, so.calderon_rhs(eo, ho)) <= 1e-11
    J = np.linalg.solve(Cp, so.calderon_rhs(eo, ho).T).T
    obs = np.linspace(0.0, 2.0 * math.pi, 41)
    F = h.farfield(k, torch.as_tensor(J, device=dev).contiguous(), obs).cpu().numpy()
    assert rel(F, ob.farfield(so.c, k, J, obs, pol="TE")) <= 1e-12
    F_tm = h.farfield(k, torch.as_tensor(J, device=dev).contiguous(), obs, pol="TM").cpu().numpy()
    assert rel(F_tm, ob.farfield(so.c, k, J, obs)) <= 1e-12


def test_te_fast_direct_solver_matches_oracle(dev, airfoil_te):
    N, k, kt, h, so, sc = airfoil_te
    Cp, Cc = so.calderon(), sc.calderon()
    om = synth.gaussian_block(N, N, seed=2)
    tol = 1e-5
    flush(f"bie2d TE skeleton N={N} k={k} tol={tol}")
    fo = ob.FastDirect(Cp, Cc, om, 16, tol)
    r, est, ref = h.skeleton(torch.as_tensor(om.T.copy(), device=dev), tol)
    flush(f"  rank gpu {r} oracle {fo.rank}")
    assert r == fo.rank
    U, Vt = (t.cpu().numpy() for t in h.factors())
    assert rel(U.T @ Vt, fo.Q @ fo.Vt) <= 1e-9
    e, hv, bp = h.rhs([0.0, 2.2])
    X = h.solve(bp).cpu().numpy()
    assert rel(X, fo.solve(bp.cpu().numpy().T).T) <= 1e-9
    xd = np.linalg.solve(Cp, bp.cpu().numpy().T).T
    assert rel(X, xd) <= 10 * tol * np.linalg.cond(Cp)


def test_te_cylinder_current_and_echo_width(dev):
    """TE on the circle (rank 0 against itself) at x = 1.8412, the first zero of J_1'
    where the TE EFIE alone is singular: the series current and echo width."""
    N, k = 400, 1.8411837813406593
    circ = synth.contour_circle(N)
    h = P.Bie2d(circ, circ, device=dev).setup(k, rmax=64, block=16, nvec=16, pol="TE")
    r, est, ref = h.skeleton(torch.as_tensor(synth.gaussian_block(N, 32, seed=3).T.copy(), device=dev), 1e-6)
    assert r == 0
    e, hv, bp = h.rhs([0.4])
    J = h.solve(bp)
    ja = ob.cylinder_current_te(k, 1.0, 2.0 * math.pi * np.arange(N) / N, 0.4)
    err = np.linalg.norm(J.cpu().numpy()[0] - ja) / np.linalg.norm(ja)
    obs = np.linspace(0.0, 2.0 * math.pi, 73)
    sw = ob.echo_width(k, h.farfield(k, J, obs).cpu().numpy()[0], pol="TE")
    sa = ob.cylinder_echo_width_te(k, 1.0, obs, 0.4)
    keep = 10 * np.log10(sa / sa.max()) > -30
    db = np.abs(10 * np.log10(sw / sa))[keep].max()
    flush(f"bie2d TE circle N={N} k={k}: current vs series {err:.2e}, echo width {db:.3f} dB")
    assert err <= 1e-3 and db < 0.02
