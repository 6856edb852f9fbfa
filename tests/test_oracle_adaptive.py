"""Pins of the oracle's distance-adaptive far rule (the 3x3 product of the
interior 3-point degree-2 rule on well-separated triangle pairs; not in the
paper).  Each value comes from the mathematics: exact monomial integrals, a
high-order composite rule as the reference integral, the symmetry of the
Galerkin operator and the Mie series."""
import math

import numpy as np
import pytest

import synth
from oracle import efie, mie, quadrature, rwg


def _monomial(a, b):
    # int over the unit right triangle (0,0), (1,0), (0,1) of x^a y^b = a! b! / (a + b + 2)!
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def test_strang_fix3_is_degree_two():
    bary, w = quadrature.strang_fix3()
    assert abs(w.sum() - 1.0) < 1e-15
    x, y = bary[:, 1], bary[:, 2]                      # vertices (0,0), (1,0), (0,1)
    for a in range(3):
        for b in range(3 - a):
            q = 0.5 * np.sum(w * x ** a * y ** b)      # weights are fractions of the area 1/2
            assert abs(q - _monomial(a, b)) < 1e-15, (a, b)
    worst = max(abs(0.5 * np.sum(w * x ** a * y ** (3 - a)) - _monomial(a, 3 - a)) for a in range(4))
    assert worst > 1e-4                                # not exact at degree 3


@pytest.fixture(scope="module")
def l2():
    return rwg.build(*synth.icosphere(2))


def test_far3_off_and_huge_ratio_are_the_seven_point_rule(l2):
    k = 1.3
    Z7 = efie.z_rows(l2, k, [0, 77])
    Zbig = efie.z_rows(l2, k, [0, 77], far3=1e6)
    assert np.array_equal(Z7, Zbig)


def test_far3_classification(l2):
    """The rule's pair set is symmetric and is the set D >= 3 h (distances taken
    here by numpy's norm; the two may differ only on pairs within rounding of the
    threshold)."""
    for p in (0, 33, 300):
        f = efie.far3_row(l2, p, 3.0)
        assert f.sum() > 0
        for q in np.nonzero(f)[0]:
            assert efie.far3_row(l2, q, 3.0)[p]
        d = np.linalg.norm(l2.centroid - l2.centroid[p], axis=1)
        lim = 3.0 * np.maximum(l2.hmax, l2.hmax[p])
        diff = f != (d >= lim)
        assert np.all(np.abs(d - lim)[diff] < 1e-12)


def test_far3_pair_blocks_against_a_high_order_reference(l2):
    """On far pairs the 3x3 blocks integrate the same integrand as the 7x7 ones:
    both approach the composite 7-point rule (16 sub-triangles per triangle) as
    the reference, the 3x3 rule within its degree-2 error, the 7x7 within its
    degree-5 error."""
    k = 2.0
    ref = quadrature.subdivided(*quadrature.radon7(), 2)
    g7 = efie.Geometry(l2)
    g3 = efie.Geometry(l2, quadrature.strang_fix3())
    gr = efie.Geometry(l2, ref)
    rng = np.random.default_rng(5)
    e3, e7 = [], []
    for p in rng.choice(l2.t, 6, replace=False):
        qs = np.nonzero(efie.far3_row(l2, p, 4.0) & ~efie.near_row(l2, p))[0][:40]
        A7, P7 = efie.pair_blocks(g7, k, p, qs)
        A3, P3 = efie.pair_blocks(g7, k, p, qs, far3=4.0, geo3=g3)
        Ar, Pr = efie.pair_blocks(gr, k, p, qs)
        sa, sp = np.abs(Ar).max(), np.abs(Pr).max()
        e3.append(max(np.abs(A3 - Ar).max() / sa, np.abs(P3 - Pr).max() / sp))
        e7.append(max(np.abs(A7 - Ar).max() / sa, np.abs(P7 - Pr).max() / sp))
    assert max(e3) < 2e-3          # observed 1e-4 .. 5e-4
    assert max(e7) < 1e-6          # observed ~1e-7
    assert max(e7) < max(e3) / 100


def test_far3_operator_symmetric_and_close_to_seven_point(l2):
    k = 1.0
    Z7 = efie.assemble(l2, k)
    Z3 = efie.assemble(l2, k, far3=3.0)
    assert np.abs(Z3 - Z3.T).max() <= 1e-13 * np.abs(Z3).max()
    rel = np.linalg.norm(Z3 - Z7) / np.linalg.norm(Z7)
    assert 1e-9 < rel < 1e-4
    # bistatic RCS against the Mie series: the adaptive rule changes the error by
    # far less than the discretisation error itself
    kh, pol = synth.planewave_x_along_minus_z()
    V = efie.excitation(l2, k, kh, pol)[0]
    ts = np.linspace(0.0, math.pi, 19)
    err = []
    for Z in (Z7, Z3):
        J = np.linalg.solve(Z, V)
        e = 0.0
        for phi in (0.0, math.pi / 2):
            d = np.stack([np.sin(ts) * math.cos(phi), np.sin(ts) * math.sin(phi), -np.cos(ts)], 1)
            s = efie.rcs(efie.farfield(l2, k, J[None], d))[0]
            e = max(e, np.max(np.abs(10 * np.log10(s / mie.bistatic_rcs(k, 1.0, ts, phi)))))
        err.append(e)
    assert abs(err[1] - err[0]) < 0.01
