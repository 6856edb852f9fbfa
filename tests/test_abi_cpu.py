"""Host-side checks of libefie that need no GPU: the library loads and exports every
symbol declared in include/efie.h, mesh validation and RWG numbering agree with
the oracle, near-pair classification agrees with the oracle, and calls made
before the device tables exist fail with EFIE_ERR_STATE instead of touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2310_15644_amd as P
import synth
from oracle import efie as oefie
from oracle import rwg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    txt = open(os.path.join(ROOT, "include", "efie.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(efie_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = P.lib()
    syms = _header_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(P.EXPORTED) == syms
    assert L.efie_abi_version() == 1


def test_ktilde_golden():
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "ktilde.txt")) if not l.startswith("#")]
    for k, a, re_, im in rows:
        kt = P.ktilde(float(k), float(a))
        assert abs(kt - complex(float(re_), float(im))) < 1e-14 * max(1.0, float(k))


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_rwg_numbering_matches_oracle(level):
    v, f = synth.icosphere(level)
    m = P.Mesh(v, f)
    om = rwg.build(v, f)
    ev, et = m.rwg_table()
    assert m.n == om.n and m.t == om.t
    assert np.array_equal(ev, om.edges)
    assert np.array_equal(et, om.edge_tri)


@pytest.mark.parametrize("nf", [1.0, 2.0, 3.5])
def test_near_pairs_match_oracle(nf):
    v, f = synth.icosphere(2)
    m = P.Mesh(v, f, near_factor=nf)
    om = rwg.build(v, f)
    assert m.n_near == int(oefie.near_pairs(om, nf).sum())


def test_near_pairs_ellipsoid_matches_oracle():
    v, f = synth.ellipsoid(5, (1.3, 0.7, 0.9))
    m = P.Mesh(v, f)
    om = rwg.build(v, f)
    assert m.n_near == int(oefie.near_pairs(om).sum())


def test_mesh_errors():
    v, f = synth.icosphere(0)
    cases = {
        "open": (v, f[:-1], P.EfieError, -2),
        "orient": (v, np.concatenate([f[:3], f[3:4][:, [0, 2, 1]], f[4:]]), P.EfieError, -4),
        "nonmanifold": (v, np.concatenate([f, f[:1]]), P.EfieError, -3),
    }
    for name, (vv, ff, exc, code) in cases.items():
        with pytest.raises(exc) as ei:
            P.Mesh(vv, ff)
        assert ei.value.code == code, name
    w = v.copy()
    w[f[0, 1]] = w[f[0, 0]]
    with pytest.raises(P.EfieError) as ei:
        P.Mesh(w, f)
    assert ei.value.code == -5
    bad = f.copy()
    bad[0, 0] = 99
    with pytest.raises(P.EfieError) as ei:
        P.Mesh(v, bad)
    assert ei.value.code == -1
    with pytest.raises(P.EfieError):
        P.Mesh(v, f, near_factor=0.0)


def test_far_rule_setter():
    v, f = synth.icosphere(1)
    m = P.Mesh(v, f)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(P.EfieError) as ei:
            m.set_far_rule(bad)
        assert ei.value.code == -1
    assert m.set_far_rule(4.0).far3 == 4.0
    assert m.set_far_rule(0.0).far3 == 0.0
    assert P.lib().efie_mesh_set_far_rule(None, 1.0) == -1


def test_calls_before_upload_fail_cleanly():
    L = P.lib()
    v, f = synth.icosphere(1)
    m = P.Mesh(v, f)
    dummy = ctypes.c_void_p(16)
    assert L.efie_assemble(m._h, 1.0, 0.0, P.ETA0, 0, dummy, None, 0, None) == -9
    assert b"not uploaded" in L.efie_last_error()
    assert L.efie_excite_planewave(m._h, 1.0, dummy, dummy, 1, 1.0, dummy, None) == -9


def test_workspace_sizes():
    L = P.lib()
    nb = ctypes.c_size_t()
    assert L.efie_solve_workspace_size(480, 1, 0, ctypes.byref(nb)) == 0
    b1 = nb.value
    assert L.efie_solve_workspace_size(480, 8, 1, ctypes.byref(nb)) == 0
    assert nb.value > b1 > 7 * 480 * 16
    assert L.efie_solve_workspace_size(0, 1, 0, ctypes.byref(nb)) == -1


def test_ktilde_library_errors():
    with pytest.raises(P.EfieError):
        P.ktilde(0.0)
    with pytest.raises(P.EfieError):
        P.ktilde(1.0, -1.0)


def test_farfield_objective_argument_errors():
    """Rejected on the host before any device work (fake device addresses)."""
    L = P.lib()
    f, j = ctypes.c_void_p(4096), ctypes.c_void_p(8192)
    assert L.efie_farfield_objective(None, 4, j, None, None) == -1   # EFIE_ERR_ARG
    assert L.efie_farfield_objective(f, 4, None, None, None) == -1   # EFIE_ERR_ARG
    assert L.efie_farfield_objective(f, 0, j, None, None) == -1   # EFIE_ERR_ARG
    assert L.efie_farfield_objective(f, 4, j, f, None) == -1   # EFIE_ERR_ARG


def test_fp32_kmax_from_bounding_box():
    """The complex64 assemblies accept |Re k| below 512 pi / (bounding-box diagonal)."""
    v, f = synth.icosphere(2)
    m = P.Mesh(v, f)
    diag = np.linalg.norm(v.max(axis=0) - v.min(axis=0))
    assert abs(m.fp32_kmax() - 512.0 * np.pi / diag) <= 1e-12 * m.fp32_kmax()
    m2 = P.Mesh(v * 10.0, f)
    assert abs(m2.fp32_kmax() * 10.0 - m.fp32_kmax()) <= 1e-12 * m.fp32_kmax()


def test_bie2d_create_checks_the_contour():
    """Host-side checks of the 2-D path's contour: orientation, degenerate segments,
    the Gauss rule; the polygon perimeter (no GPU needed)."""
    import ctypes

    L = P.lib()
    nodes = synth.contour_ellipse(64)
    circ = synth.contour_circle(64)
    h = ctypes.c_void_p()
    rev = np.ascontiguousarray(nodes[::-1])
    assert L.efie_bie2d_create(rev.ctypes.data, circ.ctypes.data, 64, 4, ctypes.byref(h)) == -4
    dup = np.ascontiguousarray(nodes.copy())
    dup[5] = dup[4]
    assert L.efie_bie2d_create(dup.ctypes.data, circ.ctypes.data, 64, 4, ctypes.byref(h)) == -5
    assert L.efie_bie2d_create(nodes.ctypes.data, circ.ctypes.data, 64, 7, ctypes.byref(h)) == -1
    assert L.efie_bie2d_create(nodes.ctypes.data, circ.ctypes.data, 64, 4, ctypes.byref(h)) == 0
    per = ctypes.c_double()
    assert L.efie_bie2d_perimeter(h, 0, ctypes.byref(per)) == 0
    d = np.linalg.norm(np.roll(nodes, -1, axis=0) - nodes, axis=1).sum()
    assert abs(per.value - d) < 1e-13
    L.efie_bie2d_destroy(h)
