"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (derived in the design notes):
  FP64 operator entries: max |dZ| <= 1e-11 max |Z| (rounding-order differences only);
  complex64 operator: max |dZ| <= 2e-5 max |Z| (FP32 phase/distance rounding);
  excitation, far field: 1e-12 relative;
  solves: ||J - J_LU|| <= 10 tol kappa-bounded, iteration counts within +-2 of the oracle's
  own Krylov on the same operator.
"""
import ctypes
import math

import numpy as np
import pytest

import synth
from oracle import calderon as ocal
from oracle import efie as oefie
from oracle import krylov as okrylov
from oracle import rwg

from .gpu_common import bipyramid, flush, icosphere, oracle_mesh, rel_max, tetrahedron

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2310_15644_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    return torch.device("cuda:0")


def gmesh(v, f, dev, nf=2.0):
    return P.Mesh(v, f, near_factor=nf).upload(dev)


# ------------------------------------------------------------ assembly
@pytest.mark.parametrize("k", [1.0, 3.0])
def test_assemble_c128_l2_full(dev, k):
    flush(f"assemble c128 L2 k={k}")
    v, f = icosphere(2)
    Zg = P.assemble(gmesh(v, f, dev), k).cpu().numpy()
    Zo = oefie.assemble(oracle_mesh(2), k)
    assert rel_max(Zg, Zo) <= 1e-11
    assert np.abs(Zg - Zg.T).max() <= 1e-14 * np.abs(Zg).max()


@pytest.mark.parametrize("k", [1.0 - 0.4j, 5.0 - 0.68399j])
def test_assemble_parts_complex_k(dev, k):
    flush(f"assemble parts L1 k={k}")
    v, f = icosphere(1)
    TA, TP = P.assemble(gmesh(v, f, dev), k, parts=True)
    _, TAo, TPo = oefie.assemble(oracle_mesh(1), k, parts=True)
    assert rel_max(TA.cpu().numpy(), TAo) <= 1e-11
    assert rel_max(TP.cpu().numpy(), TPo) <= 1e-11


def test_assemble_complex_k_z(dev):
    k = ocal.ktilde(3.0)   # the complex wavenumber of the preconditioner at k = 3
    v, f = icosphere(2)
    Zg = P.assemble(gmesh(v, f, dev), k).cpu().numpy()
    Zo = oefie.assemble(oracle_mesh(2), k)
    assert rel_max(Zg, Zo) <= 1e-11


def test_assemble_c64_l2(dev):
    flush("assemble c64 L2")
    v, f = icosphere(2)
    Zg = P.assemble(gmesh(v, f, dev), 1.0, dtype=P.C64).cpu().numpy()
    Zo = oefie.assemble(oracle_mesh(2), 1.0)
    err = rel_max(Zg.astype(np.complex128), Zo)
    flush(f"  c64 max rel err {err:.3e}")
    assert err <= 2e-5


@pytest.mark.parametrize("shape", ["tetrahedron", "bipyramid"])
def test_assemble_tiny_meshes(dev, shape):
    v, f = {"tetrahedron": tetrahedron, "bipyramid": bipyramid}[shape]()
    om = rwg.build(v, f)
    for k in (0.7, 2.0 - 0.3j):
        Zg = P.assemble(gmesh(v, f, dev), k).cpu().numpy()
        assert rel_max(Zg, oefie.assemble(om, k)) <= 1e-11


@pytest.mark.parametrize("nf", [1.0, 3.0])
def test_assemble_near_factor(dev, nf):
    v, f = icosphere(1)
    Zg = P.assemble(gmesh(v, f, dev, nf), 2.0).cpu().numpy()
    assert rel_max(Zg, oefie.assemble(oracle_mesh(1), 2.0, near_factor=nf)) <= 1e-11


@pytest.mark.parametrize("level", [2, 3])
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_assemble_tiles_vs_atomic(dev, dt, level):
    """The tile path (Z written once by owner-computes tiles; L2: 480 RWGs, 8 x 8
    tiles of 64 or 15 x 15 of 32, ragged; L3: 1920) against the atomic path,
    bit-identical when repeated and exactly symmetric; its workspace holds the
    near-pair blocks only."""
    flush(f"assemble tiles vs atomic {dt} L{level}")
    v, f = icosphere(level)
    m = gmesh(v, f, dev)
    code = P.C128 if dt == "c128" else P.C64
    lo, full = ctypes.c_size_t(), ctypes.c_size_t()
    assert P.lib().efie_assemble_workspace_size(m._h, code, ctypes.byref(lo), ctypes.byref(full)) == 0
    assert lo.value == full.value == max(256, m.n_near * 9 * (16 if dt == "c128" else 8))
    Za = P.assemble(m, 2.0, dtype=code, atomic=True).cpu().numpy()
    Z1 = P.assemble(m, 2.0, dtype=code).cpu().numpy()
    Z2 = P.assemble(m, 2.0, dtype=code).cpu().numpy()
    assert np.array_equal(Z1, Z2)
    tol = 1e-14 if dt == "c128" else 2e-7
    assert rel_max(Z1, Za) <= tol
    assert np.array_equal(Z1, Z1.T)


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_assemble_two_host_threads(dev, dt):
    """Two host threads assemble at once, each on its own stream: both results
    equal the serial one bit for bit."""
    import threading
    flush(f"assemble from two host threads {dt}")
    v, f = icosphere(2)
    m = gmesh(v, f, dev)
    code = P.C128 if dt == "c128" else P.C64
    lo, full = ctypes.c_size_t(), ctypes.c_size_t()
    assert P.lib().efie_assemble_workspace_size(m._h, code, ctypes.byref(lo), ctypes.byref(full)) == 0
    wsb = 7 * lo.value
    ref = P.assemble(m, 2.0, dtype=code, workspace_bytes=wsb).cpu().numpy()
    out, errs = [None, None], []

    def work(i):
        try:
            st = torch.cuda.Stream(device=dev)
            with torch.cuda.stream(st):
                Z = P.assemble(m, 2.0, dtype=code, workspace_bytes=wsb)
            st.synchronize()
            out[i] = Z.cpu().numpy()
        except Exception as e:  # reported by the main thread
            errs.append(e)

    ths = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    assert not errs, errs
    assert np.array_equal(out[0], ref) and np.array_equal(out[1], ref)


def test_assemble_ws_too_small(dev):
    v, f = icosphere(1)
    m = gmesh(v, f, dev)
    lo, full = ctypes.c_size_t(), ctypes.c_size_t()
    assert P.lib().efie_assemble_workspace_size(m._h, P.C128, ctypes.byref(lo), ctypes.byref(full)) == 0
    Z = torch.empty((m.n, m.n), dtype=torch.complex128, device=dev)
    ws = torch.empty(lo.value, dtype=torch.uint8, device=dev)
    rc = P.lib().efie_assemble_ws(m._h, 1.0, 0.0, P.ETA0, P.C128, P._ptr(Z), P._ptr(ws), lo.value - 16,
                                  P._stream(dev))
    assert rc == -1 and b"workspace" in P.lib().efie_last_error()


@pytest.mark.parametrize("k", [0.1, 5.0])
def test_assemble_l4_sampled_rows(dev, k):
    flush(f"assemble L4 k={k} sampled rows")
    v, f = icosphere(4)
    Zg = P.assemble(gmesh(v, f, dev), k)
    rows = [0, 3001, 7679]
    got = Zg[rows].cpu().numpy()
    ref = oefie.z_rows(oracle_mesh(4), k, rows)
    for r in range(len(rows)):
        assert rel_max(got[r], ref[r]) <= 1e-11
    # symmetry at full size, sampled block
    blk = Zg[:512, :512].cpu().numpy()
    assert np.abs(blk - blk.T).max() <= 1e-14 * np.abs(blk).max()


def test_assemble_l5_sampled_entries_c64(dev):
    """Full size (level 5, N = 30720, k = 10), complex64 tile assembly as the
    bench runs it: sampled entries, the diagonal and a near pair among them,
    against the oracle's, one by one."""
    flush("assemble L5 c64 sampled entries")
    v, f = icosphere(5)
    m = gmesh(v, f, dev)
    Zg = P.assemble(m, 10.0, dtype=P.C64)
    zmax = float(Zg.abs().max())
    rng = np.random.default_rng(23)
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, m.n, size=(12, 2))] + [(7, 7), (30719, 30719), (200, 201)]
    ref = oefie.z_entries(oracle_mesh(5), 10.0, pairs)
    got = np.array([complex(Zg[a, b]) for a, b in pairs])
    err = np.abs(got - ref).max() / zmax
    flush(f"  max err / max|Z| {err:.3e}")
    assert err <= 2e-5
    assert abs(complex(Zg[5, 9000]) - complex(Zg[9000, 5])) <= 1e-7 * zmax
    del Zg


# ------------------------------------------------------- excitation / far field
def test_excitation_l2(dev):
    v, f = icosphere(2)
    m = gmesh(v, f, dev)
    rhat, khat, pol, _, _ = synth.monostatic_grid(2, 3)
    Vg = P.excite_planewave(m, 2.5, khat, pol).cpu().numpy()
    Vo = oefie.excitation(oracle_mesh(2), 2.5, khat, pol)
    assert rel_max(Vg, Vo) <= 1e-12


def test_excitation_and_farfield_l5_bench_shape(dev):
    """Full size (level 5, N = 30720, k = 10) as the bench runs them: the 512
    plane waves of the monostatic grid excited at once, 16 of them against the
    oracle over every RWG; the far field of seeded currents in the 512 grid
    directions, 32 of them against the oracle."""
    flush("excitation and far field L5 k=10, bench shape")
    k = 10.0
    v, f = icosphere(5)
    m = gmesh(v, f, dev)
    om = oracle_mesh(5)
    rhat, khat, pol, _, _ = synth.monostatic_grid(16, 32)
    rng = np.random.default_rng(31)
    s = np.sort(rng.choice(512, 16, replace=False))
    Vg = P.excite_planewave(m, k, khat, pol)[torch.as_tensor(s, device=dev)].cpu().numpy()
    Vo = oefie.excitation(om, k, khat[s], pol[s])
    assert rel_max(Vg, Vo) <= 1e-12
    J = rng.standard_normal((4, m.n)) + 1j * rng.standard_normal((4, m.n))
    d = np.sort(rng.choice(512, 32, replace=False))
    Fg = P.farfield(m, k, torch.as_tensor(J, device=dev), rhat).cpu().numpy()[:, d]
    Fo = oefie.farfield(om, k, J, rhat[d])
    assert rel_max(Fg, Fo) <= 1e-12


def test_farfield_l2(dev):
    v, f = icosphere(2)
    m = gmesh(v, f, dev)
    om = oracle_mesh(2)
    rng = np.random.default_rng(3)
    J = rng.standard_normal((3, m.n)) + 1j * rng.standard_normal((3, m.n))
    dirs = synth.uniform_directions(17, seed=4)
    dirs = np.concatenate([dirs, [[0, 0, 1.0], [0, 0, -1.0]]])       # poles
    Fg = P.farfield(m, 1.5, torch.as_tensor(J, device=dev), dirs).cpu().numpy()
    Fo = oefie.farfield(om, 1.5, J, dirs)
    assert rel_max(Fg, Fo) <= 1e-12


# ------------------------------------------------------------- products
@pytest.mark.parametrize("n,nrhs", [(481, 1), (481, 3), (480, 64), (257, 130), (9, 2), (481, 12), (257, 40)])
@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_zx_random(dev, n, nrhs, dt):
    rng = np.random.default_rng(n + nrhs)
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    X = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    tdt = torch.complex128 if dt == "c128" else torch.complex64
    Zt = torch.as_tensor(Z, dtype=tdt, device=dev)
    Xt = torch.as_tensor(X, dtype=tdt, device=dev)
    Y = P.zx(Zt, Xt).cpu().numpy().astype(np.complex128)
    # reference from the values actually stored (rounded to the storage type)
    Zr = Zt.cpu().numpy().astype(np.complex128)
    Xr = Xt.cpu().numpy().astype(np.complex128)
    ref = Xr @ Zr.T
    err = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    tol = 1e-14 if dt == "c128" else (1e-7 if nrhs == 1 else 2e-6)   # GEMV accumulates in FP64
    assert err <= tol, err


@pytest.mark.parametrize("n,nrhs", [(257, 40), (480, 64), (33, 3)])
def test_gemm_every_variant(dev, n, nrhs):
    """Every matrix-core GEMM variant (both kernel forms, every tile shape) on both
    paths: complex64 output with FP32 accumulation (efie_zx) and complex128 output
    with FP64 flushes per K chunk (efie_zx_flush64, the mixed solves' product),
    against the FP64 product of the values actually stored; ragged in rows,
    unknowns and K for every tile."""
    flush(f"gemm variants n={n} nrhs={nrhs}")
    rng = np.random.default_rng(7 * n + nrhs)
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    X = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    Zt = torch.as_tensor(Z, dtype=torch.complex64, device=dev)
    X64 = torch.as_tensor(X, dtype=torch.complex128, device=dev)
    X32 = X64.to(torch.complex64)
    ref = X32.cpu().numpy().astype(np.complex128) @ Zt.cpu().numpy().astype(np.complex128).T
    nref = np.linalg.norm(ref)
    prev32, prev64 = P.gemm_select(False, 0), P.gemm_select(True, 0)
    try:
        for v, t in enumerate(P.gemm_variants()):
            P.gemm_select(False, v)
            P.gemm_select(True, v)
            e32 = np.linalg.norm(P.zx(Zt, X32).cpu().numpy().astype(np.complex128) - ref) / nref
            e64 = np.linalg.norm(P.zx_flush64(Zt, X64).cpu().numpy() - ref) / nref
            flush(f"  variant {v} {t}: fp32-acc {e32:.2e}, fp64-flush {e64:.2e}")
            assert e32 <= 2e-6, (v, t, e32)
            assert e64 <= 5e-7, (v, t, e64)
    finally:
        P.gemm_select(False, prev32)
        P.gemm_select(True, prev64)


def test_gemm_l5_bench_shape_sampled(dev, tmp_path):
    """The headline product at its full shape and launch configuration: the level-5
    Z at k = 10 (complex64, N = 30720) times the 512 plane-wave excitations of the
    monostatic grid, on the tile the autotuner selects, FP64-flush path -- 8 sampled
    right-hand sides against 64 sampled unknowns, and a ragged 40-column launch,
    against the FP64 product of the values actually stored; and the single-column
    product (GEMV) on the same sampled unknowns."""
    flush("GEMM at the bench shape: L5 Z (complex64) x 512 plane waves")
    k = 10.0
    v, f = icosphere(5)
    m = P.Mesh(v, f).upload(dev)
    Z = P.assemble(m, k, dtype=P.C64)
    _, khat, pol, _, _ = synth.monostatic_grid(16, 32)
    V = P.excite_planewave(m, k, khat, pol)
    prev32, prev64 = P.gemm_select(False, 0), P.gemm_select(True, 0)
    try:
        tune = P.gemm_autotune(Z, 512, cache=str(tmp_path / "tiles.txt"))
        P.gemm_select(False, tune["acc32"])
        P.gemm_select(True, tune["acc64"])
        flush(f"  selected tile {tune['tiles'][tune['acc64']]}")
        rng = np.random.default_rng(5)
        cols = np.sort(rng.choice(m.n, 64, replace=False))
        Zc = Z[torch.as_tensor(cols, device=dev)].cpu().numpy().astype(np.complex128)   # rows = columns (Z = Z^T)
        for nrhs in (512, 40):
            X = V[:nrhs].contiguous()
            Y = P.zx_flush64(Z, X)
            rows = np.sort(rng.choice(nrhs, 8, replace=False))
            Xr = X[torch.as_tensor(rows, device=dev)].to(torch.complex64).cpu().numpy().astype(np.complex128)
            ref = Xr @ Zc.T
            got = Y[torch.as_tensor(rows, device=dev)][:, torch.as_tensor(cols, device=dev)].cpu().numpy()
            err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            flush(f"  {nrhs} columns: sampled relative error {err:.2e}")
            assert err <= 5e-7, (nrhs, err)
        # one right-hand side: the HBM-bound GEMV (complex64 Z and x, FP64 sums)
        x = V[:1].to(torch.complex64)
        y = P.zx(Z, x)[0, torch.as_tensor(cols, device=dev)].cpu().numpy().astype(np.complex128)
        ref1 = Zc @ x[0].cpu().numpy().astype(np.complex128)
        err1 = np.linalg.norm(y - ref1) / np.linalg.norm(ref1)
        flush(f"  1 column (GEMV): sampled relative error {err1:.2e}")
        assert err1 <= 1e-7, err1
    finally:
        P.gemm_select(False, prev32)
        P.gemm_select(True, prev64)


@pytest.mark.parametrize("n", [480, 481])
def test_zx_c64_unaligned_operands(dev, n):
    """Matrix-core product with X and Z starting 8 bytes past a 16-byte boundary
    (views into larger buffers): the 16-byte load path must not be taken."""
    rng = np.random.default_rng(n)
    nrhs = 40
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    X = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    zb = torch.zeros(n * n + 1, dtype=torch.complex64, device=dev)
    xb = torch.zeros(nrhs * n + 1, dtype=torch.complex64, device=dev)
    zb[1:] = torch.as_tensor(Z.reshape(-1), dtype=torch.complex64, device=dev)
    xb[1:] = torch.as_tensor(X.reshape(-1), dtype=torch.complex64, device=dev)
    Zt, Xt = zb[1:].view(n, n), xb[1:].view(nrhs, n)
    assert Zt.data_ptr() % 16 == 8 and Xt.data_ptr() % 16 == 8
    Y = P.zx(Zt, Xt).cpu().numpy().astype(np.complex128)
    ref = Xt.cpu().numpy().astype(np.complex128) @ Zt.cpu().numpy().astype(np.complex128).T
    assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) <= 2e-6


# ---------------------------------------------------------------- solves
@pytest.fixture(scope="module")
def l2_system(dev):
    v, f = icosphere(2)
    m = gmesh(v, f, dev)
    om = oracle_mesh(2)
    k = 1.0
    Zo = oefie.assemble(om, k)
    kh, pol = synth.planewave_x_along_minus_z()
    Vo = oefie.excitation(om, k, kh, pol)
    Jo = np.linalg.solve(Zo, Vo[0])
    return m, k, Zo, Vo, Jo


@pytest.mark.parametrize("solver", ["cocg", "cgs"])
def test_solve_l2_vs_lu(dev, l2_system, solver):
    m, k, Zo, Vo, Jo = l2_system
    Zg = P.assemble(m, k)
    Vg = P.excite_planewave(m, k, *synth.planewave_x_along_minus_z())
    code = P.COCG if solver == "cocg" else P.CGS
    J, st = P.solve(Zg, Vg, solver=code, tol=1e-8, maxit=2000)
    assert st.code == 0 and st.status[0] == 0
    assert st.relres_true[0] <= 2e-8
    Jg = J.cpu().numpy()[0]
    assert np.linalg.norm(Jg - Jo) <= 1e-5 * np.linalg.norm(Jo)
    # iteration count against the oracle's own Krylov on the oracle operator
    ref = (okrylov.cocg if solver == "cocg" else okrylov.cgs)(lambda x: Zo @ x, Vo[0], 1e-8, 2000)
    assert abs(int(st.iters[0]) - ref[1]) <= 2


def test_solve_multi_rhs_equals_single(dev, l2_system):
    m, k, Zo, Vo, Jo = l2_system
    Zg = P.assemble(m, k)
    rhat, khat, pol, _, _ = synth.monostatic_grid(1, 5)
    V = P.excite_planewave(m, k, khat, pol)
    J, st = P.solve(Zg, V, tol=1e-10, maxit=2000)
    assert np.all(st.status == 0)
    Vo5 = oefie.excitation(oracle_mesh(2), k, khat, pol)
    Jlu = np.linalg.solve(Zo, Vo5.T).T
    for s in range(5):
        J1, st1 = P.solve(Zg, V[s:s + 1].contiguous(), tol=1e-10, maxit=2000)
        assert int(st1.iters[0]) == int(st.iters[s])
        # GEMM (several columns) and GEMV (one column) sum in different orders
        assert np.abs(J1.cpu().numpy()[0] - J.cpu().numpy()[s]).max() <= 1e-10 * np.abs(Jlu[s]).max()
        assert np.linalg.norm(J.cpu().numpy()[s] - Jlu[s]) <= 1e-7 * np.linalg.norm(Jlu[s])


@pytest.mark.parametrize("nrhs", [1, 4])
def test_solve_mixed_l2(dev, l2_system, nrhs):
    m, k, Zo, Vo, Jo = l2_system
    Z32 = P.assemble(m, k, dtype=P.C64)
    rhat, khat, pol, _, _ = synth.monostatic_grid(1, nrhs)
    V = P.excite_planewave(m, k, khat, pol)
    J, st = P.solve(Z32, V, tol=1e-8, maxit=2000, max_refine=6, inner_tol=1e-3)
    assert np.all(st.status == 0), st
    assert np.all(st.relres_true <= 1e-8)
    Vo_ = oefie.excitation(oracle_mesh(2), k, khat, pol)
    Jlu = np.linalg.solve(Zo, Vo_.T).T
    err = np.linalg.norm(J.cpu().numpy() - Jlu) / np.linalg.norm(Jlu)
    # RCS on the E- and H-plane cuts against the oracle's, over the directions
    # within 30 dB of the pattern's peak
    ts = np.linspace(0, math.pi, 181)
    d = np.concatenate([np.stack([np.sin(ts) * math.cos(ph), np.sin(ts) * math.sin(ph), -np.cos(ts)], 1)
                        for ph in (0.0, math.pi / 2)])
    s_g = oefie.rcs(P.farfield(m, k, J, d).cpu().numpy())
    s_o = oefie.rcs(oefie.farfield(oracle_mesh(2), k, Jlu, d))
    keep = 10 * np.log10(s_o / s_o.max(axis=1, keepdims=True)) >= -30.0
    db = float(np.abs(10 * np.log10(s_g / s_o))[keep].max())
    flush(f"  mixed L2 current error vs FP64 LU: {err:.3e}, RCS {db:.2e} dB")
    assert err <= 1e-5 and db <= 0.01


def test_solve_tiny_odd_order(dev):
    v, f = bipyramid()
    m = gmesh(v, f, dev)
    om = rwg.build(v, f)
    Zo = oefie.assemble(om, 1.3)
    Vo = oefie.excitation(om, 1.3, *synth.planewave_x_along_minus_z())
    for dt in (P.C128, P.C64):
        Z = P.assemble(m, 1.3, dtype=dt)
        V = P.excite_planewave(m, 1.3, *synth.planewave_x_along_minus_z())
        J, st = P.solve(Z, V, tol=1e-10, maxit=200, max_refine=8)
        assert st.status[0] == 0
        Jlu = np.linalg.solve(Zo, Vo[0])
        tol = 1e-8 if dt == P.C128 else 1e-4
        assert np.linalg.norm(J.cpu().numpy()[0] - Jlu) <= tol * np.linalg.norm(Jlu)


def test_solve_zero_rhs_and_maxit(dev, l2_system):
    m, k, Zo, Vo, Jo = l2_system
    Zg = P.assemble(m, k)
    V = torch.zeros((2, m.n), dtype=torch.complex128, device=dev)
    V[1] = P.excite_planewave(m, k, *synth.planewave_x_along_minus_z())[0]
    J, st = P.solve(Zg, V, tol=1e-8, maxit=3)
    assert st.status[0] == 0 and st.iters[0] == 0 and float(J[0].abs().max()) == 0.0
    assert st.status[1] == 1 and st.code == 1 and st.iters[1] == 3


# ------------------------------------------------ end to end vs oracle and Mie
def test_end_to_end_l2_rcs(dev, l2_system):
    from oracle import mie

    m, k, Zo, Vo, Jo = l2_system
    Z = P.assemble(m, k)
    V = P.excite_planewave(m, k, *synth.planewave_x_along_minus_z())
    J, st = P.solve(Z, V, tol=1e-10, maxit=2000)
    ts = np.linspace(0, math.pi, 181)
    for phi in (0.0, math.pi / 2):
        d = np.stack([np.sin(ts) * math.cos(phi), np.sin(ts) * math.sin(phi), -np.cos(ts)], 1)
        F = P.farfield(m, k, J, d).cpu().numpy()
        Fo = oefie.farfield(oracle_mesh(2), k, Jo[None], d)
        s_g = oefie.rcs(F)[0]
        s_o = oefie.rcs(Fo)[0]
        assert np.max(np.abs(10 * np.log10(s_g / s_o))) <= 1e-6
        s_m = mie.bistatic_rcs(1.0, 1.0, ts, phi)
        assert np.max(np.abs(10 * np.log10(s_g / s_m))) <= 0.5     # L2 discretisation vs Mie


@pytest.mark.parametrize("fp32_acc", [False, True])
@pytest.mark.parametrize("solver", ["cocg", "cgs"])
def test_solve_mixed_many_rhs_matrix_cores(dev, solver, fp32_acc):
    """16 right-hand sides: the mixed-precision solve runs its products on the FP32
    matrix cores (more than 8 active columns; FP64 flushes per K chunk, or FP32
    accumulation) and must still reach the FP64-accumulated true residual, with currents
    close to the FP64 solution."""
    flush(f"mixed 16-rhs {solver} fp32_acc={fp32_acc}")
    v, f = icosphere(3)
    m = gmesh(v, f, dev)
    k = 2.0
    rhat, khat, pol, _, _ = synth.monostatic_grid(4, 4)
    Z32 = P.assemble(m, k, dtype=P.C64)
    Z64 = P.assemble(m, k)
    V = P.excite_planewave(m, k, khat, pol)
    code = P.COCG if solver == "cocg" else P.CGS
    J32, st32 = P.solve(Z32, V, solver=code, tol=1e-7, maxit=2000, max_refine=8, inner_tol=1e-2, fp32_acc=fp32_acc)
    J64, st64 = P.solve(Z64, V, solver=code, tol=1e-10, maxit=2000)
    assert np.all(st32.status == 0) and np.all(st32.relres_true <= 1e-7), st32
    err = float((J32 - J64).norm() / J64.norm())
    flush(f"  mixed vs FP64 current error {err:.3e}, iters {st32.iters.max()} vs {st64.iters.max()}")
    assert err <= 1e-5
