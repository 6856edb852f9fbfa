"""Many uneven meshes in one persistent tile launch and one grouped solve: every
block is bit-identical to its single-mesh assembly (the same tile device code on
a view of each mesh's concatenated tables, no atomics), two batched assemblies
are bit-identical, the grouped solve of a mesh is bit-identical to the same mesh
solved alone by the grouped solver (equal step counts) and matches the general
single-mesh solver (the solutions to 1e-8, the step counts within 6 %), one mesh
against the oracle; the
64-ellipsoid set (semi-axes U[0.5, 1.5], 1k-8k unknowns) at k = 2."""
import time

import numpy as np
import pytest

import synth
from oracle import efie as oefie
from oracle import rwg

from .gpu_common import flush, icosphere, rel_max

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2310_15644_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def small_set():
    shapes = [synth.ellipsoid(3, (1.2, 0.8, 0.6)), synth.ellipsoid(5, (0.7, 1.1, 1.3)), icosphere(2),
              synth.ellipsoid(2, (1.0, 1.0, 0.5)), synth.ellipsoid(4, (0.9, 0.6, 1.4))]
    return shapes


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_batch_assembly_equals_single(dev, dt):
    flush(f"batch assembly small set {dt}")
    shapes = small_set()
    meshes = [P.Mesh(v, f).upload(dev) for v, f in shapes]
    B = P.Batch(meshes)
    ks = [1.0, 2.0, 1.5, 0.7, 2.5]
    code = P.C128 if dt == "c128" else P.C64
    Zc = B.assemble(ks, dtype=code)
    Zc2 = B.assemble(ks, dtype=code)
    assert torch.equal(Zc, Zc2)                      # deterministic
    for i, m in enumerate(meshes):
        Zs = P.assemble(m, ks[i], dtype=code)
        assert torch.equal(B.z_of(Zc, i), Zs), i     # bit-identical to the single-mesh assembly
    om = rwg.build(*shapes[0])
    Zo = oefie.assemble(om, ks[0])
    tol = 1e-11 if dt == "c128" else 2e-5
    assert rel_max(B.z_of(Zc, 0).cpu().numpy().astype(np.complex128), Zo) <= tol


def test_batch_solve_equals_single(dev):
    shapes = small_set()
    meshes = [P.Mesh(v, f).upload(dev) for v, f in shapes]
    B = P.Batch(meshes)
    k = 1.3
    Zc = B.assemble(k, dtype=P.C128)
    kh, pol = synth.planewave_x_along_minus_z()
    Vc = torch.cat([P.excite_planewave(m, k, kh, pol)[0] for m in meshes])
    J6, st6 = B.solve(Zc, Vc, tol=1e-6, maxit=1000)
    J, st = B.solve(Zc, Vc, tol=1e-10, maxit=1000)
    assert np.all(st.status == 0) and np.all(st.relres_true <= 2e-10)
    for i, m in enumerate(meshes):
        Zi, Vi = B.z_of(Zc, i).contiguous(), Vc[B.voff[i]:B.voff[i + 1]].contiguous()
        _, s6 = P.solve(Zi, Vi, tol=1e-6, maxit=1000)
        J1, st1 = P.solve(Zi, Vi, tol=1e-10, maxit=1000)
        # the matrices are bit-identical, but the two solvers round differently: the
        # grouped GEMV and the single one (column slabs) sum in different orders, and
        # the single COCG replaces its recursive residual by the true one.  COCG's
        # step counts answer to rounding like a chaotic system (the recurrences agree
        # only in exact arithmetic), so they are compared within 6 % (at least 3
        # steps), and the solutions themselves tightly below
        assert abs(int(s6.iters[0]) - int(st6.iters[i])) <= max(3, int(0.06 * s6.iters[0]))
        assert abs(int(st1.iters[0]) - int(st.iters[i])) <= max(3, int(0.06 * st1.iters[0]))
        a = J[B.voff[i]:B.voff[i + 1]].cpu().numpy()
        b = J1.cpu().numpy()[0]
        assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)
        # the same mesh alone in a batch: the grouped solver's arithmetic for a mesh
        # (its rows' products, its block's reductions) does not depend on the other
        # meshes of the group, so solution and step counts are exactly those
        B1 = P.Batch([m])
        Z1 = B1.assemble(k, dtype=P.C128)
        assert torch.equal(Z1, B.z_of(Zc, i).reshape(-1))
        J1b, st1b = B1.solve(Z1, Vi, tol=1e-10, maxit=1000)
        assert int(st1b.iters[0]) == int(st.iters[i])
        assert torch.equal(J1b, J[B.voff[i]:B.voff[i + 1]])


def test_batch_64_ellipsoids(dev):
    """The 64-ellipsoid workload: one persistent launch, grouped mixed-storage solve."""
    flush("64 ellipsoids")
    batch = synth.ellipsoid_batch(64, seed=0)
    meshes = [P.Mesh(v, f).upload(dev) for v, f, _, _ in batch]
    ns = np.array([m.n for m in meshes])
    flush(f"  N range {ns.min()}..{ns.max()}, sum N^2 = {int((ns ** 2).sum())}")
    B = P.Batch(meshes)
    k = 2.0
    Zc = B.assemble(k, dtype=P.C64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Zc = B.assemble(k, dtype=P.C64, out=Zc)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    for m in meshes[:8]:
        P.assemble(m, k, dtype=P.C64)
    torch.cuda.synchronize()
    t8 = time.perf_counter() - t0
    flush(f"  batch assembly {tb * 1e3:.1f} ms ({(ns ** 2).sum() / tb / 1e6:.0f} Mentries/s); "
          f"8 single launches {t8 * 1e3:.1f} ms")
    for i in (0, 37, 63):
        Zs = P.assemble(meshes[i], k, dtype=P.C64)
        assert torch.equal(B.z_of(Zc, i), Zs)
    # one sampled row of one ellipsoid against the oracle
    v, f, _, _ = batch[5]
    om = rwg.build(v, f)
    row = om.n // 3
    ref = oefie.z_rows(om, k, [row])[0]
    got = B.z_of(Zc, 5)[row].cpu().numpy().astype(np.complex128)
    assert rel_max(got, ref) <= 2e-5
    kh, pol = synth.planewave_x_along_minus_z()
    Vc = torch.cat([P.excite_planewave(m, k, kh, pol)[0] for m in meshes])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, st = B.solve(Zc, Vc, tol=1e-6, maxit=3000)
    torch.cuda.synchronize()
    flush(f"  batch solve {time.perf_counter() - t0:.2f} s, iterations {st.iters.min()}..{st.iters.max()}")
    assert np.all(st.status == 0) and np.all(st.relres_true <= 1.01e-6)
