"""GPU parity of the distance-adaptive far rule (3x3 product of the interior
3-point rule on pairs with D >= ratio * h) against the oracle's adaptive
assembly, through the C ABI; tolerances as for the 7x7 rule (FP64 entries
1e-11 of max |Z|, complex64 2e-5)."""
import numpy as np
import pytest

import synth
from oracle import calderon as ocal
from oracle import efie as oefie

from .gpu_common import flush, icosphere, oracle_mesh, rel_max

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2310_15644_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()
    return torch.device("cuda:0")


def far_mesh(level, ratio, dev):
    v, f = icosphere(level)
    return P.Mesh(v, f).set_far_rule(ratio).upload(dev)


@pytest.mark.parametrize("k", [1.0, 3.0, ocal.ktilde(3.0)])
def test_far_rule_l2_c128_every_path(dev, k):
    flush(f"far rule L2 c128 k={k}")
    m = far_mesh(2, 3.0, dev)
    Zo = oefie.assemble(oracle_mesh(2), k, far3=3.0)
    Z7 = oefie.assemble(oracle_mesh(2), k)
    assert rel_max(Zo, Z7) > 1e-8                       # the rule changed the operator
    Zw = P.assemble(m, k).cpu().numpy()                 # tile (workspace) path
    Za = P.assemble(m, k, atomic=True).cpu().numpy()    # atomic path
    assert rel_max(Zw, Zo) <= 1e-11 and rel_max(Za, Zo) <= 1e-11
    assert np.abs(Zw - Zw.T).max() <= 1e-14 * np.abs(Zw).max()
    TA, TP = P.assemble(m, k, parts=True)
    _, TAo, TPo = oefie.assemble(oracle_mesh(2), k, parts=True, far3=3.0)
    assert rel_max(TA.cpu().numpy(), TAo) <= 1e-11 and rel_max(TP.cpu().numpy(), TPo) <= 1e-11


def test_far_rule_l2_c64(dev):
    flush("far rule L2 c64")
    m = far_mesh(2, 3.0, dev)
    Zg = P.assemble(m, 1.0, dtype=P.C64).cpu().numpy().astype(np.complex128)
    Zo = oefie.assemble(oracle_mesh(2), 1.0, far3=3.0)
    err = rel_max(Zg, Zo)
    flush(f"  c64 max rel err {err:.3e}")
    assert err <= 2e-5


def test_far_rule_off_again_is_seven_point(dev):
    v, f = icosphere(2)
    m = P.Mesh(v, f).upload(dev)
    Z0 = P.assemble(m, 2.0).cpu().numpy()
    m.set_far_rule(3.0)
    Z3 = P.assemble(m, 2.0).cpu().numpy()
    m.set_far_rule(0.0)
    Z1 = P.assemble(m, 2.0).cpu().numpy()
    assert np.array_equal(Z0, Z1) and not np.array_equal(Z0, Z3)


def test_far_rule_l4_sampled_rows(dev):
    flush("far rule L4 sampled rows")
    m = far_mesh(4, 4.0, dev)
    Zg = P.assemble(m, 5.0)
    rows = [0, 3001, 7679]
    got = Zg[rows].cpu().numpy()
    ref = oefie.z_rows(oracle_mesh(4), 5.0, rows, far3=4.0)
    for r in range(len(rows)):
        assert rel_max(got[r], ref[r]) <= 1e-11
    blk = Zg[:512, :512].cpu().numpy()
    assert np.abs(blk - blk.T).max() <= 1e-14 * np.abs(blk).max()


def test_far_rule_l5_sampled_entries_c64(dev):
    """Full size (level 5, N = 30720, k = 10), complex64 tile assembly as the
    bench runs it: sampled entries against the oracle's, one by one."""
    flush("far rule L5 c64 sampled entries")
    m = far_mesh(5, 4.0, dev)
    Zg = P.assemble(m, 10.0, dtype=P.C64)
    zmax = float(Zg.abs().max())
    rng = np.random.default_rng(11)
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, m.n, size=(12, 2))] + [(5, 5), (100, 101)]
    ref = oefie.z_entries(oracle_mesh(5), 10.0, pairs, far3=4.0)
    got = np.array([complex(Zg[a, b]) for a, b in pairs])
    err = np.abs(got - ref).max() / zmax
    flush(f"  max err / max|Z| {err:.3e}")
    assert err <= 2e-5
    del Zg


def test_far_rule_calderon_l1(dev):
    """The barycentric operator of T_BC follows the primal mesh's far rule."""
    flush("far rule calderon L1")
    k = 1.0
    kt = P.ktilde(k)
    m = far_mesh(1, 2.5, dev)
    cal = P.Calderon(m).upload(dev)
    Pm, Tbc = cal.assemble(kt, with_tbc=True)
    C = ocal.Calderon(oracle_mesh(1), k, ocal.ktilde(k), far3=2.5)
    C7 = ocal.Calderon(oracle_mesh(1), k, ocal.ktilde(k))
    assert rel_max(C.Tbc, C7.Tbc) > 1e-8
    assert rel_max(Tbc.cpu().numpy(), C.Tbc) <= 1e-11
    assert rel_max(Pm.cpu().numpy(), C.P) <= 1e-10


def test_calderon_own_far_rule_l1(dev):
    """A rule for the barycentric operator alone: T_BC and P follow it, Z does not."""
    flush("calderon own far rule L1")
    k = 1.0
    kt = P.ktilde(k)
    v, f = icosphere(1)
    m = P.Mesh(v, f).upload(dev)
    cal = P.Calderon(m).upload(dev).set_far_rule(2.5)
    Pm, Tbc = cal.assemble(kt, with_tbc=True)
    C = ocal.Calderon(oracle_mesh(1), k, ocal.ktilde(k), far3=None, far3_bary=2.5)
    assert rel_max(Tbc.cpu().numpy(), C.Tbc) <= 1e-11
    assert rel_max(Pm.cpu().numpy(), C.P) <= 1e-10
    assert rel_max(P.assemble(m, k).cpu().numpy(), oefie.assemble(oracle_mesh(1), k)) <= 1e-11
    # back to following the primal mesh (7x7 here)
    cal.set_far_rule(-1.0)
    _, Tbc7 = cal.assemble(kt, with_tbc=True)
    assert rel_max(Tbc7.cpu().numpy(), ocal.Calderon(oracle_mesh(1), k, ocal.ktilde(k)).Tbc) <= 1e-11
    with pytest.raises(P.EfieError):
        cal.set_far_rule(float("nan"))


def test_far_rule_rejected_by_gradient_followed_by_batch(dev):
    """The vertex gradient keeps the 7x7 rule and rejects a mesh with the far rule
    on; the batched assembly runs the single-mesh tile kernels and follows it."""
    m = far_mesh(2, 3.0, dev)
    n = m.n
    J = torch.zeros(n, dtype=torch.complex128, device=dev)
    W = torch.zeros(2, dtype=torch.complex128, device=dev)
    kh, pol = synth.planewave_x_along_minus_z()
    with pytest.raises(P.EfieError) as ei:
        P.vertex_grad(m, 1.0, J, J, W, np.array([[0.0, 0.0, 1.0]]), kh, pol)
    assert ei.value.code == -1
    for code in (P.C64, P.C128):
        Zb = P.Batch([m]).assemble([2.0], dtype=code)
        assert torch.equal(Zb.view(n, n), P.assemble(m, 2.0, dtype=code))
