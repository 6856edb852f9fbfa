"""GPU parity of the adjoint vertex gradient: the far-field adjoint source, each of
the three gradient terms against the oracle's autograd terms, the full objective
gradient through the torch autograd function, and -- on the level-4 perturbed
sphere (k = 3, 32 seeded directions) -- central finite differences, translation
invariance and the scaling identity sum_v x_v . g_v = 2 J + k dJ/dk."""
import functools

import numpy as np
import pytest

import synth
from oracle import gradient as ograd
from oracle import rwg

from .gpu_common import flush

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2310_15644_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@functools.lru_cache(maxsize=None)
def _oracle(level, k):
    v, f = synth.perturbed_sphere(level, seed=0)
    m = rwg.build(v, f)
    kh, pol = synth.planewave_x_along_minus_z()
    dirs = synth.uniform_directions(32, seed=1)
    prob = ograd.Problem(m, k, kh[0], pol[0], dirs)
    j, F, W, lam = ograd.adjoint_vectors(prob, v)
    terms = ograd.term_gradients(prob, v, j, lam, W)
    J, g = ograd.objective_and_gradient(prob, v)
    return v, f, prob, j, F, W, lam, terms, J, g


def _c(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.complex128), device=dev)


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("level,k", [(1, 1.5), (2, 3.0)])
def test_farfield_adjoint(dev, level, k):
    flush(f"farfield adjoint L{level} k={k}")
    v, f, prob, j, F, W, lam, terms, J, g = _oracle(level, k)
    m = P.Mesh(v, f).upload(dev)
    rng = np.random.default_rng(3)
    Wr = rng.standard_normal((2, len(prob.dirs), 2)) + 1j * rng.standard_normal((2, len(prob.dirs), 2))
    G = P.farfield_adjoint(m, k, _c(Wr, dev), prob.dirs).cpu().numpy()
    with torch.no_grad():
        Rm = prob.parts(torch.as_tensor(v))[2].numpy()
    ref = Wr.reshape(2, -1) @ Rm
    assert _rel(G, ref) <= 1e-12


@pytest.mark.parametrize("level,k", [(1, 1.5), (2, 3.0)])
def test_vertex_grad_terms(dev, level, k):
    """Radiation (lambda = 0), excitation (j = 0) and operator terms separately."""
    flush(f"vertex grad terms L{level} k={k}")
    v, f, prob, j, F, W, lam, (rad, exc, op), J, g = _oracle(level, k)
    m = P.Mesh(v, f).upload(dev)
    zero = np.zeros_like(j)
    args = (prob.dirs, prob.khat, prob.pol)
    jd, ld, Wd, zd = _c(j, dev), _c(lam, dev), _c(W, dev), _c(zero, dev)
    g_rad = P.vertex_grad(m, k, jd, zd, Wd, *args).cpu().numpy()
    g_exc = P.vertex_grad(m, k, zd, ld, Wd, *args).cpu().numpy()
    g_all = P.vertex_grad(m, k, jd, ld, Wd, *args).cpu().numpy()
    g_op = g_all - g_rad - g_exc
    e = (_rel(g_rad, rad), _rel(g_exc, exc), _rel(g_op, op), _rel(g_all, g))
    flush(f"  rel errors rad {e[0]:.2e} exc {e[1]:.2e} op {e[2]:.2e} total {e[3]:.2e}")
    assert max(e) <= 1e-10


@pytest.mark.parametrize("shape", [(1, 32, 2), (3, 700, 2)])
def test_farfield_objective(dev, shape):
    """J = sum |F|^2 and W = conj(F) from the library against their definitions on
    the same seeded F (a count below and above the block's 256 threads); the sum is
    the same on a second call."""
    rng = np.random.default_rng(7)
    Fh = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    F = torch.tensor(Fh, dtype=torch.complex128, device=dev)
    J1, W = P.farfield_objective(F)
    J2, none = P.farfield_objective(F, with_weight=False)
    assert none is None
    ref = float(np.sum(Fh.real ** 2 + Fh.imag ** 2))
    assert abs(float(J1) - ref) <= 1e-14 * ref
    assert float(J1) == float(J2)
    assert torch.equal(W.cpu(), torch.tensor(np.conj(Fh), dtype=torch.complex128))


def test_objective_autograd_l2(dev):
    from paper_2310_15644_amd.objective import far_field_objective

    flush("FarFieldObjective L2 k=3")
    v, f, prob, j, F, W, lam, terms, J, g = _oracle(2, 3.0)
    x = torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True)
    Jg = far_field_objective(x, f, 3.0, prob.khat, prob.pol, prob.dirs, tol=1e-13)
    Jg.backward()
    flush(f"  J gpu {float(Jg):.15e} oracle {J:.15e}")
    assert abs(float(Jg) - J) <= 1e-10 * J
    assert _rel(x.grad.cpu().numpy(), g) <= 1e-8


# --------------------------------------------------------------- level 4
K4 = 3.0


@pytest.fixture(scope="module")
def l4(dev):
    from paper_2310_15644_amd.objective import far_field_objective

    v, f = synth.perturbed_sphere(4, seed=0)
    kh, pol = synth.planewave_x_along_minus_z()
    dirs = synth.uniform_directions(32, seed=1)

    def objective(xyz, k=K4, grad=False):
        if grad:
            x = torch.tensor(xyz, dtype=torch.float64, device=dev, requires_grad=True)
            J = far_field_objective(x, f, k, kh[0], pol[0], dirs, tol=1e-13)
            J.backward()
            return float(J), x.grad.cpu().numpy()
        # finite-difference values: library assembly, excitation and far field with
        # a dense LU solve, whose rounding is smooth in x (an iterative solve's
        # stopping point is not, and its error does not cancel between x +- h d)
        m = P.Mesh(xyz, f).upload(dev)
        Z = P.assemble(m, k)
        V = P.excite_planewave(m, k, kh, pol)
        j = torch.linalg.solve(Z, V[0])
        F = P.farfield(m, k, j.reshape(1, -1).contiguous(), dirs)
        return float((F.real ** 2 + F.imag ** 2).sum()), m.n_near

    flush("L4 objective and gradient")
    torch.cuda.synchronize()
    P.prof_enable(True)
    P.prof_reset()
    J, g = objective(v, grad=True)
    stats = P.prof_read(with_work=True)
    for name in ("grad_far", "grad_near", "grad_tri"):
        n, ms, work = stats[name]
        flush(f"  {name}: {n} launch(es) {ms:.3f} ms, {work:.0f} units")
    P.prof_enable(False)
    return v, f, objective, J, g


def _fd(objective, v, d, h, n0):
    """Central difference of J along d, or None when the near-pair classification
    differs at v +- h d (J jumps there)."""
    (Jp, np_), (Jm, nm) = objective(v + h * d), objective(v - h * d)
    if np_ != n0 or nm != n0:
        return None
    return (Jp - Jm) / (2 * h)


def test_l4_finite_differences(l4):
    """Central differences with h = 1e-6 along 8 seeded random unit directions.  The
    objective is smooth only while the near-pair classification is fixed; a
    direction whose +-h points classify a pair differently (a jump of J, seen as
    a change in the near-pair count) is replaced by the next seeded one."""
    v, f, objective, J, g = l4
    rng = np.random.default_rng(11)
    h = 1e-6
    gn = np.linalg.norm(g)
    n0 = objective(v)[1]
    done = tried = 0
    worst = 0.0
    while done < 8:
        tried += 1
        assert tried <= 16, "too many directions change the near-pair classification"
        d = rng.standard_normal(v.shape)
        d /= np.linalg.norm(d)
        fd = _fd(objective, v, d, h, n0)
        if fd is None:
            flush(f"  L4 direction {tried}: near-pair classification changes: skipped")
            continue
        ad = float(np.sum(g * d))
        worst = max(worst, abs(fd - ad) / gn)
        assert abs(fd - ad) <= 1e-6 * gn, (tried, fd, ad)
        done += 1
    flush(f"  L4: 8 directions, max |FD - adjoint| / |g| = {worst:.2e}")


def test_l4_single_coordinates(l4):
    """Central differences (h = 1e-6) of 32 seeded single vertex coordinates among
    the gradient components above 1e-3 of the largest: each within 1e-5 of the
    component (relative) plus the rounding floor of a central difference, 16 eps |J| / h
    (the FP64 evaluations of J, an LU solve included, each carry a few eps |J| of
    rounding that does not cancel between x + h e and x - h e: 2.3e-8 here against
    components down to 9e-4); coordinates whose +-h points change the near-pair
    classification are replaced by the next seeded ones."""
    v, f, objective, J, g = l4
    h = 1e-6
    floor = 16 * np.finfo(float).eps * abs(J) / h
    n0 = objective(v)[1]
    big = np.flatnonzero(np.abs(g).ravel() > 1e-3 * np.abs(g).max())
    rng = np.random.default_rng(12)
    order = rng.permutation(big)
    done = 0
    worst = 0.0
    for c in order:
        d = np.zeros(v.size)
        d[c] = 1.0
        fd = _fd(objective, v, d.reshape(v.shape), h, n0)
        if fd is None:
            continue
        gi = float(g.ravel()[c])
        rel = abs(fd - gi) / abs(gi)
        worst = max(worst, rel)
        assert abs(fd - gi) <= 1e-5 * abs(gi) + floor, (int(c), fd, gi, floor)
        done += 1
        if done == 32:
            break
    assert done == 32
    flush(f"  L4: 32 single coordinates (of {len(big)} above 1e-3 max), max relative error {worst:.2e}, "
          f"rounding floor {floor:.1e}")


def test_l4_translation_and_scaling(l4):
    v, f, objective, J, g = l4
    assert np.abs(g.sum(axis=0)).max() <= 1e-9 * np.abs(g).max() * len(v)
    h = 1e-6
    dJdk = (objective(v, K4 * (1 + h))[0] - objective(v, K4 * (1 - h))[0]) / (2 * h * K4)
    lhs = float(np.sum(v * g))
    flush(f"  L4 sum x.g {lhs:.12e}  2J + k dJ/dk {2 * J + K4 * dJdk:.12e}")
    assert abs(lhs - (2 * J + K4 * dJdk)) <= 1e-6 * abs(lhs)
