"""Pins of the oracle vertex gradient (oracle.gradient).

The torch re-expression of Z, V and the far-field rows must equal the numpy
oracle; its autograd gradient must match central finite differences of the
objective, vanish in sum over the vertices (J is translation invariant: a shift
only multiplies F by a unit-modulus phase), and satisfy the scaling identity
sum_v x_v . dJ/dx_v = 2 J + k dJ/dk (under x -> s x, k -> k/s the current is
unchanged and F scales by s, so J(s x, k/s) = s^2 J(x, k))."""
import functools

import numpy as np
import pytest

import synth
from oracle import efie, gradient, rwg

K = 1.5


@functools.lru_cache(maxsize=None)
def _case(level=1, k=K):
    v, f = synth.perturbed_sphere(level, seed=0)
    m = rwg.build(v, f)
    kh, pol = synth.planewave_x_along_minus_z()
    dirs = synth.uniform_directions(32, seed=1)
    prob = gradient.Problem(m, k, kh[0], pol[0], dirs)
    J, g = gradient.objective_and_gradient(prob, v)
    return v, f, m, prob, J, g


def test_parts_match_numpy_oracle():
    import torch

    v, f, m, prob, J, g = _case()
    with torch.no_grad():
        Z, V, Rm = (t.numpy() for t in prob.parts(torch.as_tensor(v)))
    Zo = efie.assemble(m, K)
    kh, pol = synth.planewave_x_along_minus_z()
    Vo = efie.excitation(m, K, kh, pol)[0]
    assert np.abs(Z - Zo).max() / np.abs(Zo).max() < 1e-13
    assert np.abs(V - Vo).max() / np.abs(Vo).max() < 1e-13
    # far-field rows: F for two random currents
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, m.n)) + 1j * rng.standard_normal((2, m.n))
    Fo = efie.farfield(m, K, x, prob.dirs)                      # (2, ndir, 2)
    F = (Rm @ x.T).T.reshape(2, -1, 2)
    assert np.abs(F - Fo).max() / np.abs(Fo).max() < 1e-13
    jo = np.linalg.solve(Zo, Vo)
    Jo = float(np.sum(np.abs(efie.farfield(m, K, jo[None], prob.dirs)) ** 2))
    assert abs(J - Jo) / Jo < 1e-12


def test_gradient_matches_finite_differences():
    v, f, m, prob, J, g = _case()
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(3):
        d = rng.standard_normal(v.shape)
        d /= np.linalg.norm(d)
        fd = (gradient.objective_value(prob, v + h * d) - gradient.objective_value(prob, v - h * d)) / (2 * h)
        ad = float(np.sum(g * d))
        assert abs(fd - ad) <= 1e-6 * np.abs(g).max() * np.sqrt(g.size), (fd, ad)


def test_gradient_translation_invariance():
    v, f, m, prob, J, g = _case()
    assert np.abs(g.sum(axis=0)).max() < 1e-11 * np.abs(g).max() * len(v)
    assert np.abs(g).max() > 1e-3 * J          # not trivially zero


def test_gradient_scaling_identity():
    v, f, m, prob, J, g = _case()
    h = 1e-6
    kh, pol = synth.planewave_x_along_minus_z()
    Jp = gradient.objective_value(gradient.Problem(m, K * (1 + h), kh[0], pol[0], prob.dirs), v)
    Jm = gradient.objective_value(gradient.Problem(m, K * (1 - h), kh[0], pol[0], prob.dirs), v)
    dJdk = (Jp - Jm) / (2 * h * K)
    lhs = float(np.sum(v * g))
    assert abs(lhs - (2 * J + K * dJdk)) < 1e-7 * abs(lhs)


def test_terms_sum_to_total():
    v, f, m, prob, J, g = _case()
    j, F, W, lam = gradient.adjoint_vectors(prob, v)
    r, e, o = gradient.term_gradients(prob, v, j, lam, W)
    assert np.abs(r + e + o - g).max() < 1e-12 * np.abs(g).max()
    # each term is substantial on its own (none is identically zero)
    for t in (r, e, o):
        assert np.abs(t).max() > 1e-3 * np.abs(g).max()


@pytest.mark.parametrize("term", ["rad", "exc", "op"])
def test_terms_match_finite_differences(term):
    """Each term alone against central differences of its scalar with fixed vectors."""
    import torch

    v, f, m, prob, J, g = _case()
    j, F, W, lam = gradient.adjoint_vectors(prob, v)
    grads = dict(zip(("rad", "exc", "op"), gradient.term_gradients(prob, v, j, lam, W)))
    jt, lt, Wt = (torch.as_tensor(a) for a in (j, lam, W.reshape(-1)))

    def scalar(x):
        with torch.no_grad():
            Z, V, Rm = prob.parts(torch.as_tensor(x))
            if term == "rad":
                return 2.0 * float((Wt * (Rm @ jt)).sum().real)
            if term == "exc":
                return 2.0 * float((lt * V).sum().real)
            return -2.0 * float((lt * (Z @ jt)).sum().real)

    rng = np.random.default_rng(7)
    d = rng.standard_normal(v.shape)
    d /= np.linalg.norm(d)
    h = 1e-6
    fd = (scalar(v + h * d) - scalar(v - h * d)) / (2 * h)
    ad = float(np.sum(grads[term] * d))
    assert abs(fd - ad) <= 1e-6 * np.abs(grads[term]).max() * np.sqrt(v.size), (fd, ad)
