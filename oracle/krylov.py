"""Reference solves (oracle).

The paper names CG, PCG and CGS only as acronyms.  Readings taken:
  * LU with partial pivoting (numpy.linalg.solve) is the exact reference of Z j = V.
  * CGS: Sonneveld, SIAM J. Sci. Stat. Comput. 10(1), 1989 (also Saad, Iterative
    Methods for Sparse Linear Systems, 2nd ed., Alg. 7.6), conjugated inner product
    (a, b) = a^H b, shadow residual r~ = r0, x0 = 0.
  * "CG" for the complex-symmetric Z is COCG (van der Vorst and Melissen, IEEE
    Trans. Magn. 26(2), 1990): CG with the unconjugated bilinear form a^T b.
Both stop when ||r_k||_2 / ||b||_2 <= tol on the recurrence residual.
"""
from __future__ import annotations

import numpy as np


def lu_solve(A, b):
    return np.linalg.solve(A, b)


def cgs(matvec, b, tol=1e-8, maxit=1000):
    """Returns (x, iterations, converged, recurrence residual history)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0.0:
        return x, 0, True, hist
    rt = r.copy()
    rho = np.vdot(rt, r)
    u = r.copy()
    p = r.copy()
    for it in range(1, maxit + 1):
        v = matvec(p)
        sigma = np.vdot(rt, v)
        if sigma == 0 or rho == 0:
            return x, it - 1, False, hist
        alpha = rho / sigma
        q = u - alpha * v
        uq = u + q
        x = x + alpha * uq
        r = r - alpha * matvec(uq)
        res = np.linalg.norm(r) / nb
        hist.append(res)
        if res <= tol:
            return x, it, True, hist
        rho_new = np.vdot(rt, r)
        beta = rho_new / rho
        rho = rho_new
        u = r + beta * q
        p = u + beta * (q + beta * p)
    return x, maxit, False, hist


def cocg(matvec, b, tol=1e-8, maxit=1000):
    """COCG for complex-symmetric operators.  Returns (x, iterations, converged, history)."""
    b = np.asarray(b, dtype=np.complex128)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    hist = [1.0]
    if nb == 0.0:
        return x, 0, True, hist
    p = r.copy()
    rho = np.dot(r, r)
    for it in range(1, maxit + 1):
        q = matvec(p)
        mu = np.dot(p, q)
        if mu == 0 or rho == 0:
            return x, it - 1, False, hist
        alpha = rho / mu
        x = x + alpha * p
        r = r - alpha * q
        res = np.linalg.norm(r) / nb
        hist.append(res)
        if res <= tol:
            return x, it, True, hist
        rho_new = np.dot(r, r)
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p
    return x, maxit, False, hist
