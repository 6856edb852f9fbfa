"""Vertex gradient of a far-field objective (oracle, torch CPU autograd).

Objective: J(x) = sum_d ||F(rhat_d)||^2 over a set of observation directions,
F the far-field pattern (theta and phi components) of the current that solves
Z(x) j = V(x), as functions of the vertex positions x.  The gradient is the
exact derivative of the discrete objective: the same RWG / 7-point / singular-
extraction definitions as `efie`, written again with torch operations on the
vertex coordinates, differentiated by reverse-mode autograd, with the linear
solve done by torch.linalg.solve (its adjoint is the transpose solve).  The
near-pair classification is frozen at the unperturbed mesh, as the objective's
definition requires for differentiability.  Meant for small meshes (the 7x7
pair tensors of the whole mesh are held for the backward pass).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import efie, quadrature

ETA0 = efie.ETA0
DT = torch.complex128


def _geometry(x, tri):
    P = x[tri]                                            # (T, 3, 3)
    e1, e2 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
    cr = torch.linalg.cross(e1, e2)
    dbl = torch.linalg.norm(cr, dim=1)
    area = 0.5 * dbl
    nrm = cr / dbl[:, None]
    # length of the edge opposite local vertex i
    L = torch.stack([torch.linalg.norm(P[:, 1] - P[:, 2], dim=1), torch.linalg.norm(P[:, 2] - P[:, 0], dim=1),
                     torch.linalg.norm(P[:, 0] - P[:, 1], dim=1)], dim=1)
    return P, area, nrm, L


def _potentials(r, v, nrm):
    """Closed-form I0, I1 (see oracle.singular) in torch: r (M, 7, 3), v (M, 3, 3), nrm (M, 3)."""
    n_ = nrm[:, None, :]
    d = ((r - v[:, None, 0, :]) * n_).sum(-1)
    rho = r - d[..., None] * n_
    ad = d.abs()
    I0 = torch.zeros_like(d)
    I1 = torch.zeros_like(r)
    for i in range(3):
        rm, rp = v[:, None, i, :], v[:, None, (i + 1) % 3, :]
        lt = (rp - rm) / torch.linalg.norm(rp - rm, dim=-1, keepdim=True)
        u = torch.linalg.cross(lt.expand_as(rho), n_.expand_as(rho))
        lp = ((rp - rho) * lt).sum(-1)
        lm = ((rm - rho) * lt).sum(-1)
        P0 = ((rm - rho) * u).sum(-1)
        R02 = P0 * P0 + d * d
        Rp = torch.linalg.norm(r - rp, dim=-1)
        Rm = torch.linalg.norm(r - rm, dim=-1)
        # (R + l) as R0^2 / (R - l) for l < 0; the points here never sit on an edge line
        fp = torch.where(lp >= 0, Rp + lp, R02 / torch.where(lp >= 0, torch.ones_like(Rp), Rp - lp))
        fm = torch.where(lm >= 0, Rm + lm, R02 / torch.where(lm >= 0, torch.ones_like(Rm), Rm - lm))
        lg = torch.log(fp / fm)
        at = torch.atan(P0 * lp / (R02 + ad * Rp)) - torch.atan(P0 * lm / (R02 + ad * Rm))
        I0 = I0 + P0 * lg - ad * at
        I1 = I1 + (0.5 * (R02 * lg + lp * Rp - lm * Rm))[..., None] * u
    return I0, I1


class Problem:
    """Topology (numpy, from oracle.rwg) plus the frozen near-pair list."""

    def __init__(self, mesh, k, khat, pol, dirs, near_factor=2.0, eta=ETA0):
        self.mesh = mesh
        self.k = float(k)
        self.eta = eta
        self.khat = np.asarray(khat, dtype=np.float64).reshape(3)
        self.pol = np.asarray(pol, dtype=np.float64).reshape(3)
        self.dirs = np.atleast_2d(dirs)
        near = efie.near_pairs(mesh, near_factor)
        self.near = torch.as_tensor(near)
        pq = np.argwhere(near)
        self.np_, self.nq_ = torch.as_tensor(pq[:, 0]), torch.as_tensor(pq[:, 1])
        bary, w = quadrature.radon7()
        self.bary = torch.as_tensor(bary)
        self.w = torch.as_tensor(w)
        self.tri = torch.as_tensor(mesh.tri)
        self.sign = torch.as_tensor(mesh.tri_sign, dtype=torch.float64)
        self.te = torch.as_tensor(mesh.tri_edge)

    # ------------------------------------------------------------------ pieces
    def parts(self, x):
        """Z, V and the radiation rows R (2D, N) as differentiable functions of x."""
        k, eta = self.k, self.eta
        P, area, nrm, L = _geometry(x, self.tri)
        qp = torch.einsum("ak,tkx->tax", self.bary, P)               # (T, 7, 3)
        W = self.w[None, :] * area[:, None]                            # (T, 7)
        coef = self.sign * L / (2.0 * area[:, None])                   # (T, 3)
        div = self.sign * L / area[:, None]
        f = coef[:, :, None, None] * (qp[:, None, :, :] - P[:, :, None, :])   # (T, 3i, 7a, 3)
        T, N = len(self.tri), self.mesh.n
        diff = qp[:, None, :, None, :] - qp[None, :, None, :, :]         # (T, T, 7, 7, 3)
        R2 = (diff * diff).sum(-1)
        zero = R2 == 0                                                  # coincident points (self pairs)
        near = self.near[:, :, None, None]
        Rsafe = torch.sqrt(torch.where(zero, torch.ones_like(R2), R2))   # sqrt never sees 0 (finite gradient)
        ph = -k * Rsafe
        # far kernel exp(-jkR)/(4 pi R); near: smooth (exp(-jkR)-1)/(4 pi R), -jk/(4 pi) at R = 0
        cosr, sinr = torch.cos(ph), torch.sin(ph)
        far_re, far_im = cosr / Rsafe, sinr / Rsafe
        sm_re = -2.0 * torch.sin(0.5 * ph) ** 2 / Rsafe
        sm_im = sinr / Rsafe
        sm_re = torch.where(zero, torch.zeros_like(sm_re), sm_re)
        sm_im = torch.where(zero, torch.full_like(sm_im, -k), sm_im)
        Gr = torch.where(near, sm_re, far_re) / (4 * math.pi)
        Gi = torch.where(near, sm_im, far_im) / (4 * math.pi)
        G = torch.complex(Gr, Gi)
        WW = W[:, None, :, None] * W[None, :, None, :]                  # (T, T, 7, 7)
        dot = torch.einsum("piax,qjbx->pqijab", f, f)                   # (T, T, 3, 3, 7, 7)
        TA = torch.einsum("pqab,pqijab->pqij", (WW * G), dot.to(DT))
        S = (WW * G).sum((-1, -2))
        TP = div[:, None, :, None] * div[None, :, None, :] * S[:, :, None, None]
        # singular part of the near pairs, symmetrised
        ps, qs = self.np_, self.nq_

        def sing(tp, tq):
            I0, I1 = _potentials(qp[tp], P[tq], nrm[tq])
            d = ((qp[tp] - P[tq][:, None, 0, :]) * nrm[tq][:, None, :]).sum(-1)
            rho = qp[tp] - d[..., None] * nrm[tq][:, None, :]
            inner = coef[tq][:, :, None, None] * (I1[:, None] + (rho[:, None] - P[tq][:, :, None, :]) * I0[:, None, :, None])
            fa = f[tp]
            A = torch.einsum("pa,piax,pjax->pij", W[tp], fa, inner) / (4 * math.pi)
            s0 = (W[tp] * I0).sum(-1) / (4 * math.pi)
            Pp = div[tp][:, :, None] * div[tq][:, None, :] * s0[:, None, None]
            return A, Pp

        A1, P1 = sing(ps, qs)
        A2, P2 = sing(qs, ps)
        TA = TA.index_put((ps, qs), TA[ps, qs] + (0.5 * (A1 + A2.transpose(1, 2))).to(DT))
        TP = TP.index_put((ps, qs), TP[ps, qs] + (0.5 * (P1 + P2.transpose(1, 2))).to(DT))
        Zb = eta * (1j * k * TA + TP / (1j * k))                         # (T, T, 3, 3)
        # scatter the triangle-pair blocks onto RWG pairs
        rows = self.te[:, None, :, None].expand(T, T, 3, 3).reshape(-1)
        cols = self.te[None, :, None, :].expand(T, T, 3, 3).reshape(-1)
        Z = torch.zeros(N * N, dtype=DT).index_add(0, rows * N + cols, Zb.reshape(-1)).reshape(N, N)
        # excitation
        phase = torch.exp(torch.complex(torch.zeros_like(qp[..., 0]), -k * (qp @ torch.as_tensor(self.khat))))
        fe = (f * torch.as_tensor(self.pol)).sum(-1)                     # (T, 3, 7)
        cv = (W[:, None, :] * fe * phase[:, None, :]).sum(-1)          # (T, 3)
        V = torch.zeros(N, dtype=DT).index_add(0, self.te.reshape(-1), cv.reshape(-1))
        # radiation rows: -(j k eta / 4 pi) e_c . a_n(rhat_d)
        that, phat = efie.sph_basis(self.dirs)
        rows_R = []
        for d, rh in enumerate(self.dirs):
            ph_d = torch.exp(torch.complex(torch.zeros_like(qp[..., 0]), k * (qp @ torch.as_tensor(rh))))
            a = torch.einsum("ta,tiax->tix", W.to(DT) * ph_d, f.to(DT))      # (T, 3, 3)
            for e in (that[d], phat[d]):
                c = (a * torch.as_tensor(e).to(DT)).sum(-1) * (-1j * k * eta / (4 * math.pi))
                rows_R.append(torch.zeros(N, dtype=DT).index_add(0, self.te.reshape(-1), c.reshape(-1)))
        Rm = torch.stack(rows_R)                                          # (2D, N)
        return Z, V, Rm

    def objective(self, x):
        Z, V, Rm = self.parts(x)
        j = torch.linalg.solve(Z, V)
        F = Rm @ j
        return (F.real ** 2 + F.imag ** 2).sum()


def objective_and_gradient(prob, xyz):
    x = torch.tensor(np.asarray(xyz, dtype=np.float64), requires_grad=True)
    J = prob.objective(x)
    (g,) = torch.autograd.grad(J, x)
    return float(J.detach()), g.numpy()


def objective_value(prob, xyz):
    with torch.no_grad():
        return float(prob.objective(torch.as_tensor(np.asarray(xyz, dtype=np.float64))))


def term_gradients(prob, xyz, j, lam, W):
    """The three parts of the adjoint gradient for fixed vectors j, lambda, W:
    2 Re[W^T (dR/dx) j], 2 Re[lambda^T dV/dx] and -2 Re[lambda^T (dZ/dx) j],
    each as the autograd derivative of the real scalar it differentiates."""
    x = torch.tensor(np.asarray(xyz, dtype=np.float64), requires_grad=True)
    Z, V, Rm = prob.parts(x)
    j = torch.as_tensor(np.asarray(j, dtype=np.complex128))
    lam = torch.as_tensor(np.asarray(lam, dtype=np.complex128))
    W = torch.as_tensor(np.asarray(W, dtype=np.complex128)).reshape(-1)
    rad = 2.0 * (W * (Rm @ j)).sum().real
    exc = 2.0 * (lam * V).sum().real
    op = -2.0 * (lam * (Z @ j)).sum().real
    out = []
    for s in (rad, exc, op):
        (g,) = torch.autograd.grad(s, x, retain_graph=True)
        out.append(g.numpy())
    return tuple(out)


def adjoint_vectors(prob, xyz):
    """j, F, W = conj(F) and lambda (Z lambda = R^T W) at xyz, by dense LU."""
    with torch.no_grad():
        Z, V, Rm = prob.parts(torch.as_tensor(np.asarray(xyz, dtype=np.float64)))
        j = torch.linalg.solve(Z, V)
        F = Rm @ j
        W = F.conj().resolve_conj()
        lam = torch.linalg.solve(Z, Rm.T @ W)
    return j.numpy(), F.numpy(), W.numpy(), lam.numpy()
