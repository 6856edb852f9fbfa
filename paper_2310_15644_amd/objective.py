"""Far-field objective of the vertex positions as a differentiable torch function.

J(x) = sum_{d,c} |F_c(rhat_d)|^2 for the current that solves Z(x) j = V(x) under
one incident plane wave, F = R(x) j the far field in (theta, phi) components --
the discretised EFIE (Sec. II, with the Galerkin matrices of Sec. III) seen as a
function of the mesh vertices.  Every step runs in libefie:

  forward : efie_assemble (FP64) -> efie_excite_planewave -> efie_solve (COCG)
            -> efie_farfield -> efie_farfield_objective (J and W = conj(F));
            Z, j and W are kept for the backward pass.
  backward: g = R^T W (efie_farfield_adjoint); the adjoint solve
            Z lambda = g reuses the saved Z because Z = Z^T; then
            dJ/dx = 2 Re[W^T dR/dx j + lambda^T dV/dx - lambda^T dZ/dx j]
            (efie_vertex_grad).

The near-pair classification is the one of the mesh at x (it is frozen while
differentiating: the objective is piecewise defined by it).
"""
from __future__ import annotations

import numpy as np
import torch

from . import (C128, COCG, ETA0, Mesh, assemble, excite_planewave, farfield, farfield_adjoint, farfield_objective,
               solve, vertex_grad)


class FarFieldObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, triangles, k, khat, pol, dirs, e0=1.0, eta=ETA0, tol=1e-12, near_factor=2.0,
                maxit=20000):
        dev = torch.device("cuda", torch.cuda.current_device()) if not xyz.is_cuda else xyz.device
        mesh = Mesh(xyz.detach().to("cpu", torch.float64).numpy(), np.asarray(triangles), near_factor,
                    device=dev).upload(dev)
        Z = assemble(mesh, k, eta, C128)
        V = excite_planewave(mesh, k, np.asarray(khat, np.float64).reshape(1, 3),
                             np.asarray(pol, np.float64).reshape(1, 3), e0)
        J, st = solve(Z, V, COCG, tol=tol, maxit=maxit)
        if int(st.status[0]) != 0:
            raise RuntimeError(f"forward solve did not converge (relres {st.relres_true[0]:.3e})")
        d = torch.as_tensor(np.asarray(dirs, dtype=np.float64).reshape(-1, 3), device=dev)
        F = farfield(mesh, k, J, d, eta)
        obj, W = farfield_objective(F)
        ctx.mesh, ctx.Z, ctx.J, ctx.W, ctx.d = mesh, Z, J, W, d
        ctx.args = (float(k), np.asarray(khat, np.float64).reshape(3), np.asarray(pol, np.float64).reshape(3),
                    float(e0), float(eta), float(tol), int(maxit))
        ctx.xyz_device = xyz.device
        return obj.to(xyz.device)

    @staticmethod
    def backward(ctx, gout):
        k, khat, pol, e0, eta, tol, maxit = ctx.args
        mesh, Z, J, W, d = ctx.mesh, ctx.Z, ctx.J, ctx.W, ctx.d
        g = farfield_adjoint(mesh, k, W, d, eta)
        lam, st = solve(Z, g, COCG, tol=tol, maxit=maxit)
        if int(st.status[0]) != 0:
            raise RuntimeError(f"adjoint solve did not converge (relres {st.relres_true[0]:.3e})")
        dx = vertex_grad(mesh, k, J.reshape(-1), lam.reshape(-1), W.reshape(-1), d, khat, pol, e0, eta)
        grad = dx.to(ctx.xyz_device) * gout.to(ctx.xyz_device)
        return (grad,) + (None,) * 10


def far_field_objective(xyz, triangles, k, khat, pol, dirs, e0=1.0, eta=ETA0, tol=1e-12, near_factor=2.0):
    """J = sum |F|^2 as a differentiable function of xyz (nv, 3) float64."""
    return FarFieldObjective.apply(xyz, triangles, k, khat, pol, dirs, e0, eta, tol, near_factor)
