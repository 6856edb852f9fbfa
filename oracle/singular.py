"""Closed-form potential integrals over a flat triangle (oracle).

For an observation point r and a flat source triangle with unit normal n:
  I0(r)  = integral over the triangle of 1/|r - r'| dS'
  I1(r)  = integral over the triangle of (rho' - rho)/|r - r'| dS'
where rho, rho' are the projections of r, r' on the triangle plane.
Formulas: Wilton et al., IEEE TAP 32(3), 1984; Graglia, IEEE TAP 41(10), 1993.
Per edge i (end points r-, r+ in counter-clockwise order about n):
  unit tangent lt, outward in-plane normal u = lt x n,
  l+- = (r+- - rho) . lt,  P0 = (r- - rho) . u,  d = n . (r - r-),
  R0^2 = P0^2 + d^2,  R+- = |r - r+-|,
  I0 = sum_i P0 ln[(R+ + l+)/(R- + l-)]
         - |d| sum_i [atan(P0 l+ / (R0^2 + |d| R+)) - atan(P0 l- / (R0^2 + |d| R-))],
  I1 = 1/2 sum_i u [R0^2 ln((R+ + l+)/(R- + l-)) + l+ R+ - l- R-].
The gradient form used by the magnetic (double-layer) operator:
  J(r) = integral over the triangle of (r - r')/|r - r'|^3 dS' = -grad_r I0(r)
       = sgn(d) n sum_i beta_i + sum_i u ln[(R+ + l+)/(R- + l-)],
  beta_i = atan(P0 l+ / (R0^2 + |d| R+)) - atan(P0 l- / (R0^2 + |d| R-))
(Wilton et al. 1984, the gradient of their potential formula), with sgn(d) = 0
where |d| <= 1e-12 times the longest edge: for a point in the plane of the
triangle the principal value, which carries no normal component.
The paper does not treat singular integrals; this is the reading taken for the
singularity extraction on near pairs.  Where an observation point lies on the
line of an edge (R0 ~ 0) the log coefficients vanish and the log terms are
dropped.  (R + l) is evaluated as R0^2 / (R - l) when l < 0 to avoid
cancellation; both are the same number in exact arithmetic.
"""
from __future__ import annotations

import numpy as np


def _r_plus_l(R, l, R02):
    return np.where(l >= 0.0, R + l, R02 / np.where(l >= 0.0, 1.0, R - l))


def _cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


def _dot(a, b):
    return np.sum(a * b, axis=-1)


def potential_integrals(r, v, drop_tol=1e-12):
    """r (..., M, 3) observation points; v (..., 3, 3) source triangle vertices (CCW).
    Leading dimensions broadcast.  Returns I0 (..., M) and I1 (..., M, 3)."""
    r = np.asarray(r, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    if r.ndim == 1:
        r = r[None, :]
    nrm = _cross(v[..., 1, :] - v[..., 0, :], v[..., 2, :] - v[..., 0, :])
    nrm = nrm / np.linalg.norm(nrm, axis=-1, keepdims=True)
    h = np.max(np.linalg.norm(v - np.roll(v, -1, axis=-2), axis=-1), axis=-1)   # (...)
    nrm_ = nrm[..., None, :]                                   # (..., 1, 3)
    d = _dot(r - v[..., None, 0, :], nrm_)                     # (..., M)
    rho = r - d[..., None] * nrm_
    ad = np.abs(d)
    I0 = np.zeros(d.shape)
    I1 = np.zeros(rho.shape)
    for i in range(3):
        rm, rp = v[..., None, i, :], v[..., None, (i + 1) % 3, :]   # (..., 1, 3)
        lt = (rp - rm) / np.linalg.norm(rp - rm, axis=-1, keepdims=True)
        u = _cross(lt, nrm_)
        lp = _dot(rp - rho, lt)
        lm = _dot(rm - rho, lt)
        P0 = _dot(rm - rho, u)
        R02 = P0 * P0 + d * d
        Rp = np.linalg.norm(r - rp, axis=-1)
        Rm = np.linalg.norm(r - rm, axis=-1)
        keep = np.sqrt(R02) >= drop_tol * h[..., None]
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.log(_r_plus_l(Rp, lp, R02) / _r_plus_l(Rm, lm, R02))
            at = np.arctan(P0 * lp / (R02 + ad * Rp)) - np.arctan(P0 * lm / (R02 + ad * Rm))
        lg = np.where(keep, lg, 0.0)
        at = np.where(keep, at, 0.0)
        I0 = I0 + P0 * lg - ad * at
        I1 = I1 + 0.5 * (R02 * lg + lp * Rp - lm * Rm)[..., None] * u
    return I0, I1


def gradient_integral(r, v, drop_tol=1e-12):
    """J(r) = int (r - r')/|r - r'|^3 dS' over the source triangle v (..., 3, 3), CCW,
    for observation points r (..., M, 3).  Returns (..., M, 3)."""
    r = np.asarray(r, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    if r.ndim == 1:
        r = r[None, :]
    nrm = _cross(v[..., 1, :] - v[..., 0, :], v[..., 2, :] - v[..., 0, :])
    nrm = nrm / np.linalg.norm(nrm, axis=-1, keepdims=True)
    h = np.max(np.linalg.norm(v - np.roll(v, -1, axis=-2), axis=-1), axis=-1)
    nrm_ = nrm[..., None, :]
    d = _dot(r - v[..., None, 0, :], nrm_)
    rho = r - d[..., None] * nrm_
    ad = np.abs(d)
    beta = np.zeros(d.shape)
    out = np.zeros(rho.shape)
    for i in range(3):
        rm, rp = v[..., None, i, :], v[..., None, (i + 1) % 3, :]
        lt = (rp - rm) / np.linalg.norm(rp - rm, axis=-1, keepdims=True)
        u = _cross(lt, nrm_)
        lp = _dot(rp - rho, lt)
        lm = _dot(rm - rho, lt)
        P0 = _dot(rm - rho, u)
        R02 = P0 * P0 + d * d
        Rp = np.linalg.norm(r - rp, axis=-1)
        Rm = np.linalg.norm(r - rm, axis=-1)
        keep = np.sqrt(R02) >= drop_tol * h[..., None]
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.log(_r_plus_l(Rp, lp, R02) / _r_plus_l(Rm, lm, R02))
            at = np.arctan(P0 * lp / (R02 + ad * Rp)) - np.arctan(P0 * lm / (R02 + ad * Rm))
        lg = np.where(keep, lg, 0.0)
        at = np.where(keep, at, 0.0)
        beta = beta + at
        out = out + lg[..., None] * u
    sd = np.where(ad <= drop_tol * h[..., None], 0.0, np.sign(d))
    return out + (sd * beta)[..., None] * nrm_
