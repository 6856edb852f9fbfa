"""Seeded synthetic inputs shared by the GPU path, the oracle, the tests and the bench.

This module only builds geometry and excitation parameters (meshes, directions,
polarisations, wavenumbers).  It contains none of the method's arithmetic: no
basis functions, no Green's function, no quadrature, no operator.

Workloads (all in metres, free space):
  * PEC unit sphere meshed as an icosphere: recursive 4-split of the regular
    icosahedron with projection to the unit sphere after every level
    (level L has T = 20*4**L triangles, N = 30*4**L edges, V = 10*4**L + 2 vertices),
    vertices numbered in Morton order.
  * Ellipsoids: Class-I geodesic subdivision of frequency n of the icosahedron
    (each face split into n*n triangles), projected to the unit sphere and then
    scaled per axis.  N = 30*n*n edges.
  * Vertex-perturbed spheres: radius 1 + delta(theta, phi), delta a seeded real
    spherical-harmonic series of degree <= lmax scaled to max |delta| = amp.
  * Plane-wave grids and seeded observation directions.
  * 2-D contours (the paper's Sec. IV geometries): an ellipse of aspect ratio
    1.5 and perimeter 2 pi, a Joukowsky airfoil of perimeter 2 pi and the circle
    of the same perimeter, as nodes equally spaced in arc length; seeded complex
    Gaussian test matrices for the randomized range finder.

Every triangle is listed counter-clockwise seen from outside (outward normal).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "icosahedron",
    "icosphere",
    "geodesic_sphere",
    "ellipsoid",
    "perturbed_sphere",
    "uniform_directions",
    "monostatic_grid",
    "planewave_x_along_minus_z",
    "ellipsoid_batch",
    "contour_ellipse",
    "contour_joukowsky",
    "contour_circle",
    "gaussian_block",
    "morton_order",
]


def icosahedron():
    """Regular icosahedron on the unit sphere, 12 vertices, 20 outward CCW faces."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array(
        [
            [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
            [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
            [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
        ],
        dtype=np.float64,
    )
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int32,
    )
    return _orient_outward(v, f)


def _orient_outward(v, f):
    """Flip any face whose normal points towards the origin (star-shaped meshes)."""
    f = f.copy()
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    nrm = np.cross(b - a, c - a)
    inward = np.einsum("ij,ij->i", nrm, (a + b + c)) < 0
    f[inward] = f[inward][:, [0, 2, 1]]
    return v, f


def morton_order(v, bits: int = 21):
    """Permutation sorting points (V, 3) by their Morton (Z-order) code in the
    bounding box, `bits` per axis: neighbouring indices are neighbours in space."""
    v = np.asarray(v, dtype=np.float64)
    lo, hi = v.min(axis=0), v.max(axis=0)
    span = np.where(hi > lo, hi - lo, 1.0)
    q = np.minimum(((v - lo) / span * (2 ** bits - 1)).astype(np.int64), 2 ** bits - 1)
    code = np.zeros(len(v), dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            code |= ((q[:, d] >> b) & 1) << (3 * b + d)
    return np.argsort(code, kind="stable")


def icosphere(level: int):
    """Unit icosphere: recursive 4-split with projection after every level.

    Children of triangle t at one level are triangles 4t..4t+3 at the next,
    so the triangle order is hierarchical (spatially local).  The vertices are
    numbered in Morton order of their positions, so that RWG functions, numbered
    by their vertex ids, are spatially coherent in index ranges as well.
    """
    v, f = icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (i, j) if i < j else (j, i)
            if key not in cache:
                m = np.add(verts[i], verts[j]) * 0.5
                m /= np.linalg.norm(m)
                cache[key] = len(verts)
                verts.append(tuple(m))
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int32)
    v = np.array(verts, dtype=np.float64)
    order = morton_order(v)
    rank = np.empty(len(order), dtype=np.int32)
    rank[order] = np.arange(len(order), dtype=np.int32)
    return v[order], rank[np.asarray(f)].astype(np.int32)


def geodesic_sphere(n: int):
    """Class-I geodesic sphere of frequency n: every icosahedron face is split into
    n*n triangles on a barycentric lattice, then all points go to the unit sphere."""
    v0, f0 = icosahedron()
    verts = []
    index = {}

    def vid(key, pos):
        if key not in index:
            index[key] = len(verts)
            verts.append(pos / np.linalg.norm(pos))
        return index[key]

    faces = []
    for a, b, c in f0:
        A, B, C = v0[a], v0[b], v0[c]
        ids = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                k = n - i - j
                # canonical key: lattice point expressed on the shared corners so
                # points on shared edges/corners of neighbouring faces coincide
                parts = sorted(((a, i), (b, j), (c, k)))
                key = tuple((g, w) for g, w in parts if w > 0)
                pos = (i * A + j * B + k * C) / n
                ids[(i, j)] = vid(key, pos)
        for i in range(n):
            for j in range(n - i):
                # upward triangle
                p0, p1, p2 = ids[(i, j)], ids[(i + 1, j)], ids[(i, j + 1)]
                faces.append((p0, p1, p2))
                if i + j < n - 1:
                    q0, q1, q2 = ids[(i + 1, j)], ids[(i + 1, j + 1)], ids[(i, j + 1)]
                    faces.append((q0, q1, q2))
    v = np.array(verts, dtype=np.float64)
    f = np.array(faces, dtype=np.int32)
    return _orient_outward(v, f)


def ellipsoid(n: int, axes):
    """Geodesic sphere of frequency n scaled to semi-axes (a, b, c)."""
    v, f = geodesic_sphere(n)
    return v * np.asarray(axes, dtype=np.float64)[None, :], f


def ellipsoid_batch(count: int = 64, seed: int = 0, nmin: int = 6, nmax: int = 16):
    """Seeded batch of uneven ellipsoid meshes: n ~ U{nmin..nmax}, semi-axes ~ U[0.5, 1.5].
    Returns a list of (vertices, triangles, axes, n)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        axes = rng.uniform(0.5, 1.5, size=3)
        v, f = ellipsoid(n, axes)
        out.append((v, f, axes, n))
    return out


def _real_sph_harm(l, m, theta, phi):
    """Real spherical harmonic of degree l, order m (theta polar, phi azimuth)."""
    from scipy.special import lpmv

    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    p = lpmv(am, l, np.cos(theta))
    if m == 0:
        return norm * p
    if m > 0:
        return math.sqrt(2.0) * norm * p * np.cos(am * phi)
    return math.sqrt(2.0) * norm * p * np.sin(am * phi)


def perturbed_sphere(level: int, lmax: int = 6, amp: float = 0.05, seed: int = 0):
    """Icosphere with vertex radii 1 + delta, delta = s * sum c_lm Y_lm (c_lm ~ N(0,1)),
    s chosen so that max_v |delta| = amp."""
    v, f = icosphere(level)
    rng = np.random.default_rng(seed)
    theta = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    phi = np.arctan2(v[:, 1], v[:, 0])
    delta = np.zeros(len(v))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            delta += rng.standard_normal() * _real_sph_harm(l, m, theta, phi)
    delta *= amp / np.max(np.abs(delta))
    return v * (1.0 + delta)[:, None], f


def uniform_directions(count: int, seed: int = 1):
    """Seeded unit vectors uniform on the sphere (z ~ U[-1,1], phi ~ U[0, 2pi))."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, size=count)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=count)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)


def monostatic_grid(ntheta: int = 16, nphi: int = 32):
    """Uniform (theta, phi) grid: theta_i = (i + 1/2) pi / ntheta, phi_j = 2 pi j / nphi.

    Returns (rhat, khat, pol, theta, phi): observation/incidence direction rhat,
    propagation direction khat = -rhat, polarisation theta-hat, each (ntheta*nphi, 3).
    """
    th = (np.arange(ntheta) + 0.5) * math.pi / ntheta
    ph = 2.0 * math.pi * np.arange(nphi) / nphi
    T, P = np.meshgrid(th, ph, indexing="ij")
    T, P = T.ravel(), P.ravel()
    rhat = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=1)
    that = np.stack([np.cos(T) * np.cos(P), np.cos(T) * np.sin(P), -np.sin(T)], axis=1)
    return rhat, -rhat, that, T, P


def planewave_x_along_minus_z():
    """The single plane wave of the small sphere case: propagation -z, polarisation +x."""
    return np.array([[0.0, 0.0, -1.0]]), np.array([[1.0, 0.0, 0.0]])


# ------------------------------------------------------------- 2-D contours
def _equal_arclength(curve, n: int, samples: int = 1 << 16):
    """n points of the closed parametric curve z(t), t in [0, 1), equally spaced in
    arc length, counter-clockwise, the first at t = 0; and the curve's perimeter.
    Arc length from composite 5-point Gauss-Legendre on `samples` intervals, the
    inverse by interpolation refined with Newton steps on |z'(t)|."""
    x, w = np.polynomial.legendre.leggauss(5)
    t0 = np.arange(samples) / samples
    h = 1.0 / samples
    tq = t0[:, None] + 0.5 * h * (x[None, :] + 1.0)
    _, dz = curve(tq)
    seg = 0.5 * h * (np.abs(dz) * w[None, :]).sum(axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    per = cum[-1]
    target = per * np.arange(n) / n
    t = np.interp(target, cum, np.concatenate([t0, [1.0]]))
    for _ in range(3):   # Newton on s(t) = target with the local 5-point arc length
        i = np.minimum((t * samples).astype(np.int64), samples - 1)
        a = t0[i]
        tl = a[:, None] + 0.5 * (t - a)[:, None] * (x[None, :] + 1.0)
        _, dzl = curve(tl)
        s = cum[i] + 0.5 * (t - a) * (np.abs(dzl) * w[None, :]).sum(axis=1)
        _, dzt = curve(t)
        t = t - (s - target) / np.abs(dzt)
    z, _ = curve(t)
    return np.stack([z.real, z.imag], axis=1), per


def contour_ellipse(n: int, aspect: float = 1.5, perimeter: float = 2.0 * math.pi):
    """n nodes of the ellipse x^2/a^2 + y^2/b^2 = 1 with a = aspect * b and the given
    perimeter, equally spaced in arc length, counter-clockwise from (a, 0)."""
    from scipy.special import ellipe

    e2 = 1.0 - 1.0 / aspect ** 2
    b = perimeter / (4.0 * aspect * ellipe(e2))          # perimeter = 4 a E(e)
    a = aspect * b

    def curve(t):
        th = 2.0 * math.pi * t
        return a * np.cos(th) + 1j * b * np.sin(th), 2.0 * math.pi * (-a * np.sin(th) + 1j * b * np.cos(th))

    nodes, _ = _equal_arclength(curve, n)
    return nodes


def contour_joukowsky(n: int, center=(-0.08, 0.08), round_te: float = 1.02, perimeter: float = 2.0 * math.pi):
    """n nodes of a Joukowsky airfoil w = z + 1/z, the image of the circle through
    z = 1 about `center` with its radius enlarged by round_te (a rounded trailing
    edge instead of the cusp), scaled to the given perimeter; equally spaced in arc
    length, counter-clockwise, the first node at the trailing edge."""
    c = complex(*center)
    r0 = round_te * abs(1.0 - c)

    def raw(t):
        th = 2.0 * math.pi * t
        z = c + r0 * np.exp(1j * th)
        dz = 2.0j * math.pi * r0 * np.exp(1j * th)
        return z + 1.0 / z, dz * (1.0 - 1.0 / z ** 2)

    _, per = _equal_arclength(raw, 8, samples=1 << 16)
    s = perimeter / per

    def curve(t):
        w, dw = raw(t)
        return s * w, s * dw

    nodes, _ = _equal_arclength(curve, n)
    return nodes


def contour_circle(n: int, perimeter: float = 2.0 * math.pi):
    """n nodes of the circle of the given perimeter, node i at angle 2 pi i / n."""
    r = perimeter / (2.0 * math.pi)
    th = 2.0 * math.pi * np.arange(n) / n
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def gaussian_block(n: int, cols: int, seed: int = 0):
    """Seeded complex Gaussian test matrix (n, cols): real and imaginary parts
    N(0, 1/2), so that each entry has unit variance (the random draws of a
    randomized range finder, passed to it as an input)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, cols)) + 1j * rng.standard_normal((n, cols))) / math.sqrt(2.0)
