"""The paper's 2-D method on a closed curve (oracle): boundary integral operators,
the TM CFIE of a PEC cylinder, its Calderon-stabilized form, the circular
counterpart, the randomized skeleton of their difference and the Woodbury inverse.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Operators (paper Sec. II, eqs. 1-5), time factor e^{+j omega t}:
  G_k(R) = -(j/4) H0^(2)(k R)                         (eq. 5)
  (S psi)(r)  = int G_k(r - r') psi(r') dS'            (eq. 1, single layer)
  (D* psi)(r) = p.v. int d/dn_r G_k(r - r') psi dS'    (eq. 3, adjoint double layer)
  (N psi)(r)  = -f.p. int d/dn_r d/dn_r' G_k psi dS'   (eq. 4, hypersingular)
with n the outward normal.  k may be complex (the paper's k~ has Im k~ < 0);
H0^(2) and H1^(2) of complex argument come from scipy.special (a library routine
used as a step).

Galerkin (paper Sec. III: (O)_ij = (lambda_i, O lambda_j), G_ij = (lambda_i,
lambda_j)) with piecewise-linear lambda_i on the polygon through the nodes:
segment a runs from node a to node a+1 (mod N), x in [0, 1] its local parameter,
lambda_a = 1 - x and lambda_{a+1} = x on it.  N enters through the Maue identity
  (lambda_i, N lambda_j) = int int G [lambda_i' lambda_j' - k^2 (n . n') lambda_i lambda_j]
(primes: arc-length derivatives), a reading: the paper defines N by its finite
part only.

Quadrature of a segment pair (a reading; the paper names none), identical on the
GPU side:
  * pairs that share no node: q x q Gauss-Legendre;
  * adjacent pairs (one shared node V): each segment parametrized from V (u, w in
    [0, 1]); the square split along u = w into two triangles, each mapped by
    (s, t) -> (s, s t) (Duffy), s = sigma^2 (grading), NQ x NQ Gauss-Legendre in
    (sigma, t); the full kernels are integrated so;
  * the segment with itself: D* vanishes (straight segment: (r - r') . n = 0);
    G = -(1/2 pi) ln R + G_reg(R), the log part in closed form
    (int int ln|x - y| dx dy over the unit square: -3/2; with weights x: -3/4;
    x y: -7/16), G_reg by NQ x NQ Gauss-Legendre; G_reg(0) = -j/4 -
    (ln(k/2) + gamma)/(2 pi).
NQ = 8.

PEC cylinder, TM incidence E_z^inc = exp(-j k khat . r) (paper Sec. III, eq. 7,
first row, with the readings below):
  EFIE part  S j = E_z^inc / (j k eta),
  MFIE part  (1/2 + D*) j = H_t^inc,  H_t = (n x H) . z = -(khat . n) E_z^inc / eta,
  CFIE       C = S + G/2 + D*,  right-hand side e/(j k eta) + h,
with e_i = (lambda_i, E_z^inc), h_i = (lambda_i, H_t^inc) (q-point rule per
segment).  The Calderon-stabilized operator (eq. 16) and its right-hand side:
  C_p = N_k~ G^-1 S_k + (G/2 - D*_k~) G^-1 (G/2 + D*_k),
  b_p = N_k~ G^-1 e/(j k eta) + (G/2 - D*_k~) G^-1 h,
TE incidence H_z^inc = exp(-j k khat . r) (the paper's "other polarization", whose
formulas it does not print; the readings follow by the same Calderon structure),
unknown the tangential current j_t along t = z x n:
  EFIE part  N j = (j k / eta) (lambda, E_t^inc),  E_t = eta (khat . n) H_z^inc,
  MFIE part  (1/2 - D) j = -(lambda, H_z^inc),   D = D*^T the double layer,
  C_p^TE = S_k~ G^-1 N_k + (G/2 + D_k~) G^-1 (G/2 - D_k)   (S N = 1/4 - D^2),
  b_p^TE = S_k~ G^-1 (j k / eta) e_t - (G/2 + D_k~) G^-1 h_z.
k~ = k - 0.4 j k^(1/3) a^(-2/3) with a = P / 2 pi, P the curve's perimeter (the
reciprocal of the arc-length mean of the curvature of a closed curve, whose
total curvature is 2 pi: a reading of the paper's "suitable average"; a = 1 for
the perimeter-2 pi contours).  The circular counterpart C_p,c is C_p on the circle
of the same perimeter with the same N, k and k~ (circulant); A = C_p - C_p,c is
compressed by an adaptive blocked randomized range finder (Halko et al.) and C_p
is inverted by the Woodbury identity (eqs. 17-18).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

ETA0 = 376.730313668
EULER_GAMMA = 0.57721566490153286061
NQ = 8          # Gauss points per direction of the near-pair rules

# int int_{[0,1]^2} phi_a(x) phi_b(y) ln|x - y| dx dy for phi_0 = 1 - x, phi_1 = x
_LOGMOM = np.array([[-7.0 / 16.0, -5.0 / 16.0], [-5.0 / 16.0, -7.0 / 16.0]])


def gauss01(q):
    """q-point Gauss-Legendre rule on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def green(k, R):
    """G_k(R) = -(j/4) H0^(2)(k R)."""
    return -0.25j * special.hankel2(0, k * R)


def dgreen_dR(k, R):
    """d G_k / dR = (j k / 4) H1^(2)(k R)."""
    return 0.25j * k * special.hankel2(1, k * R)


def green_reg(k, R):
    """G_k(R) + ln(R) / (2 pi), with its limit -j/4 - (ln(k/2) + gamma)/(2 pi) at R = 0."""
    k = complex(k)
    R = np.asarray(R, dtype=float)
    zero = R == 0.0
    Rs = np.where(zero, 1.0, R)
    val = green(k, Rs) + np.log(Rs) / (2.0 * math.pi)
    lim = -0.25j - (np.log(k / 2.0) + EULER_GAMMA) / (2.0 * math.pi)
    return np.where(zero, lim, val)


class Contour:
    """Closed polygon through nodes (N, 2), counter-clockwise (outward normal to
    the right of the direction of travel)."""

    def __init__(self, nodes):
        self.nodes = np.asarray(nodes, dtype=float)
        self.n = len(self.nodes)
        self.A = self.nodes
        self.B = np.roll(self.nodes, -1, axis=0)
        d = self.B - self.A
        self.L = np.linalg.norm(d, axis=1)
        self.t = d / self.L[:, None]
        self.nrm = np.stack([self.t[:, 1], -self.t[:, 0]], axis=1)
        self.perimeter = float(self.L.sum())

    def point(self, a, x):
        """Points of segment(s) a at local parameter(s) x."""
        return self.A[a] + np.asarray(x)[..., None] * (self.B[a] - self.A[a])


def ktilde(k, a=1.0):
    """k~ = k - 0.4 j k^(1/3) a^(-2/3) (paper Sec. III); a = P / 2 pi for a curve of
    perimeter P (a = 1 for the paper's perimeter-2 pi contours)."""
    return complex(k, -0.4 * np.cbrt(k) / np.cbrt(a) ** 2)


# ----------------------------------------------------------- segment-pair blocks
def _phi(x):
    """(phi_0, phi_1) = (1 - x, x), stacked on a new first axis."""
    x = np.asarray(x)
    return np.stack([1.0 - x, x])


def _blocks_from_samples(k, c, a, b, ra, rb, xa, yb, wgt):
    """2 x 2 blocks (S, D*, N) of test segment a and source segment b from kernel
    samples at points ra (test) and rb (source) with local parameters xa, yb and
    weights wgt (already including every Jacobian; no segment lengths)."""
    d = ra - rb
    R = np.linalg.norm(d, axis=-1)
    G = green(k, R)
    dG = dgreen_dR(k, R) * (d @ c.nrm[a]) / R
    pa, pb = _phi(xa), _phi(yb)
    pa, pb = pa.reshape(2, -1), pb.reshape(2, -1)
    mS = np.einsum("ip,jp,p->ij", pa, pb, (wgt * G).ravel())
    mD = np.einsum("ip,jp,p->ij", pa, pb, (wgt * dG).ravel())
    m0 = np.sum(wgt * G)
    return mS, mD, m0


def pair_blocks(c, k, a, b, q=4):
    """(S, D*, N) 2 x 2 local blocks of test segment a against source segment b:
    block[alpha][beta] couples lambda of the start (alpha = 0) or end (1) node of a
    with that of b."""
    n = c.n
    La, Lb = c.L[a], c.L[b]
    sig = np.array([-1.0, 1.0])
    if a == b:
        xg, wg = gauss01(NQ)
        X, Y = np.meshgrid(xg, xg, indexing="ij")
        W = wg[:, None] * wg[None, :]
        R = La * np.abs(X - Y)
        Gr = green_reg(k, R)
        pa, pb = _phi(X), _phi(Y)
        sing = -(1.0 / (2.0 * math.pi)) * (np.log(La) * 0.25 + _LOGMOM)
        mS = np.einsum("ip,jp,p->ij", pa.reshape(2, -1), pb.reshape(2, -1), (W * Gr).ravel()) + sing
        m0 = np.sum(W * Gr) - (1.0 / (2.0 * math.pi)) * (np.log(La) + (-1.5))
        mD = np.zeros((2, 2), dtype=complex)
    elif b == (a + 1) % n or b == (a - 1) % n:
        sg, swt = gauss01(NQ)
        tg, twt = gauss01(NQ)
        S_, T_ = np.meshgrid(sg, tg, indexing="ij")
        W = (swt[:, None] * twt[None, :]) * 2.0 * S_ ** 3     # Duffy (s) times grading (2 sigma)
        s = S_ ** 2
        if b == (a + 1) % n:
            V, Pa, Pb = c.B[a], c.A[a], c.B[b]
            xa_of = lambda u: 1.0 - u
            yb_of = lambda w: w
        else:
            V, Pa, Pb = c.A[a], c.B[a], c.A[b]
            xa_of = lambda u: u
            yb_of = lambda w: 1.0 - w
        mS = np.zeros((2, 2), dtype=complex)
        mD = np.zeros((2, 2), dtype=complex)
        m0 = 0.0j
        for u, w in ((s, s * T_), (s * T_, s)):
            ra = V + u[..., None] * (Pa - V)
            rb = V + w[..., None] * (Pb - V)
            s1, d1, z1 = _blocks_from_samples(k, c, a, b, ra, rb, xa_of(u), yb_of(w), W)
            mS += s1
            mD += d1
            m0 += z1
    else:
        xg, wg = gauss01(q)
        X, Y = np.meshgrid(xg, xg, indexing="ij")
        W = wg[:, None] * wg[None, :]
        ra = c.point(a, X)
        rb = c.point(b, Y)
        mS, mD, m0 = _blocks_from_samples(k, c, a, b, ra, rb, X, Y, W)
    S = La * Lb * mS
    D = La * Lb * mD
    N = np.outer(sig, sig) * m0 - k * k * float(c.nrm[a] @ c.nrm[b]) * S
    return S, D, N


def _regular_row(c, k, a, q):
    """(S, D*, m0) moments of test segment a against every source segment by the
    q x q rule: mS, mD (N, 2, 2) raw (no lengths), m0 (N,)."""
    xg, wg = gauss01(q)
    n = c.n
    ra = c.point(a, xg)                                   # (q, 2)
    rb = c.point(np.arange(n)[:, None], xg[None, :])      # (N, q, 2)
    d = ra[None, :, None, :] - rb[:, None, :, :]          # (N, q, q, 2)
    R = np.linalg.norm(d, axis=-1)
    G = green(k, R)
    dG = dgreen_dR(k, R) * (d @ c.nrm[a]) / R
    W = wg[:, None] * wg[None, :]
    ph = _phi(xg)
    mS = np.einsum("ip,jq,bpq->bij", ph, ph, W[None] * G)
    mD = np.einsum("ip,jq,bpq->bij", ph, ph, W[None] * dG)
    m0 = np.einsum("pq,bpq->b", W, G)
    return mS, mD, m0


def assemble(c, k, q=4):
    """Dense Galerkin matrices (S_k, D*_k, N_k) of the contour, each (N, N) complex."""
    n = c.n
    S = np.zeros((n, n), dtype=complex)
    D = np.zeros((n, n), dtype=complex)
    Nm = np.zeros((n, n), dtype=complex)
    sig = np.array([-1.0, 1.0])
    nn = c.nrm @ c.nrm.T
    for a in range(n):
        mS, mD, m0 = _regular_row(c, k, a, q)
        sb = c.L[a] * c.L[:, None, None] * mS
        db = c.L[a] * c.L[:, None, None] * mD
        nb = np.outer(sig, sig)[None] * m0[:, None, None] - k * k * nn[a][:, None, None] * sb
        for b in {(a - 1) % n, a, (a + 1) % n}:
            sb[b], db[b], nb[b] = pair_blocks(c, k, a, b, q)
        ia = (a, (a + 1) % n)
        cols = (np.arange(n), (np.arange(n) + 1) % n)
        for al in range(2):
            for be in range(2):
                np.add.at(S[ia[al]], cols[be], sb[:, al, be])
                np.add.at(D[ia[al]], cols[be], db[:, al, be])
                np.add.at(Nm[ia[al]], cols[be], nb[:, al, be])
    return S, D, Nm


def assemble_rows(c, k, rows, q=4):
    """Selected rows of (S_k, D*_k, N_k): each (len(rows), N), from the segment pairs
    of the two segments around each row's node (the same blocks as assemble)."""
    n = c.n
    rows = list(rows)
    out = [np.zeros((len(rows), n), dtype=complex) for _ in range(3)]
    sig = np.array([-1.0, 1.0])
    nn = c.nrm @ c.nrm.T
    cols = (np.arange(n), (np.arange(n) + 1) % n)
    for r, i in enumerate(rows):
        for a, al in (((i - 1) % n, 1), (i, 0)):
            mS, mD, m0 = _regular_row(c, k, a, q)
            sb = c.L[a] * c.L[:, None, None] * mS
            db = c.L[a] * c.L[:, None, None] * mD
            nb = np.outer(sig, sig)[None] * m0[:, None, None] - k * k * nn[a][:, None, None] * sb
            for b in {(a - 1) % n, a, (a + 1) % n}:
                sb[b], db[b], nb[b] = pair_blocks(c, k, a, b, q)
            for be in range(2):
                np.add.at(out[0][r], cols[be], sb[:, al, be])
                np.add.at(out[1][r], cols[be], db[:, al, be])
                np.add.at(out[2][r], cols[be], nb[:, al, be])
    return tuple(out)


def gram(c):
    """(lambda_i, lambda_j): L/3 + L/3 on the diagonal, L/6 beside it (cyclic)."""
    n = c.n
    G = np.zeros((n, n))
    for a in range(n):
        i, j = a, (a + 1) % n
        G[i, i] += c.L[a] / 3.0
        G[j, j] += c.L[a] / 3.0
        G[i, j] += c.L[a] / 6.0
        G[j, i] += c.L[a] / 6.0
    return G


def excitation(c, k, phis, q=4, eta=ETA0):
    """(e, h): e_i = (lambda_i, E_z^inc), h_i = (lambda_i, H_t^inc) for plane waves
    E_z^inc = exp(-j k khat . r), khat = (cos phi, sin phi), H_t^inc = -(khat . n) E / eta.
    Returns two (S, N) arrays."""
    phis = np.atleast_1d(phis)
    xg, wg = gauss01(q)
    n = c.n
    e = np.zeros((len(phis), n), dtype=complex)
    h = np.zeros((len(phis), n), dtype=complex)
    pts = c.point(np.arange(n)[:, None], xg[None, :])          # (N seg, q, 2)
    ph = _phi(xg)                                                # (2, q)
    for s, p in enumerate(phis):
        kh = np.array([math.cos(p), math.sin(p)])
        E = np.exp(-1j * k * (pts @ kh))                         # (N, q)
        Ht = -(c.nrm @ kh)[:, None] * E / eta
        for al in range(2):
            ce = c.L * np.sum(wg * ph[al] * E, axis=1)
            ch = c.L * np.sum(wg * ph[al] * Ht, axis=1)
            idx = (np.arange(n) + al) % n
            np.add.at(e[s], idx, ce)
            np.add.at(h[s], idx, ch)
    return e, h


def excitation_te(c, k, phis, q=4, eta=ETA0):
    """(e_t, h_z): e_t,i = (lambda_i, E_t^inc), h_z,i = (lambda_i, H_z^inc) for TE plane
    waves H_z^inc = exp(-j k khat . r): E = (eta / (j k)) grad(H_z) x z, so that
    E_t = E . (z x n) = eta (khat . n) H_z.  Returns two (S, N) arrays."""
    phis = np.atleast_1d(phis)
    xg, wg = gauss01(q)
    n = c.n
    et = np.zeros((len(phis), n), dtype=complex)
    hz = np.zeros((len(phis), n), dtype=complex)
    pts = c.point(np.arange(n)[:, None], xg[None, :])
    ph = _phi(xg)
    for s, p in enumerate(phis):
        kh = np.array([math.cos(p), math.sin(p)])
        H = np.exp(-1j * k * (pts @ kh))
        Et = eta * (c.nrm @ kh)[:, None] * H
        for al in range(2):
            idx = (np.arange(n) + al) % n
            np.add.at(et[s], idx, c.L * np.sum(wg * ph[al] * Et, axis=1))
            np.add.at(hz[s], idx, c.L * np.sum(wg * ph[al] * H, axis=1))
    return et, hz


class System:
    """The operators of one contour for one polarization: TM (S_k, D*_k, N_k~, D*_k~)
    or TE (N_k, D*_k, S_k~, D*_k~), and G."""

    def __init__(self, c, k, kt=None, q=4, pol="TM"):
        self.c = c
        self.k = complex(k)
        self.kt = ktilde(k) if kt is None else complex(kt)
        self.pol = pol
        if pol == "TM":
            self.S, self.D, _ = assemble(c, self.k, q)
            _, self.Dt, self.Nt = assemble(c, self.kt, q)
        elif pol == "TE":
            _, self.D, self.N = assemble(c, self.k, q)
            self.St, self.Dt, _ = assemble(c, self.kt, q)
        else:
            raise ValueError("pol must be TM or TE")
        self.G = gram(c)
        self.q = q

    def cfie(self):
        return self.S + 0.5 * self.G + self.D

    def cfie_rhs(self, e, h, eta=ETA0):
        return e / (1j * self.k * eta) + h

    def calderon(self):
        """TM: C_p = N_k~ G^-1 S_k + (G/2 - D*_k~) G^-1 (G/2 + D*_k) (paper eq. 16);
        TE: C_p = S_k~ G^-1 N_k + (G/2 + D_k~) G^-1 (G/2 - D_k), D = D*^T."""
        Gi = np.linalg.inv(self.G)
        if self.pol == "TE":
            return self.St @ Gi @ self.N + (0.5 * self.G + self.Dt.T) @ Gi @ (0.5 * self.G - self.D.T)
        return self.Nt @ Gi @ self.S + (0.5 * self.G - self.Dt) @ Gi @ (0.5 * self.G + self.D)

    def calderon_rhs(self, e, h, eta=ETA0):
        """TM: b_p = N_k~ G^-1 e/(j k eta) + (G/2 - D*_k~) G^-1 h for e = (lambda, E_z),
        h = (lambda, H_t); TE: b_p = S_k~ G^-1 (j k/eta) e - (G/2 + D_k~) G^-1 h for
        e = (lambda, E_t), h = (lambda, H_z).  (S, N) stacks in and out."""
        Gi = np.linalg.inv(self.G)
        if self.pol == "TE":
            ee = (1j * self.k / eta * e).T
            return (self.St @ (Gi @ ee) - (0.5 * self.G + self.Dt.T) @ (Gi @ h.T)).T
        ee = (e / (1j * self.k * eta)).T
        return (self.Nt @ (Gi @ ee) + (0.5 * self.G - self.Dt) @ (Gi @ h.T)).T


def farfield(c, k, J, phis, q=4, pol="TM"):
    """Far-field pattern of currents J (S, N): (S, len(phis)).
    TM: F(phi) = int J(r') exp(j k rhat . r') dS' (E_z ~ -j k eta G F);
    TE: F(phi) = int (rhat . n(r')) J(r') exp(j k rhat . r') dS' (the tangential
    current along z x n radiates H_z = curl(A)_z ~ -j k (rhat x t)_z G F, and
    rhat x (z x n) = z (rhat . n))."""
    if pol not in ("TM", "TE"):
        raise ValueError("pol must be TM or TE")
    phis = np.atleast_1d(phis)
    xg, wg = gauss01(q)
    n = c.n
    pts = c.point(np.arange(n)[:, None], xg[None, :])
    ph = _phi(xg)
    J = np.atleast_2d(J)
    out = np.zeros((len(J), len(phis)), dtype=complex)
    for d, p in enumerate(phis):
        rh = np.array([math.cos(p), math.sin(p)])
        ex = np.exp(1j * k * (pts @ rh))                         # (N seg, q)
        for al in range(2):
            col = c.L * np.sum(wg * ph[al] * ex, axis=1)           # contribution of node a+al per segment a
            if pol == "TE":
                col = col * (c.nrm @ rh)
            idx = (np.arange(n) + al) % n
            out[:, d] += J[:, idx] @ col
    return out


def echo_width(k, F, eta=ETA0, pol="TM"):
    """2-D scattering width for unit incident amplitude: sigma = lim 2 pi rho |u_s|^2
    with u_s ~ c G F and |G|^2 ~ 1/(8 pi k rho): TM (u = E_z, c = -j k eta)
    sigma = (k eta^2 / 4) |F|^2; TE (u = H_z, c = -j k) sigma = (k / 4) |F|^2."""
    f = eta * eta if pol == "TM" else 1.0
    return 0.25 * k * f * np.abs(F) ** 2


# ------------------------------------------------------------ fast direct solver
def circulant_first_column(Cc):
    return Cc[:, 0].copy()


def circulant_solve(col, b):
    """x with C x = b for the circulant C of first column col (numpy FFT)."""
    lam = np.fft.fft(col)
    return np.fft.ifft(np.fft.fft(b, axis=0) / lam[:, None] if b.ndim == 2 else np.fft.fft(b) / lam, axis=0)


def range_finder(A, omega, block, tol, Cp):
    """Adaptive blocked randomized range finder (Halko, Martinsson, Tropp, SIAM
    Review 53(2), 2011, the adaptive range finder) on the dense A with the given
    test matrix omega (N, nblocks * block).  The reference scale is the largest
    column norm of C_p Omega_0 (the first block of the test matrix applied to the
    whole operator).  Each block Y = A Omega_b is projected twice against the basis
    Q found so far; the search stops when the largest column norm of the projected
    block is at most tol times the reference (that block is not added), else an
    orthonormal basis of the projected block (Householder QR) joins Q.
    Returns (Q, est, ref)."""
    n = A.shape[0]
    Q = np.zeros((n, 0), dtype=complex)
    ref = float(np.linalg.norm(Cp @ omega[:, :block], axis=0).max())
    est = 0.0
    for b0 in range(0, omega.shape[1], block):
        Y = A @ omega[:, b0:b0 + block]
        for _ in range(2):
            Y = Y - Q @ (Q.conj().T @ Y)
        est = float(np.linalg.norm(Y, axis=0).max())
        if est <= tol * ref:
            return Q, est, ref
        Qb, _ = np.linalg.qr(Y)
        Q = np.concatenate([Q, Qb[:, :n - Q.shape[1]]], axis=1)
        if Q.shape[1] == n:                 # the whole space: A is captured exactly
            return Q, 0.0, ref
    raise RuntimeError("range finder: test matrix exhausted before the tolerance was met")


class FastDirect:
    """C_p^-1 by the Woodbury identity around the circulant counterpart (eq. 18):
    C_p = C_c + U V^T with U = Q, V^T = Q^H (C_p - C_c)."""

    def __init__(self, Cp, Cc, omega, block, tol):
        self.col = circulant_first_column(Cc)
        A = Cp - Cc
        self.Q, self.est, self.ref = range_finder(A, omega, block, tol, Cp)
        self.rank = self.Q.shape[1]
        self.Vt = self.Q.conj().T @ A                      # (r, N)
        self.W = circulant_solve(self.col, self.Q) if self.rank else self.Q
        self.M = np.eye(self.rank) + self.Vt @ self.W       # I + V^T C_c^-1 U

    def solve(self, b):
        """x = C_c^-1 b - C_c^-1 U (I + V^T C_c^-1 U)^-1 V^T C_c^-1 b for b (N,) or (N, S)."""
        y = circulant_solve(self.col, b)
        if self.rank == 0:
            return y
        return y - self.W @ np.linalg.solve(self.M, self.Vt @ y)


# ----------------------------------------------------------------- analytic
def cylinder_current(k, a, phi, phi_inc=0.0, eta=ETA0, nmax=None):
    """Surface current J_z(phi) of a PEC circular cylinder of radius a under the TM
    plane wave exp(-j k khat . r), khat = (cos phi_inc, sin phi_inc):
    J = (2 / (pi k a eta)) sum_n j^-n exp(j n (phi - phi_inc)) / H_n^(2)(k a)
    (separation of variables; the Wronskian J_n H_n^(2)' - J_n' H_n^(2) = -2j/(pi x))."""
    x = k * a
    if nmax is None:
        nmax = int(x + 4.0 * x ** (1.0 / 3.0) + 15)
    ns = np.arange(-nmax, nmax + 1)
    phi = np.atleast_1d(phi)
    terms = (1j ** (-ns.astype(float)))[None, :] * np.exp(1j * ns[None, :] * (phi[:, None] - phi_inc)) \
        / special.hankel2(ns, x)[None, :]
    return 2.0 / (math.pi * x * eta) * terms.sum(axis=1)


def cylinder_echo_width(k, a, phi, phi_inc=0.0, nmax=None):
    """sigma(phi) = (4/k) |sum_n J_n(ka)/H_n^(2)(ka) exp(j n (phi - phi_inc))|^2, TM, PEC."""
    x = k * a
    if nmax is None:
        nmax = int(x + 4.0 * x ** (1.0 / 3.0) + 15)
    ns = np.arange(-nmax, nmax + 1)
    phi = np.atleast_1d(phi)
    c = special.jv(ns, x) / special.hankel2(ns, x)
    s = (c[None, :] * np.exp(1j * ns[None, :] * (phi[:, None] - phi_inc))).sum(axis=1)
    return 4.0 / k * np.abs(s) ** 2


def cylinder_echo_width_te(k, a, phi, phi_inc=0.0, nmax=None):
    """sigma(phi) = (4/k) |sum_n J_n'(ka)/H_n^(2)'(ka) exp(j n (phi - phi_inc))|^2, TE, PEC."""
    x = k * a
    if nmax is None:
        nmax = int(x + 4.0 * x ** (1.0 / 3.0) + 15)
    ns = np.arange(-nmax, nmax + 1)
    phi = np.atleast_1d(phi)
    c = special.jvp(ns, x) / special.h2vp(ns, x)
    s = (c[None, :] * np.exp(1j * ns[None, :] * (phi[:, None] - phi_inc))).sum(axis=1)
    return 4.0 / k * np.abs(s) ** 2


def cylinder_current_te(k, a, phi, phi_inc=0.0, nmax=None):
    """Tangential current j_t (along z x n) of a PEC circular cylinder of radius a under
    the TE plane wave H_z = exp(-j k khat . r): j_t = -H_z^tot on the surface,
    j_t = (2j / (pi k a)) sum_n j^-n exp(j n (phi - phi_inc)) / H_n^(2)'(k a)."""
    x = k * a
    if nmax is None:
        nmax = int(x + 4.0 * x ** (1.0 / 3.0) + 15)
    ns = np.arange(-nmax, nmax + 1)
    phi = np.atleast_1d(phi)
    terms = (1j ** (-ns.astype(float)))[None, :] * np.exp(1j * ns[None, :] * (phi[:, None] - phi_inc)) \
        / special.h2vp(ns, x)[None, :]
    return 2j / (math.pi * x) * terms.sum(axis=1)
