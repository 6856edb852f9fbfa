"""Mie series for a perfectly conducting sphere (oracle).

Bohren and Huffman, Absorption and Scattering of Light by Small Particles (1983),
ch. 4, in the limit of infinite conductivity:
  a_n = psi_n'(x) / xi_n'(x),  b_n = psi_n(x) / xi_n(x),
  psi_n = x j_n(x),  xi_n = x h_n^(1)(x),  x = k a,
  S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),
  S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n),
  pi_n = P_n^1(cos t)/sin t,  tau_n = d P_n^1(cos t)/dt  (Bohren-Huffman sign: no Condon-Shortley phase),
  sigma(t, phi) = (4 pi / k^2) (|S2|^2 cos^2 phi + |S1|^2 sin^2 phi),
with t the scattering angle from the propagation direction and phi measured
from the incident polarisation.  Magnitudes do not depend on the time convention.
Truncation n_max = x + 4 x^(1/3) + 10 (Wiscombe).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def coefficients(x):
    nmax = int(x + 4.0 * x ** (1.0 / 3.0) + 10)
    n = np.arange(1, nmax + 1)
    jn = spherical_jn(n, x)
    yn = spherical_yn(n, x)
    jnp = spherical_jn(n, x, derivative=True)
    ynp = spherical_yn(n, x, derivative=True)
    psi = x * jn
    xi = x * (jn + 1j * yn)
    dpsi = jn + x * jnp
    dxi = (jn + 1j * yn) + x * (jnp + 1j * ynp)
    return n, dpsi / dxi, psi / xi


def angular(nmax, t):
    """pi_n, tau_n for n = 1..nmax at scattering angles t (upward recurrences, B&H 4.47)."""
    mu = np.cos(t)
    pi = np.zeros((nmax + 1,) + np.shape(t))
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, nmax + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * (pi[n - 2] if n >= 2 else 0.0)
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def amplitudes(x, t):
    n, a, b = coefficients(x)
    pi, tau = angular(len(n), np.asarray(t, dtype=np.float64))
    c = ((2 * n + 1) / (n * (n + 1))).reshape((-1,) + (1,) * np.ndim(t))
    S1 = np.sum(c * (a.reshape(c.shape) * pi + b.reshape(c.shape) * tau), axis=0)
    S2 = np.sum(c * (a.reshape(c.shape) * tau + b.reshape(c.shape) * pi), axis=0)
    return S1, S2


def bistatic_rcs(ka, radius, t, phi):
    """sigma(t, phi) in m^2 for a sphere of the given radius at k = ka / radius."""
    k = ka / radius
    S1, S2 = amplitudes(ka, t)
    return 4.0 * math.pi / k ** 2 * (np.abs(S2) ** 2 * np.cos(phi) ** 2 + np.abs(S1) ** 2 * np.sin(phi) ** 2)


def efficiencies(x):
    """Q_ext (optical theorem) and Q_sca."""
    n, a, b = coefficients(x)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * (a + b).real)
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return qext, qsca
