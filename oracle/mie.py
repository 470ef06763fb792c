"""Mie series for a perfectly conducting sphere (Section 4's analytic reference).

Incident E = x_hat exp(i k z) (E0 = 1 V/m), exp(-i w t) convention.  With
psi_n(x) = x j_n(x), xi_n(x) = x h_n^(1)(x) and size parameter x = k a, the
PEC coefficients are a_n = psi_n'(x)/xi_n'(x), b_n = psi_n(x)/xi_n(x); the
amplitude functions are
    S1 = sum (2n+1)/(n(n+1)) (a_n pi_n + b_n tau_n),
    S2 = sum (2n+1)/(n(n+1)) (a_n tau_n + b_n pi_n),
with the angular functions pi_n = P_n^1(cos t)/sin t, tau_n = d P_n^1/dt,
and the far field F = lim r e^{-ikr} E^s = (i/k)[cos(phi) S2 theta_hat -
sin(phi) S1 phi_hat]  (Bohren & Huffman, ch. 4, perfect-conductor limit).

Pin: its small-sphere limit against the radiation of the induced electric
and magnetic dipoles p = 4 pi eps0 a^3 E0 x_hat, m = -2 pi a^3 H0 y_hat
(tests/test_oracle_mie.py), which is an independent textbook result.
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def coefficients(ka, nmax=None):
    if nmax is None:
        nmax = int(np.ceil(ka + 4.0 * ka ** (1.0 / 3.0) + 8))
    n = np.arange(1, nmax + 1)
    j = spherical_jn(n, ka)
    jp = spherical_jn(n, ka, derivative=True)
    y = spherical_yn(n, ka)
    yp = spherical_yn(n, ka, derivative=True)
    h = j + 1j * y
    hp = jp + 1j * yp
    psi = ka * j
    psip = j + ka * jp
    xi = ka * h
    xip = h + ka * hp
    return n, psip / xip, psi / xi


def farfield(ka, k, dirs):
    """Far-field vector F [nd,3] of the PEC sphere of radius a = ka/k."""
    dirs = np.atleast_2d(dirs)
    n, a, b = coefficients(ka)
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    th = np.arccos(np.clip(z, -1.0, 1.0))
    ph = np.arctan2(y, x)
    mu = np.cos(th)
    nmax = n[-1]
    pi = np.zeros((nmax + 1, mu.size))
    tau = np.zeros((nmax + 1, mu.size))
    pi[1] = 1.0
    tau[1] = mu
    for m in range(2, nmax + 1):
        pi[m] = (2 * m - 1) / (m - 1) * mu * pi[m - 1] - m / (m - 1) * pi[m - 2]
        tau[m] = m * mu * pi[m] - (m + 1) * pi[m - 1]
    c = (2 * n + 1) / (n * (n + 1))
    S1 = np.sum((c * a)[:, None] * pi[1:] + (c * b)[:, None] * tau[1:], axis=0)
    S2 = np.sum((c * a)[:, None] * tau[1:] + (c * b)[:, None] * pi[1:], axis=0)
    th_hat = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], 1)
    ph_hat = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], 1)
    return (1j / k) * ((np.cos(ph) * S2)[:, None] * th_hat - (np.sin(ph) * S1)[:, None] * ph_hat)


def dipole_farfield(a, k, dirs):
    """Rayleigh limit: far field of p = 4 pi eps0 a^3 x_hat and
    m = -2 pi a^3 (1/eta0) y_hat for E0 = 1 (times the usual factors):
    F = (k^2/(4 pi eps0)) [(rhat x p) x rhat] - (k^2 eta0/(4 pi)) (rhat x m)."""
    dirs = np.atleast_2d(dirs)
    p = 4.0 * np.pi * a ** 3 * np.array([1.0, 0.0, 0.0])          # p/eps0
    m_eta = -2.0 * np.pi * a ** 3 * np.array([0.0, 1.0, 0.0])     # m*eta0
    Fp = np.cross(np.cross(dirs, p), dirs)
    Fm = np.cross(dirs, m_eta)
    return (k ** 2 / (4.0 * np.pi)) * (Fp - Fm)
