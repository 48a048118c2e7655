"""Mie series for a perfectly conducting sphere (Bohren and Huffman, Absorption and
Scattering of Light by Small Particles, 1983, sections 4.4 and 4.8): an analytic
reference for the scattering the oracle's EFIE, excitation and far field compute.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a plane wave polarised along x and travelling along the sphere's z axis, the
scattered far field is E_theta ~ cos(phi) S2(theta), E_phi ~ sin(phi) S1(theta) with
theta the scattering angle from the forward direction, and
    S1 = sum_n (2n + 1) / (n (n + 1)) (a_n pi_n + b_n tau_n),
    S2 = sum_n (2n + 1) / (n (n + 1)) (a_n tau_n + b_n pi_n),
where for a perfect conductor a_n = psi_n'(x) / xi_n'(x), b_n = psi_n(x) / xi_n(x)
(x = k a, psi_n = x j_n, xi_n = x h_n^(1)) and pi_n, tau_n are the angular functions of
the associated Legendre functions P_n^1.  The bistatic cross-section is
    sigma = (4 pi / k^2) (cos^2 phi |S2|^2 + sin^2 phi |S1|^2).
The time convention only conjugates S1, S2, so sigma does not depend on it.
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def coefficients(x: float, n_max: int | None = None):
    """a_n, b_n for n = 1 .. n_max (Wiscombe's n_max = x + 4 x^(1/3) + 2 by default)."""
    if n_max is None:
        n_max = int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0))
    n = np.arange(1, n_max + 1)
    j, jd = spherical_jn(n, x), spherical_jn(n, x, derivative=True)
    y, yd = spherical_yn(n, x), spherical_yn(n, x, derivative=True)
    h, hd = j + 1j * y, jd + 1j * yd
    psi, psid = x * j, j + x * jd
    xi, xid = x * h, h + x * hd
    return n, psid / xid, psi / xi


def angular(n_max: int, mu: np.ndarray):
    """pi_n(mu), tau_n(mu) for n = 1 .. n_max (upward recurrence), shape (n_max, len(mu))."""
    mu = np.asarray(mu, dtype=np.float64)
    pi = np.zeros((n_max + 1, mu.size))
    tau = np.zeros((n_max + 1, mu.size))
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, n_max + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def amplitudes(x: float, scatter_angle: np.ndarray, n_max: int | None = None):
    n, a, b = coefficients(x, n_max)
    pi, tau = angular(n.size, np.cos(scatter_angle))
    w = ((2 * n + 1) / (n * (n + 1)))[:, None]
    return (w * (a[:, None] * pi + b[:, None] * tau)).sum(0), (w * (a[:, None] * tau + b[:, None] * pi)).sum(0)


def bistatic_rcs(k: float, radius: float, scatter_angle: np.ndarray, phi: np.ndarray,
                 n_max: int | None = None) -> np.ndarray:
    """sigma (in the square of the length unit) at scattering angle theta from the
    forward direction and azimuth phi from the incident polarisation."""
    S1, S2 = amplitudes(k * radius, np.asarray(scatter_angle, dtype=np.float64), n_max)
    c2, s2 = np.cos(phi) ** 2, np.sin(phi) ** 2
    return 4.0 * np.pi / k ** 2 * (c2 * np.abs(S2) ** 2 + s2 * np.abs(S1) ** 2)


def extinction_and_scattering(k: float, radius: float, n_max: int | None = None):
    """(sigma_ext from the optical theorem, sigma_sca from the coefficient sum)."""
    n, a, b = coefficients(k * radius, n_max)
    S1, _ = amplitudes(k * radius, np.array([0.0]), n_max)
    ext = 4.0 * np.pi / k ** 2 * S1[0].real
    sca = 2.0 * np.pi / k ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return ext, sca
