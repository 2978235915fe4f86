"""Mie series for a homogeneous sphere (oracle pin; textbook, Bohren &
Huffman ch. 4), used to check the single-sphere PMCHWT solution the way
Sec. V.A checks arrays against multiparticle Mie theory.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def mie_coefficients(x: float, m: complex, n_max: int | None = None):
    """a_n, b_n for size parameter x = k a and relative index m."""
    if n_max is None:
        n_max = int(np.ceil(x + 4 * x ** (1 / 3) + 2))
    n = np.arange(1, n_max + 1)
    mx = m * x

    def psi(nn, z):                                 # Riccati-Bessel z j_n(z)
        return z * spherical_jn(nn, z)

    def dpsi(nn, z):
        return spherical_jn(nn, z) + z * spherical_jn(nn, z, derivative=True)

    def xi(nn, z):                                  # z h_n^(1)(z)
        return z * (spherical_jn(nn, z) + 1j * spherical_yn(nn, z))

    def dxi(nn, z):
        h = spherical_jn(nn, z) + 1j * spherical_yn(nn, z)
        dh = spherical_jn(nn, z, derivative=True) + 1j * spherical_yn(nn, z, derivative=True)
        return h + z * dh

    px, dpx = psi(n, x), dpsi(n, x)
    pm, dpm = psi(n, mx), dpsi(n, mx)
    xx, dxx = xi(n, x), dxi(n, x)
    a = (m * pm * dpx - px * dpm) / (m * pm * dxx - xx * dpm)
    b = (pm * dpx - m * px * dpm) / (pm * dxx - m * xx * dpm)
    return a, b


def mie_cross_sections(radius: float, k: float, m: complex, n_max=None):
    """(C_sca, C_ext) for a sphere of the given radius."""
    x = k * radius
    a, b = mie_coefficients(x, m, n_max)
    n = np.arange(1, len(a) + 1)
    csca = 2 * np.pi / k ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    cext = 2 * np.pi / k ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    return float(csca), float(cext)


def mie_s1_s2(radius: float, k: float, m: complex, theta, n_max=None):
    """Scattering amplitudes S1 (perpendicular), S2 (parallel) vs theta."""
    x = k * radius
    a, b = mie_coefficients(x, m, n_max)
    mu = np.cos(np.asarray(theta, float))
    N = len(a)
    pi_n = np.zeros((N + 1, len(mu)))
    tau_n = np.zeros((N + 1, len(mu)))
    pi_n[1] = 1.0
    if N >= 2:
        pi_n[2] = 3 * mu
    for n in range(3, N + 1):
        pi_n[n] = ((2 * n - 1) / (n - 1)) * mu * pi_n[n - 1] - (n / (n - 1)) * pi_n[n - 2]
    for n in range(1, N + 1):
        tau_n[n] = n * mu * pi_n[n] - (n + 1) * pi_n[n - 1]
    s1 = np.zeros(len(mu), complex)
    s2 = np.zeros(len(mu), complex)
    for n in range(1, N + 1):
        c = (2 * n + 1) / (n * (n + 1))
        s1 += c * (a[n - 1] * pi_n[n] + b[n - 1] * tau_n[n])
        s2 += c * (a[n - 1] * tau_n[n] + b[n - 1] * pi_n[n])
    return s1, s2
