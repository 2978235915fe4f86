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


def mie_near_field(radius: float, k: float, m: complex, pts, n_max=None):
    """Scattered E at exterior points of a sphere centred at the origin, lit
    by E_inc = x exp(-j k z) (unit amplitude, exp(+jwt)), from the vector
    spherical wave expansion (Bohren & Huffman sec. 4.4, written there for
    exp(-iwt) and E_inc = x exp(ikz)):
      E_s = sum_n E_n (i a_n N_e1n - b_n M_o1n),  E_n = i^n (2n+1)/(n(n+1)),
      M_o1n = cos(phi) pi_n h_n th_hat - sin(phi) tau_n h_n ph_hat,
      N_e1n = cos(phi) n(n+1) sin(th) pi_n h_n/rho r_hat
              + cos(phi) tau_n (rho h_n)'/rho th_hat - sin(phi) pi_n (rho h_n)'/rho ph_hat,
    with h_n the outgoing spherical Hankel function h_n^(1)(rho), rho = k r,
    and pi_n, tau_n the angular functions of mie_s1_s2.  For a real index m
    the exp(+jwt) field of E_inc = x exp(-jkz) is the complex conjugate of
    that one.  pts [D][3] -> E [D][3] (Cartesian)."""
    from scipy.special import spherical_jn, spherical_yn
    m = complex(m)
    if abs(m.imag) > 0:
        raise ValueError("mie_near_field: the conjugation argument needs a real index")
    x = k * radius
    a, b = mie_coefficients(x, m, n_max)
    N = len(a)
    pts = np.atleast_2d(np.asarray(pts, float))
    r = np.linalg.norm(pts, axis=1)
    th = np.arccos(np.clip(pts[:, 2] / r, -1.0, 1.0))
    ph = np.arctan2(pts[:, 1], pts[:, 0])
    mu = np.cos(th)
    rho = k * r
    pi_n = np.zeros((N + 1, len(mu)))
    tau_n = np.zeros((N + 1, len(mu)))
    pi_n[1] = 1.0
    if N >= 2:
        pi_n[2] = 3 * mu
    for n in range(3, N + 1):
        pi_n[n] = ((2 * n - 1) / (n - 1)) * mu * pi_n[n - 1] - (n / (n - 1)) * pi_n[n - 2]
    for n in range(1, N + 1):
        tau_n[n] = n * mu * pi_n[n] - (n + 1) * pi_n[n - 1]
    Er = np.zeros(len(r), complex)
    Et = np.zeros(len(r), complex)
    Ep = np.zeros(len(r), complex)
    cp, sp_, st = np.cos(ph), np.sin(ph), np.sin(th)
    for n in range(1, N + 1):
        h = spherical_jn(n, rho) + 1j * spherical_yn(n, rho)
        dh = spherical_jn(n, rho, derivative=True) + 1j * spherical_yn(n, rho, derivative=True)
        drh = (h + rho * dh) / rho                          # (rho h)'/rho
        En = (1j ** n) * (2 * n + 1) / (n * (n + 1))
        M_t, M_p = cp * pi_n[n] * h, -sp_ * tau_n[n] * h
        N_r = cp * n * (n + 1) * st * pi_n[n] * h / rho
        N_t, N_p = cp * tau_n[n] * drh, -sp_ * pi_n[n] * drh
        Er += En * (1j * a[n - 1] * N_r)
        Et += En * (1j * a[n - 1] * N_t - b[n - 1] * M_t)
        Ep += En * (1j * a[n - 1] * N_p - b[n - 1] * M_p)
    rh = np.stack([st * cp, st * sp_, mu], -1)
    thh = np.stack([mu * cp, mu * sp_, -st], -1)
    phh = np.stack([-sp_, cp, 0 * cp], -1)
    E = Er[:, None] * rh + Et[:, None] * thh + Ep[:, None] * phh
    return np.conj(E)
