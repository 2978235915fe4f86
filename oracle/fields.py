"""Scattered fields and cross-sections from the equivalent currents (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The exterior scattered field of currents (j_e, j_m) is z- L j_e + K j_m with
the operators of Sec. II (Green's function g-, wavenumber k- and impedance
z- of the background; see ``pmchwt``).  In the far zone,
g ~ exp(-jkr)/(4 pi r) exp(+jk rhat . r'), so
  r exp(jkr) E_s(r rhat) = -(jk/4pi) [ z- (I - rhat rhat) Jhat - rhat x Mhat ],
  Jhat = sum_mu sum_n J_{mu,e,n} int psi_n exp(jk rhat . r') dS'   (same for M).
C_sca = int |r E_s|^2 dOmega / |E0|^2 over the unit sphere (Sec. V.A).
"""
from __future__ import annotations

import numpy as np

from .pmchwt import DenseProblem


def far_amplitude(prob: DenseProblem, x, rhat):
    """F(rhat) = r exp(jkr) E_s for unknowns x [P][n]; rhat [D][3] -> [D][3]."""
    rhat = np.atleast_2d(rhat)
    k, zeta = prob.k, prob.zeta
    Jh = np.zeros((len(rhat), 3), complex)
    Mh = np.zeros((len(rhat), 3), complex)
    for mu in range(prob.n_particles):
        pc = prob.classes[prob.class_id[mu]]
        N = pc.n_modes
        X = pc.bs.X + prob.centers[mu][None, :]
        ph = np.exp(1j * k * (rhat @ X.T)) * pc.bs.W[None, :]        # [D][Q]
        for c in range(3):
            modes = pc.bs.Psi[c]                                       # [N][Q]
            Jh[:, c] += ph @ (modes.T @ x[mu][:N])
            Mh[:, c] += ph @ (modes.T @ x[mu][N:])
    Jt = Jh - rhat * np.einsum("dc,dc->d", rhat, Jh)[:, None]
    return -(1j * k / (4 * np.pi)) * (zeta * Jt - np.cross(rhat, Mh))


def sphere_grid(n_theta: int = 32, n_phi: int = 64):
    """Gauss-Legendre in cos(theta) x uniform phi directions and weights."""
    u, wu = np.polynomial.legendre.leggauss(n_theta)
    th = np.arccos(u)
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    T, Ph = np.meshgrid(th, ph, indexing="ij")
    rhat = np.stack([np.sin(T) * np.cos(Ph), np.sin(T) * np.sin(Ph), np.cos(T)], -1).reshape(-1, 3)
    w = (wu[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).ravel()
    return rhat, w


def scattering_cross_section(prob: DenseProblem, x, n_theta=32, n_phi=64):
    rhat, w = sphere_grid(n_theta, n_phi)
    F = far_amplitude(prob, x, rhat)
    return float(np.sum(w * np.sum(np.abs(F) ** 2, axis=1)))


def extinction_cross_section(prob: DenseProblem, x, khat, pol):
    """Optical theorem for exp(+jwt): C_ext = (4 pi / k) Im[pol* . F(khat)] with
    the sign fixed by the exp(+jwt) phasor convention (|pol| = 1)."""
    F = far_amplitude(prob, x, np.asarray(khat, float)[None, :])[0]
    return float(-(4 * np.pi / prob.k) * np.imag(np.vdot(pol, F)))


def near_field(prob: DenseProblem, x, pts):
    """Scattered E at exterior points (>= a few triangle sizes from every
    surface) by direct quadrature of z- L j_e + K j_m."""
    pts = np.atleast_2d(pts)
    k, zeta = prob.k, prob.zeta
    E = np.zeros((len(pts), 3), complex)
    for mu in range(prob.n_particles):
        pc = prob.classes[prob.class_id[mu]]
        N = pc.n_modes
        X = pc.bs.X + prob.centers[mu][None, :]
        W = pc.bs.W
        Je = np.stack([pc.bs.Psi[c].T @ x[mu][:N] for c in range(3)], -1) * W[:, None]   # [Q][3]
        Jm = np.stack([pc.bs.Psi[c].T @ x[mu][N:] for c in range(3)], -1) * W[:, None]
        dJ = (pc.bs.Sig.T @ x[mu][:N]) * W                                              # [Q]
        Rv = pts[:, None, :] - X[None, :, :]
        R = np.linalg.norm(Rv, axis=-1)
        g = np.exp(-1j * k * R) / (4 * np.pi * R)
        h = -(1 + 1j * k * R) * np.exp(-1j * k * R) / (4 * np.pi * R ** 3)            # grad g = Rv h
        # zeta L j = zeta (-jk int g j + (1/jk) grad int g div'j)
        E += zeta * (-1j * k * (g @ Je) + (1 / (1j * k)) * np.einsum("pq,pqc->pc", h * dJ[None, :], Rv))
        # K m = int m x grad g
        E += np.einsum("pq,pqc->pc", h, np.cross(Jm[None, :, :], Rv))
    return E
