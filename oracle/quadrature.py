"""Triangle quadrature and closed-form static potential integrals (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

* ``triangle_rule``: Radon's 7-point rule, exact for polynomials of total
  degree <= 5 on a triangle.  Used for every surface integral (Sec. II.A
  Galerkin testing, eq. kspace_Rap patterns).
* ``potential_integrals``: for a flat triangle T' and observation points r,
      I0(r)   = int_T' 1/|r-r'| dS'
      J(r)    = int_T' (r'-r)/|r-r'| dS'
      gI0(r)  = grad_r int_T' 1/|r-r'| dS'
  in closed form (edge-by-edge formulas of the kind the paper cites for the
  singular integrals, Sec. IV: refs. Graglia 1993 / Hodges 1997).  The normal
  part of gI0 on the plane of T' is taken as 0 (principal value).
"""
from __future__ import annotations

import math

import numpy as np


def triangle_rule():
    """Barycentric nodes [7][3] and weights [7] (weights sum to 1; multiply by
    the triangle area).  Radon's degree-5 formula: centroid, and two orbits
    with parameters (6 -+ sqrt 15)/21 and weights (155 -+ sqrt 15)/1200."""
    s15 = math.sqrt(15.0)
    a1 = (6.0 - s15) / 21.0
    a2 = (6.0 + s15) / 21.0
    w1 = (155.0 - s15) / 1200.0
    w2 = (155.0 + s15) / 1200.0
    bary = [(1 / 3, 1 / 3, 1 / 3)]
    wts = [9.0 / 40.0]
    for a, w in ((a1, w1), (a2, w2)):
        b = 1.0 - 2.0 * a
        bary += [(b, a, a), (a, b, a), (a, a, b)]
        wts += [w, w, w]
    return np.array(bary), np.array(wts)


def subdivided_rule(levels: int):
    """The 7-point rule applied on each of the 4**levels congruent pieces of a
    uniform midpoint subdivision: barycentric nodes [7*4**levels][3] and
    weights summing to 1."""
    bary, w = triangle_rule()
    subs = [np.eye(3)]
    for _ in range(levels):
        nxt = []
        for t in subs:
            m01, m12, m20 = (t[0] + t[1]) / 2, (t[1] + t[2]) / 2, (t[2] + t[0]) / 2
            nxt += [np.array([t[0], m01, m20]), np.array([m01, t[1], m12]),
                    np.array([m20, m12, t[2]]), np.array([m01, m12, m20])]
        subs = nxt
    nodes = np.concatenate([bary @ s for s in subs])
    wts = np.tile(w, len(subs)) / len(subs)
    return nodes, wts


def _safe_log_ratio(Rp, lp, Rm, lm, R0sq):
    """ln((R+ + l+)/(R- + l-)) without cancellation.  Since l+ > l-, either
    both are >= 0, both < 0, or l- < 0 <= l+; for l < 0 the identity
    R + l = R0^2/(R - l) removes the cancellation."""
    out = np.empty_like(Rp)
    pos = lm >= 0
    neg = lp < 0
    mix = ~(pos | neg)
    out[pos] = np.log((Rp[pos] + lp[pos]) / (Rm[pos] + lm[pos]))
    out[neg] = np.log((Rm[neg] - lm[neg]) / (Rp[neg] - lp[neg]))
    out[mix] = np.log((Rp[mix] + lp[mix]) * (Rm[mix] - lm[mix]) / R0sq[mix])
    return out


def potential_integrals(r: np.ndarray, tri: np.ndarray):
    """Closed-form I0, J, gI0 for observation points r [N][3] and one flat
    triangle tri [3][3] (vertices, counter-clockwise about its normal)."""
    r = np.atleast_2d(np.asarray(r, float))
    a = np.asarray(tri, float)
    n = np.cross(a[1] - a[0], a[2] - a[0])
    n /= np.linalg.norm(n)
    d = (r - a[0]) @ n                       # signed height [N]
    rho = r - d[:, None] * n[None, :]        # projection on the plane
    ad = np.abs(d)
    I0 = np.zeros(len(r))
    J = np.zeros((len(r), 3))
    g_in = np.zeros((len(r), 3))
    omega = np.zeros(len(r))
    tiny = 1e-14 * max(np.linalg.norm(a[1] - a[0]), 1e-300)
    for i in range(3):
        p, q = a[i], a[(i + 1) % 3]
        L = np.linalg.norm(q - p)
        lhat = (q - p) / L
        uhat = np.cross(lhat, n)             # outward in-plane edge normal
        lp = (q[None, :] - rho) @ lhat
        lm = (p[None, :] - rho) @ lhat
        P0 = (p[None, :] - rho) @ uhat       # > 0 when rho is on the inner side
        R0sq = P0 ** 2 + d ** 2
        Rp = np.sqrt(R0sq + lp ** 2)
        Rm = np.sqrt(R0sq + lm ** 2)
        f = np.zeros(len(r))
        ok = R0sq > tiny ** 2
        f[ok] = _safe_log_ratio(Rp[ok], lp[ok], Rm[ok], lm[ok], R0sq[ok])
        # an observation point on the edge line but outside the segment
        on_line = ~ok & ((lp < 0) == (lm < 0)) & (np.abs(lp) > tiny) & (np.abs(lm) > tiny)
        f[on_line] = np.log(np.abs(lp[on_line]) / np.abs(lm[on_line])) * np.sign(lp[on_line])
        beta = np.zeros(len(r))
        nz = np.abs(P0) > tiny
        beta[nz] = (np.arctan(P0[nz] * lp[nz] / (R0sq[nz] + ad[nz] * Rp[nz]))
                    - np.arctan(P0[nz] * lm[nz] / (R0sq[nz] + ad[nz] * Rm[nz])))
        I0 += np.where(nz, P0 * f, 0.0) - ad * beta
        J += 0.5 * (np.where(ok, R0sq * f, 0.0) + lp * Rp - lm * Rm)[:, None] * uhat[None, :]
        g_in -= f[:, None] * uhat[None, :]
        omega += beta
    # (r' - r) = (rho' - rho) - d n
    J = J - (d * I0)[:, None] * n[None, :]
    sd = np.where(ad > tiny, np.sign(d), 0.0)  # on the plane: principal value
    gI0 = g_in - (sd * omega)[:, None] * n[None, :]
    return I0, J, gI0


def brute_force_integrals(r, tri, levels: int = 6):
    """Reference for ``potential_integrals`` by uniform subdivision of the
    triangle into 4**levels pieces with the 7-point rule on each (slow)."""
    r = np.atleast_2d(np.asarray(r, float))
    tri = np.asarray(tri, float)
    bary, w = triangle_rule()
    subs = [tri]
    for _ in range(levels):
        nxt = []
        for t in subs:
            m01, m12, m20 = (t[0] + t[1]) / 2, (t[1] + t[2]) / 2, (t[2] + t[0]) / 2
            nxt += [np.array([t[0], m01, m20]), np.array([m01, t[1], m12]),
                    np.array([m20, m12, t[2]]), np.array([m01, m12, m20])]
        subs = nxt
    subs = np.array(subs)                                   # [S][3][3]
    area = 0.5 * np.linalg.norm(np.cross(subs[:, 1] - subs[:, 0], subs[:, 2] - subs[:, 0]), axis=1)
    pts = np.einsum("qk,skc->sqc", bary, subs).reshape(-1, 3)
    ww = (area[:, None] * w[None, :]).ravel()
    diff = pts[None, :, :] - r[:, None, :]                  # r' - r
    R = np.linalg.norm(diff, axis=-1)
    I0 = (ww / R).sum(1)
    J = np.einsum("nq,nqc->nc", ww / R, diff)
    gI0 = np.einsum("nq,nqc->nc", ww / R ** 3, diff)        # grad_r 1/R = (r'-r)/R^3
    return I0, J, gI0
