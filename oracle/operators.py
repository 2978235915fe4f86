"""Galerkin operators T, K and the static operators (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

For basis functions u_m (on particle mu) and v_n (on particle nu, shifted by
the centre offset) this module computes, by direct quadrature (7-point rule
on every triangle of both surfaces, Sec. II.A testing):

  T_mn = -jk <u_m, int g v_n> + (j/k) <div u_m, int g div' v_n>
  K_mn = <u_m, int v_n x grad g>           (grad on the observation point)

i.e. the Galerkin entries of eqs. PMCHWT_Finite1 written through the dyadic
Green's function of eq. T_far1 (Sec. IV), with g = exp(-jkR)/(4 pi R).

On the self surface, triangle pairs that share a vertex are integrated by
singularity subtraction (Sec. IV cites Graglia 1993 / Hodges 1997 for these
integrals): g = g0 + (g - g0) with g0 = 1/(4 pi R); the smooth remainder uses
the same 7x7 point rule and the g0 part uses the closed-form inner integrals
of ``quadrature.potential_integrals`` with the 7-point outer rule.  The
static operators of Sec. III (eqs. Operator_Tlo and Operator_Tto, kernel g0
of eq. StaticGreen) are the same construction with k -> 0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .basis import MeshBasis
from .quadrature import potential_integrals, subdivided_rule

FOUR_PI = 4.0 * np.pi


class SelfSingular:
    """Closed-form g0 parts over touching triangle pairs in the local basis
    (3F x 3F dense):
      Xvec[(a,i),(b,j)] = int_a h_ai . int_b h_bj g0
      Xdiv[(a,i),(b,j)] = int_a div h_ai  int_b div h_bj g0
      XK  [(a,i),(b,j)] = int_a h_ai . int_b h_bj x grad g0
    The inner integral over b is exact (closed form); the outer integral over
    a uses the 7-point rule on 4**outer_levels pieces of a, because the
    inner integral of grad g0 has a logarithmic edge singularity when a and b
    share an edge.
    """

    def __init__(self, mb: MeshBasis, outer_levels: int = 2):
        F = mb.nF
        self.touch = np.zeros((F, F), dtype=bool)
        pairs = mb.touching_pairs()
        self.touch[pairs[:, 0], pairs[:, 1]] = True
        nodes, wq = subdivided_rule(outer_levels)
        nr = len(wq)
        pts_all = np.einsum("qk,tkc->tqc", nodes, mb.tri_verts)        # [F][nr][3]
        wts_all = mb.area[:, None] * wq[None, :]
        Xvec = np.zeros((F, 3, F, 3))
        Xdiv = np.zeros((F, 3, F, 3))
        XK = np.zeros((F, 3, F, 3))
        for b in range(F):
            A = np.nonzero(self.touch[:, b])[0]                 # outer triangles
            r = pts_all[A].reshape(-1, 3)
            w = wts_all[A].reshape(-1)
            I0, J, gI0 = potential_integrals(r, mb.tri_verts[b])
            ab, bb = mb.loc_a[b], mb.loc_b[b]                   # [3], [3][3]
            inner_vec = (ab[None, :, None] * (J + r * I0[:, None])[:, None, :]
                         + bb[None, :, :] * I0[:, None, None]) / FOUR_PI     # [n][3j][3c]
            ext = ab[None, :, None] * r[:, None, :] + bb[None, :, :]         # [n][3j][3c]
            inner_K = np.cross(ext, gI0[:, None, :]) / FOUR_PI               # [n][3j][3c]
            aa = np.repeat(mb.loc_a[A], nr, axis=0)                          # [n][3i]
            ba = np.repeat(mb.loc_b[A], nr, axis=0)                          # [n][3i][3c]
            h_out = aa[:, :, None] * r[:, None, :] + ba                      # [n][3i][3c]
            hw = h_out * w[:, None, None]
            Xvec[A, :, b, :] = np.einsum("nic,njc->nij", hw, inner_vec).reshape(len(A), nr, 3, 3).sum(1)
            XK[A, :, b, :] = np.einsum("nic,njc->nij", hw, inner_K).reshape(len(A), nr, 3, 3).sum(1)
            Xdiv[A, :, b, :] = np.einsum("ni,n,j->nij", 2.0 * aa, w * I0 / FOUR_PI, 2.0 * ab).reshape(len(A), nr, 3, 3).sum(1)
        self.Xvec = Xvec.reshape(3 * F, 3 * F)
        self.Xdiv = Xdiv.reshape(3 * F, 3 * F)
        self.XK = XK.reshape(3 * F, 3 * F)


class SampledBasis:
    """N functions (rows of C over the RWG functions of ``mb``) sampled at the
    quadrature points: values Psi[c] (N x Q), divergence Sig (N x Q), local
    coefficients B (N x 3F)."""

    def __init__(self, mb: MeshBasis, C):
        self.mb = mb
        self.B = mb.mode_local(C)
        Hc, Hd = mb.local_values()
        self.Psi = [np.asarray((Hc[c].T @ self.B.T).T) for c in range(3)]
        self.Sig = np.asarray((Hd.T @ self.B.T).T)
        self.X, self.W = mb.flat_points()


def _cmul(Z, Rm):
    """complex [m][q] times real [q][n] as two real products"""
    return np.ascontiguousarray(Z.real) @ Rm + 1j * (np.ascontiguousarray(Z.imag) @ Rm)


def direct_TK(bp: SampledBasis, bq: SampledBasis, offset, k, touch=None, chunk=1024):
    """Direct-quadrature T and K between the functions of bp (observation
    surface) and bq (source surface translated by ``offset``).  If ``touch``
    (F x F bool, self surface only) is given, the touching triangle pairs use
    the smooth remainder g - g0 in place of g.

    With grad g(r - r') = (r - r') h(R), K is evaluated as
      K_mn = sum_a [ (r_a x psi_m(a)) . U_n(a) - psi_m(a) . V_n(a) ],
      U_n(a) = sum_b h_ab psi_n(b),  V_n(a) = sum_b h_ab psi_n(b) x r_b,
    which is psi_m . (psi_n x (r_a - r_b)) h summed over all point pairs."""
    Xp, Wp = bp.X, bp.W
    Xq = bq.X + np.asarray(offset, float)[None, :]
    Wq = bq.W
    Np, Nq = bp.Sig.shape[0], bq.Sig.shape[0]
    T = np.zeros((Np, Nq), complex)
    K = np.zeros((Np, Nq), complex)
    nq = bp.mb.nq
    Psq = np.stack(bq.Psi, -1)                              # [Nq][Q][3]
    cross_q = np.cross(Psq, Xq[None, :, :])                 # psi_n(b) x r_b
    # source columns: G side [psi_x psi_y psi_z div], H side [psi_x.. , (psi x r)_x..]
    Gcols = np.ascontiguousarray(np.concatenate([bq.Psi[0], bq.Psi[1], bq.Psi[2], bq.Sig], 0).T)
    Hcols = np.ascontiguousarray(np.concatenate([bq.Psi[0], bq.Psi[1], bq.Psi[2],
                                                 cross_q[..., 0], cross_q[..., 1], cross_q[..., 2]], 0).T)
    Psp = np.stack(bp.Psi, -1)                              # [Np][Q][3]
    rxpsi = np.cross(Xp[None, :, :], Psp)                   # r_a x psi_m(a)
    blk = lambda M, c: M[:, c * Nq:(c + 1) * Nq]
    real_k = np.isreal(k) and touch is None
    kr = float(np.real(k))
    for r0 in range(0, len(Xp), chunk):
        r1 = min(r0 + chunk, len(Xp))
        Rv = Xp[r0:r1, None, :] - Xq[None, :, :]            # r - r'
        R = np.sqrt(np.einsum("ijc,ijc->ij", Rv, Rv))
        wrow = Wp[r0:r1, None]
        ww = wrow * Wq[None, :]
        if real_k:
            kR = kr * R
            c, s = np.cos(kR), np.sin(kR)
            inv = ww / (FOUR_PI * R)
            Gr, Gi = c * inv, -s * inv
            inv3 = inv / (R * R)
            Hr, Hi = -(c + kR * s) * inv3, -(kR * c - s) * inv3
            A = Gr @ Gcols + 1j * (Gi @ Gcols)
            B = Hr @ Hcols + 1j * (Hi @ Hcols)
        else:
            if touch is not None:
                tmask = touch[np.ix_(np.arange(r0, r1) // nq, np.arange(len(Xq)) // nq)]
            else:
                tmask = np.zeros(R.shape, bool)
            Rs = np.where(R > 0, R, 1.0)
            e = np.exp(-1j * k * Rs)
            g = np.where(tmask, (e - 1.0) / (FOUR_PI * Rs), e / (FOUR_PI * Rs))
            g = np.where(R > 0, g, -1j * k / FOUR_PI)
            h = -(1.0 + 1j * k * Rs) * e / (FOUR_PI * Rs ** 3)
            h = np.where(tmask, h + 1.0 / (FOUR_PI * Rs ** 3), h)
            h = np.where(R > 0, h, 0.0)
            A = _cmul(g * ww, Gcols)
            B = _cmul(h * ww, Hcols)
        for cc in range(3):
            T += -1j * k * (bp.Psi[cc][:, r0:r1] @ blk(A, cc))
            K += rxpsi[:, r0:r1, cc] @ blk(B, cc) - bp.Psi[cc][:, r0:r1] @ blk(B, 3 + cc)
        T += (1j / k) * (bp.Sig[:, r0:r1] @ blk(A, 3))
    return T, K


def self_TK(bs: SampledBasis, sing: SelfSingular, k):
    """T and K of one surface on itself for wavenumber k (complex allowed):
    direct part with g - g0 on touching pairs plus the closed-form g0 parts."""
    T, K = direct_TK(bs, bs, np.zeros(3), k, touch=sing.touch)
    B = bs.B
    T += -1j * k * (B @ sing.Xvec @ B.T) + (1j / k) * (B @ sing.Xdiv @ B.T)
    K += B @ sing.XK @ B.T
    return T, K


def static_rwg_operators(mb: MeshBasis, sing: SelfSingular):
    """RWG-basis Gram G, single-layer S0 = int int f_i . f_j g0 and
    Phi0 = int int div f_i div' f_j g0 (the matrices of the static operators
    of Sec. III tested with the same functions)."""
    Hc, Hd = mb.local_values()
    X, W = mb.flat_points()
    nq = mb.nq
    Rv = X[:, None, :] - X[None, :, :]
    R = np.linalg.norm(Rv, axis=-1)
    tmask = np.repeat(np.repeat(sing.touch, nq, axis=0), nq, axis=1)
    G0 = np.where(tmask, 0.0, 1.0 / (FOUR_PI * np.where(R > 0, R, 1.0)))
    G0w = W[:, None] * G0 * W[None, :]
    Sloc = sum((Hc[c] @ (Hc[c] @ G0w.T).T) for c in range(3))
    Dloc = Hd @ (Hd @ G0w.T).T
    Sloc = np.asarray(Sloc) + sing.Xvec
    Dloc = np.asarray(Dloc) + sing.Xdiv
    Wd = sp.diags(W)
    Gloc = sum((Hc[c] @ Wd @ Hc[c].T) for c in range(3)).toarray()
    P = mb.P
    S0 = np.asarray(P @ Sloc @ P.T)
    Phi0 = np.asarray(P @ Dloc @ P.T)
    Gram = np.asarray(P @ Gloc @ P.T)
    return Gram, S0, Phi0
