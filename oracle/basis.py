"""RWG, loop and star functions on a closed triangle mesh (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The RWG function of edge e (Sec. II.A, the sub-domain basis xi) is
    f_e(r) = +(l_e / 2A+) (r - p+)   on T+,
    f_e(r) = -(l_e / 2A-) (r - p-)   on T-,
with p+- the vertices of T+- opposite e; its surface divergence is +-l_e/A+-.
It is written as the difference of two "local" triangle functions
    h_{t,i}(r) = (l_i / 2A_t) (r - v_i),   i = local vertex of triangle t,
so that every operator can be assembled triangle pair by triangle pair and
then mapped to RWG (matrix P) or to static modes (M P, eq.
BasisTransformation).

Loop functions (div-free, used for the transverse modes, Sec. III) are
n x grad(lambda_v) of the vertex hat functions; in RWG they have
coefficients +-1/l_e on the edges incident to v.  Star functions (used for
the longitudinal modes) are the RWG sums around a triangle with +1 where the
triangle is T+ and -1 where it is T-.  On a closed genus-0 surface the
loops sum to zero and so do the stars, so the last of each is dropped.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .quadrature import triangle_rule


class MeshBasis:
    """Geometry, quadrature points and local/RWG function data of one mesh
    (particle-local coordinates)."""

    def __init__(self, verts, tris, edges):
        self.verts = np.asarray(verts, float)
        self.tris = np.asarray(tris, np.int64)
        self.edges = np.asarray(edges, np.int64)
        V, F, E = len(self.verts), len(self.tris), len(self.edges)
        self.nV, self.nF, self.nE = V, F, E
        tv = self.verts[self.tris]                           # [F][3][3]
        cr = np.cross(tv[:, 1] - tv[:, 0], tv[:, 2] - tv[:, 0])
        self.area = 0.5 * np.linalg.norm(cr, axis=1)
        self.normal = cr / (2.0 * self.area[:, None])
        self.tri_verts = tv
        bary, wq = triangle_rule()
        self.nq = len(wq)
        self.pts = np.einsum("qk,tkc->tqc", bary, tv)           # [F][7][3]
        self.wts = self.area[:, None] * wq[None, :]             # [F][7]
        # local functions h_{t,i}: length of the edge opposite vertex i
        opp = np.stack([tv[:, 2] - tv[:, 1], tv[:, 0] - tv[:, 2], tv[:, 1] - tv[:, 0]], axis=1)
        self.loc_len = np.linalg.norm(opp, axis=2)              # [F][3]
        self.loc_a = self.loc_len / (2.0 * self.area[:, None])  # [F][3]
        self.loc_b = -self.loc_a[:, :, None] * tv               # [F][3][3]
        # RWG <-> local map: P[e, 3t+i]
        rows, cols, vals = [], [], []
        self.rwg_len = np.zeros(E)
        for e, (v0, v1, tp, tm) in enumerate(self.edges):
            ip = self._free_local(tp, v0, v1)
            im = self._free_local(tm, v0, v1)
            rows += [e, e]
            cols += [3 * tp + ip, 3 * tm + im]
            vals += [1.0, -1.0]
            self.rwg_len[e] = np.linalg.norm(self.verts[v1] - self.verts[v0])
        self.P = sp.csr_matrix((vals, (rows, cols)), shape=(E, 3 * F))

    def _free_local(self, t, v0, v1):
        tri = self.tris[t]
        for i in range(3):
            if tri[i] != v0 and tri[i] != v1:
                return i
        raise ValueError("degenerate edge table")

    # ---- local-function values at the quadrature points (sparse) --------
    def local_values(self):
        """Sparse matrices Hc[c] (3F x Q) of component c of h_{t,i} at every
        quadrature point, and Hd (3F x Q) of the divergence 2 a_{t,i}.  Point
        index = 7 t + q."""
        F, nq = self.nF, self.nq
        Q = F * nq
        rows = np.repeat(np.arange(3 * F), nq)
        t_of = np.repeat(np.arange(F), 3)
        cols = (t_of[:, None] * nq + np.arange(nq)[None, :]).ravel()
        a = self.loc_a.reshape(-1)                              # [3F]
        b = self.loc_b.reshape(-1, 3)                           # [3F][3]
        pts = self.pts[t_of]                                    # [3F][7][3]
        val = a[:, None, None] * pts + b[:, None, :]            # [3F][7][3]
        Hc = [sp.csr_matrix((val[:, :, c].ravel(), (rows, cols)), shape=(3 * F, Q)) for c in range(3)]
        dv = np.repeat(2.0 * a, nq)
        Hd = sp.csr_matrix((dv, (rows, cols)), shape=(3 * F, Q))
        return Hc, Hd

    def flat_points(self):
        return self.pts.reshape(-1, 3), self.wts.reshape(-1)

    # ---- touching triangle pairs (share at least one vertex) ------------
    def touching_pairs(self):
        vt = {}
        for t, tri in enumerate(self.tris):
            for v in tri:
                vt.setdefault(int(v), set()).add(t)
        pairs = set()
        for ts in vt.values():
            for a in ts:
                for b in ts:
                    pairs.add((a, b))
        return np.array(sorted(pairs), dtype=np.int64)

    # ---- loop and star coefficient matrices (RWG x functions) -----------
    def loops(self):
        """E x (V-1): loop at vertex v = sum_{e: v0=v} f_e/l_e - sum_{e: v1=v} f_e/l_e."""
        E, V = self.nE, self.nV
        L = np.zeros((E, V))
        for e, (v0, v1, _, _) in enumerate(self.edges):
            L[e, v0] += 1.0 / self.rwg_len[e]
            L[e, v1] -= 1.0 / self.rwg_len[e]
        return L[:, : V - 1]

    def stars(self):
        """E x (F-1): star at triangle t = sum of f_e (+1 if t = T+, -1 if T-)."""
        E, F = self.nE, self.nF
        S = np.zeros((E, F))
        for e, (_, _, tp, tm) in enumerate(self.edges):
            S[e, tp] += 1.0
            S[e, tm] -= 1.0
        return S[:, : F - 1]

    def rwg_divergence(self):
        """E x F matrix of the (constant) divergence of f_e on each triangle."""
        D = np.zeros((self.nE, self.nF))
        for e, (_, _, tp, tm) in enumerate(self.edges):
            D[e, tp] += self.rwg_len[e] / self.area[tp]
            D[e, tm] -= self.rwg_len[e] / self.area[tm]
        return D

    def mode_local(self, C):
        """Coefficients of N functions given as rows of C over RWG, expressed
        in the local basis: B = C P (N x 3F)."""
        return np.asarray((self.P.T @ np.asarray(C, dtype=float).T).T)
