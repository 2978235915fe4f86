"""Static surface-current modes (oracle).  Sec. III.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Transverse modes (eqs. AuxProb_Tt, Operator_Tto): expanded and tested with
loop functions, the eigenproblem is (L^T S0 L) v = gamma (L^T G L) v; the N_perp
largest gamma are kept (descending).  Longitudinal modes (eqs. AuxProb_Tl,
Operator_Tlo): expanded and tested with star functions,
(S^T Phi0 S) v = gamma (S^T G S) v; the N_par smallest gamma are kept
(ascending).  The basis order is {transverse..., longitudinal...} (Sec. III).

Readings where the paper is silent: each mode is normalised to <psi, psi> = 1
and signed so that its RWG coefficient of largest magnitude is positive.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .basis import MeshBasis
from .operators import SelfSingular, static_rwg_operators


def static_modes(mb: MeshBasis, n_perp: int, n_par: int, sing: SelfSingular | None = None):
    """Return (M [(n_perp+n_par) x E], gamma_perp [n_perp], gamma_par [n_par])."""
    sing = sing or SelfSingular(mb)
    Gram, S0, Phi0 = static_rwg_operators(mb, sing)
    Lp = mb.loops()
    St = mb.stars()
    Ap, Bp = Lp.T @ S0 @ Lp, Lp.T @ Gram @ Lp
    As, Bs = St.T @ Phi0 @ St, St.T @ Gram @ St
    gp, vp = sla.eigh(0.5 * (Ap + Ap.T), 0.5 * (Bp + Bp.T))
    gs, vs = sla.eigh(0.5 * (As + As.T), 0.5 * (Bs + Bs.T))
    order_p = np.argsort(gp)[::-1][:n_perp]
    order_s = np.argsort(gs)[:n_par]
    Mp = (Lp @ vp[:, order_p]).T
    Ms = (St @ vs[:, order_s]).T
    M = np.vstack([Mp, Ms])
    # normalise <psi, psi> = 1 and fix the sign
    nrm = np.sqrt(np.einsum("ie,ef,if->i", M, Gram, M))
    M = M / nrm[:, None]
    idx = np.argmax(np.abs(M), axis=1)
    M = M * np.sign(M[np.arange(len(M)), idx])[:, None]
    return M, gp[order_p], gs[order_s]
