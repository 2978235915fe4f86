"""Pins of the static modes (Sec. III): sphere closed forms, convergence,
orthonormality and diagonalisation."""
import numpy as np
import pytest

import workloads as w
from oracle.basis import MeshBasis
from oracle.operators import SelfSingular, static_rwg_operators
from oracle.static_modes import static_modes

R = 0.15
# on a sphere: int g0 Y_n = R/(2n+1) Y_n -> gamma_perp_n = R/(2n+1);
# -grad_S of that on grad_S Y_n -> gamma_par_n = n(n+1)/((2n+1) R); mult. 2n+1
EX_PERP = np.array([1 / 3] * 3 + [1 / 5] * 5 + [1 / 7] * 7) * R
EX_PAR = np.array([2 / 3] * 3 + [6 / 5] * 5 + [12 / 7] * 7) / R


@pytest.fixture(scope="module")
def sphere2():
    v, t = w.icosphere(R, 2)
    mb = MeshBasis(v, t, w.edge_table(t))
    sing = SelfSingular(mb)
    M, gp, gs = static_modes(mb, 20, 20, sing)
    return mb, sing, M, gp, gs


def test_sphere_eigenvalues_closed_form(sphere2):
    _, _, _, gp, gs = sphere2
    assert np.all(np.diff(gp) <= 1e-12) and np.all(np.diff(gs) >= -1e-12)
    assert np.abs(gp[:15] / EX_PERP - 1).max() < 0.07
    assert np.abs(gs[:15] / EX_PAR - 1).max() < 0.03
    # multiplets: the n=1 and n=2 groups are degenerate on the icosphere
    assert np.ptp(gp[:3]) < 1e-9 * gp[0] and np.ptp(gp[3:8]) < 1e-9 * gp[0]
    assert np.ptp(gs[:3]) < 1e-9 * gs[0] and np.ptp(gs[3:8]) < 1e-9 * gs[0]


def test_sphere_eigenvalue_convergence():
    errs = []
    for sub in (1, 2):
        v, t = w.icosphere(R, sub)
        mb = MeshBasis(v, t, w.edge_table(t))
        _, gp, _ = static_modes(mb, 15, 15)
        errs.append(np.abs(gp / EX_PERP - 1).max())
    assert errs[1] < errs[0] / 2.5          # O(h^2) under 4-to-1 refinement


def test_mode_orthonormality_and_diagonalisation(sphere2):
    mb, sing, M, gp, gs = sphere2
    Gram, S0, Phi0 = static_rwg_operators(mb, sing)
    # the quadrature leaves a tiny asymmetry; the eigenproblems use the
    # symmetric parts
    assert np.abs(S0 - S0.T).max() < 5e-5 * np.abs(S0).max()
    assert np.abs(Phi0 - Phi0.T).max() < 1e-4 * np.abs(Phi0).max()
    S0, Phi0 = 0.5 * (S0 + S0.T), 0.5 * (Phi0 + Phi0.T)
    Np = len(gp)
    Mp, Ms = M[:Np], M[Np:]
    assert np.abs(Mp @ Gram @ Mp.T - np.eye(Np)).max() < 1e-10
    assert np.abs(Ms @ Gram @ Ms.T - np.eye(len(gs))).max() < 1e-10
    assert np.abs(Mp @ S0 @ Mp.T - np.diag(gp)).max() < 1e-10 * gp[0]
    assert np.abs(Ms @ Phi0 @ Ms.T - np.diag(gs)).max() < 1e-10 * gs[-1]
    # transverse modes are divergence free
    D = mb.rwg_divergence()
    assert np.abs(Mp @ D).max() < 1e-9 * np.abs(Ms @ D).max()
    # sign convention: largest-magnitude RWG coefficient positive
    idx = np.argmax(np.abs(M), axis=1)
    assert np.all(M[np.arange(len(M)), idx] > 0)
