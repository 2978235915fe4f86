"""Pins of the dense PMCHWT oracle: brute force on a tiny mesh, the Mie
series, power balance, reciprocity and mirror symmetry."""
import math

import numpy as np
import pytest

import workloads as w
from oracle.basis import MeshBasis
from oracle.fields import (extinction_cross_section, far_amplitude,
                           scattering_cross_section)
from oracle.mie import mie_cross_sections, mie_s1_s2
from oracle.operators import SampledBasis, direct_TK
from oracle.pmchwt import DenseProblem, ParticleClass, solve_dense
from oracle.quadrature import triangle_rule

K0 = 2 * math.pi


def _rwg_value(verts, tris, edges, e, t, r):
    """RWG f_e at point r of triangle t, from its definition."""
    v0, v1, tp, tm = edges[e]
    l = np.linalg.norm(verts[v1] - verts[v0])
    if t not in (tp, tm):
        return np.zeros(3)
    free = [x for x in tris[t] if x not in (v0, v1)][0]
    a = np.cross(verts[tris[t][1]] - verts[tris[t][0]], verts[tris[t][2]] - verts[tris[t][0]])
    A = 0.5 * np.linalg.norm(a)
    s = 1.0 if t == tp else -1.0
    return s * l / (2 * A) * (r - verts[free])


def _rwg_div(verts, tris, edges, e, t):
    v0, v1, tp, tm = edges[e]
    l = np.linalg.norm(verts[v1] - verts[v0])
    if t not in (tp, tm):
        return 0.0
    a = np.cross(verts[tris[t][1]] - verts[tris[t][0]], verts[tris[t][2]] - verts[tris[t][0]])
    A = 0.5 * np.linalg.norm(a)
    return (l / A) if t == tp else -(l / A)


def test_pair_block_brute_force_tiny_mesh():
    """T and K between two icosahedra (20 triangles) for 3 random
    combinations of RWG functions, by explicit loops over triangle pairs and
    quadrature points, versus the vectorised oracle."""
    v, t = w.icosphere(0.2, 0)
    e = w.edge_table(t)
    rng = np.random.default_rng(5)
    C = rng.normal(size=(3, len(e)))
    off = np.array([0.7, -0.4, 0.1])
    bary, wq = triangle_rule()
    k = K0
    pts, wts, vals, divs = [], [], [], []
    for tt, tri in enumerate(t):
        tv = v[tri]
        A = 0.5 * np.linalg.norm(np.cross(tv[1] - tv[0], tv[2] - tv[0]))
        for q in range(7):
            r = bary[q] @ tv
            pts.append(r)
            wts.append(A * wq[q])
            vals.append([sum(C[m, ee] * _rwg_value(v, t, e, ee, tt, r) for ee in range(len(e))) for m in range(3)])
            divs.append([sum(C[m, ee] * _rwg_div(v, t, e, ee, tt) for ee in range(len(e))) for m in range(3)])
    pts, wts, vals, divs = map(np.array, (pts, wts, vals, divs))
    T = np.zeros((3, 3), complex)
    K = np.zeros((3, 3), complex)
    for a in range(len(pts)):
        for b in range(len(pts)):
            Rv = pts[a] - (pts[b] + off)
            R = np.linalg.norm(Rv)
            g = np.exp(-1j * k * R) / (4 * np.pi * R)
            grad = -Rv * (1 + 1j * k * R) * np.exp(-1j * k * R) / (4 * np.pi * R ** 3)
            ww = wts[a] * wts[b]
            for m in range(3):
                for n in range(3):
                    T[m, n] += ww * (-1j * k * (vals[a, m] @ vals[b, n]) * g
                                     + (1j / k) * divs[a, m] * divs[b, n] * g)
                    K[m, n] += ww * (vals[a, m] @ np.cross(vals[b, n], grad))
    mb = MeshBasis(v, t, e)
    bs = SampledBasis(mb, C)
    To, Ko = direct_TK(bs, bs, off, k)
    assert np.abs(To - T).max() < 1e-12 * np.abs(T).max()
    assert np.abs(Ko - K).max() < 1e-12 * np.abs(K).max()


@pytest.fixture(scope="module")
def single_sphere():
    v, t = w.icosphere(0.15, 2)
    pc = ParticleClass(v, t, w.edge_table(t), 15, 15, 4.0)
    prob = DenseProblem([pc], np.zeros((1, 3)), [0])
    x = solve_dense(prob, prob.rhs([0, 0, 1], [1, 0, 0]))
    vol = w.check_closed_mesh(v, t)["volume"]
    return prob, x, (3 * vol / (4 * np.pi)) ** (1 / 3)


def test_single_sphere_vs_mie(single_sphere):
    prob, x, req = single_sphere
    m = math.sqrt(4.0)
    cs = scattering_cross_section(prob, x)
    ms, me = mie_cross_sections(req, K0, m)
    assert abs(cs / ms - 1) < 0.01           # paper's level is 0.02 (Sec. V.A)
    th = np.linspace(0.1, np.pi - 0.1, 11)
    Fe = far_amplitude(prob, x, np.stack([np.sin(th), 0 * th, np.cos(th)], -1))   # E-plane
    Fh = far_amplitude(prob, x, np.stack([0 * th, np.sin(th), np.cos(th)], -1))   # H-plane
    s1, s2 = mie_s1_s2(req, K0, m, th)
    assert np.abs(np.linalg.norm(Fe, axis=1) - np.abs(s2) / K0).max() < 0.01 * np.abs(s2 / K0).max()
    assert np.abs(np.linalg.norm(Fh, axis=1) - np.abs(s1) / K0).max() < 0.01 * np.abs(s1 / K0).max()
    # cross-polarised far field vanishes in the principal planes
    assert np.abs(Fe[:, 1]).max() < 1e-6 * np.abs(Fe).max()


def test_power_balance_lossless(single_sphere):
    prob, x, _ = single_sphere
    cs = scattering_cross_section(prob, x)
    ce = extinction_cross_section(prob, x, [0, 0, 1], np.array([1, 0, 0], complex))
    assert abs(ce / cs - 1) < 1e-3


def test_absorbing_sphere_extinction_exceeds_scattering():
    v, t = w.icosphere(0.15, 1)
    pc = ParticleClass(v, t, w.edge_table(t), 10, 10, 4.0 - 1.0j)   # loss for exp(+jwt)
    prob = DenseProblem([pc], np.zeros((1, 3)), [0])
    x = solve_dense(prob, prob.rhs([0, 0, 1], [1, 0, 0]))
    cs = scattering_cross_section(prob, x)
    ce = extinction_cross_section(prob, x, [0, 0, 1], np.array([1, 0, 0], complex))
    assert ce > 1.05 * cs > 0


@pytest.fixture(scope="module")
def array2x2():
    v, t = w.icosphere(0.15, 1)
    pc = ParticleClass(v, t, w.edge_table(t), 8, 8, 4.0)
    prob = DenseProblem([pc], w.lattice(2, 2, 0.5), np.zeros(4, int))
    return prob, pc


def test_reciprocity(array2x2):
    prob, pc = array2x2
    Z = prob.dense()
    N = pc.n_modes
    D = np.diag(np.tile(np.r_[np.ones(N), -np.ones(N)], 4))
    A = D @ Z @ D - Z.T
    n = pc.n
    off = np.kron(1 - np.eye(4), np.ones((n, n))).astype(bool)
    assert np.abs(A[off]).max() < 1e-12 * np.abs(Z).max()
    # self block: T parts symmetric to quadrature accuracy, K parts looser
    Zs = Z[:n, :n]
    As = D[:n, :n] @ Zs @ D[:n, :n] - Zs.T
    assert np.abs(As[:N, :N]).max() < 1e-5 * np.abs(Zs).max()
    assert np.abs(As[N:, N:]).max() < 1e-5 * np.abs(Zs).max()
    assert np.abs(As).max() < 5e-3 * np.abs(Zs).max()


def test_array_mirror_symmetry(array2x2):
    """2x2 array (mirror planes x=0.25, y=0.25 through its centre), normal
    incidence: |F(theta, phi)| = |F(theta, -phi)| = |F(theta, pi - phi)|."""
    prob, _ = array2x2
    x = solve_dense(prob, prob.rhs([0, 0, 1], [1, 0, 0]))
    rng = np.random.default_rng(2)
    th, ph = rng.uniform(0.2, 2.9, 8), rng.uniform(0, 2 * np.pi, 8)

    def dirs(t, p):
        return np.stack([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)], -1)

    F0 = np.abs(far_amplitude(prob, x, dirs(th, ph)))
    F1 = np.abs(far_amplitude(prob, x, dirs(th, -ph)))
    F2 = np.abs(far_amplitude(prob, x, dirs(th, np.pi - ph)))
    # components map to +- themselves under the mirrors; compare magnitudes
    assert np.abs(F0 - F1).max() < 1e-9 * F0.max()
    assert np.abs(F0 - F2).max() < 1e-9 * F0.max()
