"""Pins of the dense PMCHWT oracle: brute force on a tiny mesh, the Mie
series (cross-section, far amplitudes and the near field), power balance,
reciprocity, mirror symmetry, and Love's equivalence theorem for the
near-field quadrature."""
import math

import numpy as np
import pytest

import workloads as w
from oracle.basis import MeshBasis
from oracle.fields import (extinction_cross_section, far_amplitude, near_field,
                           scattering_cross_section)
from oracle.mie import mie_cross_sections, mie_near_field, mie_s1_s2
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


# ---------------------------------------------------------------- near field


def test_mie_near_field_far_limit_is_s1_s2():
    """The VSWF near-field sum of the Mie series, taken far out, is the
    textbook far amplitude: r exp(jkr) E_theta -> conj(j S2 / k) at phi = 0
    and |E_phi| -> |S1| / k at phi = 90 deg (exp(+jwt) is the complex
    conjugate of the exp(-iwt) series for a real index)."""
    a, m, R = 0.15, 2.0, 400.0
    th = np.array([0.4, 1.1, 2.3])
    s1, s2 = mie_s1_s2(a, K0, m, th)
    p0 = R * np.stack([np.sin(th), 0 * th, np.cos(th)], -1)
    E0 = mie_near_field(a, K0, m, p0) * R * np.exp(1j * K0 * R)
    thh = np.stack([np.cos(th), 0 * th, -np.sin(th)], -1)
    Et = np.einsum("dc,dc->d", E0, thh)
    assert np.abs(Et - np.conj(1j * s2 / K0)).max() < 5e-3 * np.abs(s2 / K0).max()
    p1 = R * np.stack([0 * th, np.sin(th), np.cos(th)], -1)
    E1 = mie_near_field(a, K0, m, p1) * R * np.exp(1j * K0 * R)
    assert np.abs(np.abs(E1[:, 0]) - np.abs(s1) / K0).max() < 5e-3 * np.abs(s1 / K0).max()


def test_near_field_far_zone_limit(single_sphere):
    """r exp(jkr) E_s(r rhat) of the oracle's near-field quadrature tends to
    its far amplitude (itself pinned by Mie above), with the error falling
    like 1/r."""
    prob, x, _ = single_sphere
    rh = np.array([[0.3, 0.2, 0.93], [-0.5, 0.6, -0.2]])
    rh /= np.linalg.norm(rh, axis=1)[:, None]
    F = far_amplitude(prob, x, rh)
    errs = []
    for R in (100.0, 200.0, 400.0):
        E = near_field(prob, x, R * rh) * R * np.exp(1j * K0 * R)
        errs.append(np.linalg.norm(E - F) / np.linalg.norm(F))
    assert errs[0] < 5e-3
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


def test_near_field_vs_mie_series(single_sphere):
    """Scattered near field of the single-sphere solution at points 0.1 to 1
    wavelength outside the surface against the Mie VSWF sum (Sec. V.A's
    check, here in the near zone), at the volume-equivalent radius."""
    prob, x, req = single_sphere
    rng = np.random.default_rng(3)
    for rr in (0.25, 0.4, 0.7, 1.15):
        d = rng.normal(size=(16, 3))
        pts = rr * d / np.linalg.norm(d, axis=1)[:, None]
        E = near_field(prob, x, pts)
        Em = mie_near_field(req, K0, 2.0, pts)
        assert np.linalg.norm(E - Em) / np.linalg.norm(Em) < 5e-3, rr


def _dipole_fields(pts, p, k=K0):
    """Closed-form fields of a point current element p at the origin
    (exp(+jwt), zeta = 1): E = -jk (I + grad grad / k^2) g p, written with
    the textbook dyadic coefficients; H = grad g x p."""
    R = np.linalg.norm(pts, axis=1)
    rh = pts / R[:, None]
    kr = k * R
    g = np.exp(-1j * kr) / (4 * np.pi * R)
    rp = rh @ p
    trans = p[None, :] - rh * rp[:, None]
    a = 1 - 1 / kr ** 2 - 1j / kr
    b = 2 / kr ** 2 + 2j / kr
    E = -1j * k * g[:, None] * (a[:, None] * trans + b[:, None] * rh * rp[:, None])
    H = (-(1 + 1j * kr) / R * g)[:, None] * np.cross(rh, p[None, :])
    return E, H


def test_near_field_love_equivalence():
    """Love's equivalence theorem: the currents n x H and E x n of a source
    inside a closed surface radiate the source's own field outside it and a
    null field inside.  A point current element at the centre of the C1
    sphere, its surface currents projected onto the 15 + 15 static modes
    (L2 projection; the element's tangential fields are degree-1 harmonics,
    which the sphere's first multiplets span up to mesh error): the
    oracle's near-field quadrature reproduces the closed form outside and
    nearly cancels inside.  Exercises both current operators (L with its
    scalar-potential term, and K) in the near zone, independently of the
    PMCHWT solve."""
    v, t = w.icosphere(0.15, 2)
    pc = ParticleClass(v, t, w.edge_table(t), 15, 15, 4.0)
    prob = DenseProblem([pc], np.zeros((1, 3)), [0])
    bs, mb = pc.bs, pc.mb
    nrm = np.repeat(mb.normal, mb.nq, axis=0)
    p = np.array([0.3, -0.2, 1.0])
    E, H = _dipole_fields(bs.X, p)
    Psi = np.stack(bs.Psi, -1)                                   # [N][Q][3]
    G = np.einsum("nqc,mqc,q->nm", Psi, Psi, bs.W)

    def proj(j):
        return np.linalg.solve(G, np.einsum("nqc,qc,q->n", Psi, j, bs.W))

    x = np.concatenate([proj(np.cross(nrm, H)), proj(np.cross(E, nrm))])[None]
    rng = np.random.default_rng(4)
    d = rng.normal(size=(24, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    for rr in (0.22, 0.4, 1.0):
        Ed, _ = _dipole_fields(rr * d, p)
        assert np.linalg.norm(near_field(prob, x, rr * d) - Ed) / np.linalg.norm(Ed) < 2e-2, rr
    for rr in (0.05, 0.08):
        Ed, _ = _dipole_fields(rr * d, p)
        assert np.linalg.norm(near_field(prob, x, rr * d)) / np.linalg.norm(Ed) < 5e-3, rr


def test_sphere_in_background_medium_vs_mie():
    """A sphere of eps+ = 4 in a background of eps- = 1.69 (Sec. II's
    particles in a background medium): the Mie series with the relative
    index sqrt(eps+ / eps-) and the background wavenumber k0 sqrt(eps-)
    gives the cross-section and the far amplitudes; the lossless power
    balance holds as in vacuum."""
    v, t = w.icosphere(0.15, 2)
    pc = ParticleClass(v, t, w.edge_table(t), 15, 15, 4.0)
    eb = 1.69
    prob = DenseProblem([pc], np.zeros((1, 3)), [0], eps_bg=eb)
    x = solve_dense(prob, prob.rhs([0, 0, 1], [1, 0, 0]))
    req = (3 * w.check_closed_mesh(v, t)["volume"] / (4 * np.pi)) ** (1 / 3)
    k, m = K0 * math.sqrt(eb), math.sqrt(4.0 / eb)
    ms, _ = mie_cross_sections(req, k, m)
    cs = scattering_cross_section(prob, x)
    assert abs(cs / ms - 1) < 0.01
    th = np.linspace(0.1, np.pi - 0.1, 9)
    Fe = far_amplitude(prob, x, np.stack([np.sin(th), 0 * th, np.cos(th)], -1))
    s1, s2 = mie_s1_s2(req, k, m, th)
    assert np.abs(np.linalg.norm(Fe, axis=1) - np.abs(s2) / k).max() < 0.01 * np.abs(s2 / k).max()
    ce = extinction_cross_section(prob, x, [0, 0, 1], np.array([1, 0, 0], complex))
    assert abs(ce / cs - 1) < 1e-3
    pts = np.array([[0.3, 0.1, 0.2], [-0.4, 0.5, -0.1], [0.0, 0.0, 0.8]])
    En = near_field(prob, x, pts)
    Em = mie_near_field(req, k, m, pts)
    assert np.linalg.norm(En - Em) / np.linalg.norm(Em) < 1e-2
