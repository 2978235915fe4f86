"""Pins of meshes, RWG, loop and star functions."""
import numpy as np
import pytest

import workloads as w
from oracle.basis import MeshBasis


@pytest.fixture(scope="module", params=["sphere", "cylinder"])
def mb(request):
    if request.param == "sphere":
        v, t = w.icosphere(0.15, 2)
    else:
        v, t = w.cylinder(0.3, 0.6)
    return MeshBasis(v, t, w.edge_table(t))


def test_mesh_counts():
    v, t = w.icosphere(0.15, 2)
    c = w.check_closed_mesh(v, t)
    assert (c["V"], c["F"], c["E"], c["euler"]) == (162, 320, 480, 2)
    assert 0 < c["volume"] < 4 / 3 * np.pi * 0.15 ** 3
    v, t = w.cylinder(0.3, 0.6)
    c = w.check_closed_mesh(v, t)
    assert (c["V"], c["F"], c["E"], c["euler"]) == (302, 600, 900, 2)
    assert abs(c["volume"] / (np.pi * 0.15 ** 2 * 0.6) - 1) < 0.05
    # jitter is seeded: same seed, same mesh; another seed differs
    v2, _ = w.cylinder(0.3, 0.6)
    v3, _ = w.cylinder(0.3, 0.6, seed=7)
    assert np.array_equal(v, v2) and not np.allclose(v, v3)


def test_rwg_divergence_and_flux(mb):
    D = mb.rwg_divergence()
    # each RWG carries equal and opposite charge on its two triangles
    assert np.abs(D @ mb.area).max() < 1e-12
    # local-function divergence 2a = l/A matches the RWG divergence
    Hc, Hd = mb.local_values()
    X, W = mb.flat_points()
    div_pts = (mb.P @ Hd).toarray()                       # E x Q
    tri_of = np.arange(len(W)) // mb.nq
    assert np.abs(div_pts - D[:, tri_of]).max() < 1e-9
    # normal flux of f_e across its own edge is 1 (continuity): check at the
    # edge midpoint from both sides
    for e in range(0, mb.nE, max(1, mb.nE // 25)):
        v0, v1, tp, tm = mb.edges[e]
        mid = 0.5 * (mb.verts[v0] + mb.verts[v1])
        pp = mb.verts[[x for x in mb.tris[tp] if x not in (v0, v1)][0]]
        pm = mb.verts[[x for x in mb.tris[tm] if x not in (v0, v1)][0]]
        l = mb.rwg_len[e]
        fp = l / (2 * mb.area[tp]) * (mid - pp)
        fm = -l / (2 * mb.area[tm]) * (mid - pm)
        t_hat = (mb.verts[v1] - mb.verts[v0]) / l
        mp = np.cross(t_hat, mb.normal[tp])
        mm = np.cross(t_hat, mb.normal[tm])
        assert abs(fp @ mp - 1) < 1e-9 and abs(fm @ mm - 1) < 1e-9


def test_loops_divergence_free_and_loop_star_complete(mb):
    L, S = mb.loops(), mb.stars()
    D = mb.rwg_divergence()
    assert np.abs(D.T @ L).max() < 1e-9 * np.abs(D).max()
    assert L.shape[1] == mb.nV - 1 and S.shape[1] == mb.nF - 1
    assert np.linalg.matrix_rank(np.hstack([L, S])) == mb.nE
    # the full sets are rank deficient by exactly one each
    Lfull = np.hstack([L, -L.sum(1, keepdims=True)])
    assert np.linalg.matrix_rank(Lfull) == mb.nV - 1
