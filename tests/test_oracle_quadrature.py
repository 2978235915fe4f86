"""Pins of the oracle's quadrature primitives against closed forms and brute
force (the 7-point degree-5 rule; the closed-form potential integrals)."""
import math

import numpy as np
import pytest

from oracle.quadrature import (brute_force_integrals, potential_integrals,
                               subdivided_rule, triangle_rule)


@pytest.mark.parametrize("rule", ["plain", "sub2"])
def test_rule_exact_to_degree5(rule):
    bary, w = triangle_rule() if rule == "plain" else subdivided_rule(2)
    assert abs(w.sum() - 1.0) < 1e-14
    # unit right triangle (0,0),(1,0),(0,1): int x^a y^b = a! b! / (a+b+2)!
    xy = bary[:, 1:3]
    for a in range(6):
        for b in range(6 - a):
            num = 0.5 * np.sum(w * xy[:, 0] ** a * xy[:, 1] ** b)
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(num - exact) < 1e-14, (a, b)
    # degree 6 is NOT integrated exactly by the plain rule (sanity of the pin)
    if rule == "plain":
        num = 0.5 * np.sum(w * xy[:, 0] ** 6)
        assert abs(num - math.factorial(6) / math.factorial(8)) > 1e-6


def test_potential_integrals_vs_brute_force():
    rng = np.random.default_rng(3)
    tri = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.3, 0.9, 0.2]])
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    pts = np.vstack([rng.normal(size=(6, 3)) * 0.8,
                     tri.mean(0) + 0.05 * n,            # close above the face
                     tri.mean(0) - 0.2 * n + 0.3 * (tri[1] - tri[0]),
                     [[3.0, -2.0, 1.0]]])
    I0, J, g = potential_integrals(pts, tri)
    bI0, bJ, bg = brute_force_integrals(pts, tri, levels=7)
    assert np.abs(I0 - bI0).max() < 1e-9
    assert np.abs(J - bJ).max() < 1e-9
    assert np.abs(g - bg).max() < 1e-7


def test_potential_on_plane_principal_value_and_edge_line():
    tri = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    # inside the face: normal part of the gradient is the principal value 0
    _, _, g = potential_integrals([[0.25, 0.25, 0.0]], tri)
    assert abs(g[0, 2]) < 1e-14
    # on the extension of an edge line, outside the triangle (in-plane):
    # compare with brute force of a point slightly off the line
    I0, J, _ = potential_integrals([[2.0, 0.0, 0.0]], tri)
    bI0, bJ, _ = brute_force_integrals([[2.0, 0.0, 0.0]], tri, levels=6)
    assert abs(I0[0] - bI0[0]) < 1e-10 and np.abs(J - bJ).max() < 1e-10
    # I0 of the unit right triangle seen from its right-angle vertex:
    # int_0^{pi/2} int_0^{1/(cos t + sin t)} dr dt = sqrt(2) asinh(1)
    I0v, _, _ = potential_integrals([[0.0, 0.0, 0.0]], tri)
    assert abs(I0v[0] - math.sqrt(2.0) * math.asinh(1.0)) < 1e-12
