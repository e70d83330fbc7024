"""Pins of the brute-force feature reference (oracle/features.py) by closed forms on circles.

Centers sit at distance r from their node along the normal, r = half the panel arclength. On a
circle much larger than r the curve is flat to O(r / R): the disk of radius 2 r (4 r) around a
center cuts an arc of 2 sqrt(3) r (2 sqrt(15) r) from it; the nearest node is the center's own,
at distance r; normals agree (coherence 1, no opposite sheet); (y - c).n = +r on the interior
side and -r on the exterior side for every node. Sums of quadrature weights over the nodes in a
disk reproduce an arc length to within about one node spacing (< 0.2 r here).
"""
import math

import numpy as np
import pytest

import gq_inputs as gi
from oracle import features as of


def _big_circle():
    # radius 400 with 12800 panels: panel arclength ~0.196, r ~0.098, r / R ~ 2.5e-4
    c = gi.StarCurve(R=400.0, amp=0.0, arms=1)
    g = gi.discretize([c], 12800)
    sel = np.arange(0, 64)          # a few nodes (both centers each) are enough
    ctr = np.concatenate([2 * sel, 2 * sel + 1])
    return g, ctr


def test_flat_limit_closed_forms():
    g, ctr = _big_circle()
    f = of.center_features(g.src_xy, g.src_nrm, g.src_w, g.ctr_xy[ctr], g.ctr_r[ctr])
    n = len(ctr) // 2
    np.testing.assert_allclose(f[:, 0], 2 * math.sqrt(3) / 4, atol=0.2 / 4)
    np.testing.assert_allclose(f[:, 1], 2 * math.sqrt(15) / 8, atol=0.2 / 8)
    np.testing.assert_allclose(f[:, 2], 1.0, atol=1e-9)
    # 16 nodes per panel of arclength 2 r: r * count / arc = 8
    np.testing.assert_allclose(f[:, 3], 3.0, atol=0.15)
    np.testing.assert_allclose(f[:, 4], 1.0, atol=1e-6)
    np.testing.assert_allclose(f[:, 5], 0.0, atol=5e-3)
    np.testing.assert_allclose(f[:n, 6], 1.0, atol=5e-3)     # interior centers
    np.testing.assert_allclose(f[n:, 6], -1.0, atol=5e-3)    # exterior centers
    np.testing.assert_array_equal(f[:, 7], 1.0)


@pytest.mark.parametrize("gap_in_r", [2.5, 3.0, 3.5])
def test_opposite_sheet_distance_between_facing_circles(gap_in_r):
    # two large circles whose facing points are gap_in_r * r apart along the x axis
    n_pan = 12800
    R = 400.0
    r = 0.5 * 2 * math.pi * R / n_pan
    gap = gap_in_r * r
    a = gi.StarCurve(cx=0.0, cy=0.0, R=R, amp=0.0, arms=1)
    b = gi.StarCurve(cx=2 * R + gap, cy=0.0, R=R, amp=0.0, arms=1)
    g = gi.discretize([a, b], n_pan)
    # exterior center of circle a nearest to the x axis on its right-hand side
    i = int(np.argmin(np.hypot(g.src_xy[:n_pan * 16, 0] - R, g.src_xy[:n_pan * 16, 1])))
    c = 2 * i + 1
    f = of.center_features(g.src_xy, g.src_nrm, g.src_w, g.ctr_xy[[c]], g.ctr_r[[c]])[0]
    # the facing node of b nearest the axis lies within one node spacing (< 0.2 r) laterally,
    # which changes the distance gap - r by at most (0.2 r)^2 / (2 (gap - r)) < 0.02 r
    assert abs(f[7] - (gap - r) / (4 * r)) < 0.02 / 4 + 1e-3
    # the interior center of the same node sees no opposite sheet within 4 r only if the gap
    # plus r exceeds 4 r
    fi = of.center_features(g.src_xy, g.src_nrm, g.src_w, g.ctr_xy[[c - 1]], g.ctr_r[[c - 1]])[0]
    if gap + r >= 4 * r + 0.2 * r:
        assert fi[7] == 1.0


@pytest.mark.parametrize("side", ["interior", "exterior"])
def test_small_circle_closed_forms(side):
    """All eight features on a curved geometry: a circle of radius R = 3 r around the origin,
    densely sampled (trapezoid weights, exact arclength sums up to one node at each end of an
    arc), and a center of radius r at distance r inside or outside the curve on the x axis.
    With y = R e^(i phi), n = e^(i phi) and c = (R -+ r, 0): the disk of radius k r about c cuts
    the arc |phi| < phi_k with cos phi_k = (R^2 + |c|^2 - k^2 r^2) / (2 R |c|); the normals have
    mean direction sin(phi_4)/phi_4; o = (y - c).n / r = (R - |c| cos phi) / r has arclength mean
    (R - |c| S1) / r and second moment (R^2 - 2 R |c| S1 + |c|^2 S2) / r^2 with S1 =
    sin(phi_4)/phi_4 and S2 = 1/2 + sin(2 phi_4)/(4 phi_4); the sources with normals opposite to
    the nearest one (|phi| > pi/2) lie inside the disk of radius 4 r only for the interior
    center, the nearest of them at distance sqrt(R^2 + |c|^2); the node count in that disk follows
    from the node map."""
    r, R, N, a = 1.0, 3.0, 200000, 0.8
    # nodes phi = u + a sin u for equispaced u (sparse near phi = 0, dense near phi = pi) with
    # weights R dphi/du du, so unweighted sums differ from the arclength integrals
    du = 2 * math.pi / N
    u = du * (np.arange(N) - N // 2)
    phi = u + a * np.sin(u)
    xy = R * np.stack([np.cos(phi), np.sin(phi)], 1)
    nrm = np.stack([np.cos(phi), np.sin(phi)], 1)
    w = R * (1 + a * np.cos(u)) * du
    cx = R - r if side == "interior" else R + r
    f = of.center_features(xy, nrm, w, np.array([[cx, 0.0]]), np.array([r]))[0]

    def half_angle(k):
        return math.acos((R * R + cx * cx - (k * r) ** 2) / (2 * R * cx))

    def u_of(ph):  # inverse of phi(u) on [0, pi] by bisection
        lo, hi = 0.0, math.pi
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if mid + a * math.sin(mid) < ph else (lo, mid)
        return lo

    p2, p4 = half_angle(2), half_angle(4)
    dphi = (1 + a) * du  # the widest node spacing
    count4 = 2 * math.floor(u_of(p4) / du) + 1
    s1 = math.sin(p4) / p4
    s2 = 0.5 + math.sin(2 * p4) / (4 * p4)
    mean = (R - cx * s1) / r
    var = (R * R - 2 * R * cx * s1 + cx * cx * s2) / r ** 2 - mean ** 2
    tol = 4 * dphi / p4  # one node at each end of the arc, relative
    assert f[0] == pytest.approx(2 * R * p2 / (4 * r), rel=4 * dphi / p2)
    assert f[1] == pytest.approx(2 * R * p4 / (8 * r), rel=tol)
    assert f[2] == pytest.approx(1.0, abs=1e-12)
    assert f[3] == pytest.approx(math.log2(r * count4 / (2 * R * p4)), abs=2 * tol)
    assert f[4] == pytest.approx(s1, abs=tol)
    assert f[5] == pytest.approx(math.sqrt(var), rel=10 * tol)
    assert f[6] == pytest.approx(mean, abs=10 * tol)
    if side == "interior":
        assert p4 > math.pi / 2
        assert f[7] == pytest.approx(math.sqrt(R * R + cx * cx) / (4 * r), abs=R * dphi)
    else:
        assert p4 < math.pi / 2
        assert f[7] == 1.0
    # the spread is far from 0 and from its square here, and the nodes are not equispaced, so a
    # dropped square root or a mean or variance without the weights cannot pass
    assert var > 0.05 and abs(math.sqrt(var) - var) > 0.05
    d = xy - np.array([cx, 0.0])
    inside = np.hypot(d[:, 0], d[:, 1]) < 4 * r
    o = (d * nrm).sum(1)[inside] / r
    assert abs(o.mean() - mean) > 30 * tol and abs(o.std() - math.sqrt(var)) > 30 * tol * math.sqrt(var)
