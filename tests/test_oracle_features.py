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
