"""Target-to-center association (Sec. 2.2.2) by the library's area query, against brute force:
every target compared with every center. Host only."""
import numpy as np
import pytest

import gq_inputs as gi
from paper_1801_04070_amd import GQError, associate_targets


def _brute(ctr, r, tgt, slack, far):
    out = np.full((len(tgt), 2), -1, np.int32)
    gaps = 0
    for t, x in enumerate(tgt):
        rho = np.hypot(*(x - ctr).T) / r
        c = int(np.argmin(rho))  # first index among ties
        if rho[c] <= 1 + slack:
            out[t, 0] = c
        elif rho[c] < far:
            gaps += 1
    return out, gaps


def _targets(g, rng, n_near=3000, n_box=2000):
    # points pushed off the curve along the normal by up to two center radii, and points anywhere
    # in the bounding box
    i = rng.integers(0, g.n_src, n_near)
    r = g.ctr_r[2 * i]
    near = g.src_xy[i] + rng.uniform(-2.2, 2.2, n_near)[:, None] * r[:, None] * g.src_nrm[i]
    lo, hi = g.src_xy.min(0) - 1.0, g.src_xy.max(0) + 1.0
    return np.concatenate([near, rng.uniform(lo, hi, (n_box, 2))])


@pytest.mark.parametrize("slack,far", [(0.2, 3.0), (0.0, 2.0), (0.5, 8.0)])
def test_association_matches_brute_force(slack, far):
    g = gi.random_stars(n_curves=3, panels_per_curve=40, seed=4, box=8.0)
    rng = np.random.default_rng(int(10 * slack + far))
    tgt = _targets(g, rng)
    got, gaps = associate_targets(g.ctr_xy, g.ctr_r, tgt, slack=slack, far_factor=far)
    ref, ref_gaps = _brute(g.ctr_xy, g.ctr_r, tgt, slack, far)
    np.testing.assert_array_equal(got, ref)
    assert gaps == ref_gaps
    assert (got[:, 0] >= 0).sum() > 1000 and (got[:, 0] < 0).sum() > 500


def test_association_on_surface_nodes_and_errors():
    """A node is one radius from each of its two centers (its own pair), so with a slack of rounding size each
    surface node is a QBX target of one of them; bad arguments are refused."""
    g = gi.starfish_c1()
    got, gaps = associate_targets(g.ctr_xy, g.ctr_r, g.src_xy, slack=1e-9, far_factor=3.0)
    assert (got[:, 0] >= 0).all() and (got[:, 1] == -1).all()
    rho = np.hypot(*(g.src_xy - g.ctr_xy[got[:, 0]]).T) / g.ctr_r[got[:, 0]]
    assert rho.max() <= 1.0 + 1e-12
    with pytest.raises(GQError):
        associate_targets(g.ctr_xy, g.ctr_r, g.src_xy, slack=-0.1)
    with pytest.raises(GQError):
        associate_targets(g.ctr_xy, g.ctr_r, g.src_xy, slack=0.2, far_factor=1.1)
    bad = g.ctr_r.copy()
    bad[3] = 0.0
    with pytest.raises(GQError):
        associate_targets(g.ctr_xy, bad, g.src_xy)
