"""GPU parity of the per-center features and the order choice (include/gigaqbx_mlp.h).

Features: the library's tree-walk kernel against the brute-force FP64 reference (every center
against every source), elementwise at FP32 output rounding. Order choice: a network whose
outputs are constants (zero last-layer weights) makes the predicted errors known exactly, so the
chosen order of every center is fixed by the rule itself.
"""
import numpy as np
import pytest

import gq_inputs as gi
from oracle import features as of

pytestmark = pytest.mark.gpu


def _fmm(geom, p_qbx=16, **kw):
    from paper_1801_04070_amd import QBXFMM
    f = QBXFMM(0)
    f.set_geometry_from(geom)
    f.build(p_qbx=p_qbx, p_fmm=kw.pop("p_fmm", 20), **kw)
    return f


@pytest.mark.parametrize("name", ["wavy_2x2", "stars", "deep_tree"])
def test_features_match_bruteforce(name):
    from paper_1801_04070_amd.learned import center_features
    if name == "wavy_2x2":
        g = gi.wavy_lattice(nx=2, ny=2, panels_per_curve=48, gap_in_radii=3.0)
        kw = {}
    elif name == "stars":
        g = gi.random_stars(n_curves=3, panels_per_curve=40, seed=5, box=8.0)
        kw = {}
    else:
        g = gi.wavy_lattice(nx=2, ny=1, panels_per_curve=64, gap_in_radii=2.5)
        kw = {"n_max": 8}
    f = center_features(_fmm(g, **kw)).cpu().numpy()
    ref = of.center_features(g.src_xy, g.src_nrm, g.src_w, g.ctr_xy, g.ctr_r)
    np.testing.assert_allclose(f, ref, rtol=2e-6, atol=2e-6)


def _constant_net(levels):
    """Network with W3 = 0 and b3 = levels: every center predicts y = levels."""
    from paper_1801_04070_amd.mlp import MLP
    net = MLP(8, 16, len(levels), seed=1)
    p = net.get_params()
    p[-(16 * len(levels) + len(levels)):] = 0.0
    p[-len(levels):] = levels
    net.set_params(p)
    return net


def _predict(fmm, net, cand, scale, shift, tol, margin, apply=0):
    import torch
    from paper_1801_04070_amd import _ptr
    out = torch.empty(fmm.n_ctr, dtype=torch.int32, device="cuda:0")
    c = np.asarray(cand, np.int32)
    m = np.broadcast_to(np.asarray(margin, np.float64), (len(c),)).copy()
    st = fmm._L.gq_orders_predict(fmm._h, net._h, c.ctypes.data, len(c), scale, shift, tol,
                                  m.ctypes.data, _ptr(out), apply)
    return st, out.cpu().numpy()


def test_order_choice_rule():
    g = gi.starfish_c1()
    fmm = _fmm(g)
    cand = (4, 6, 8, 10, 12, 16)
    # predicted log10 errors 2 y - 10: -2, -4, -6, -8, -10, -14
    net = _constant_net([4.0, 3.0, 2.0, 1.0, 0.0, -2.0])
    for tol, margin, want in [(-6.0, 0.0, 8), (-6.0, 0.5, 10), (-9.0, 1.0, 12), (-3.0, 0.0, 6),
                              (-20.0, 0.0, 16), (0.0, 0.0, 4)]:
        st, o = _predict(fmm, net, cand, 2.0, -10.0, tol, margin)
        assert st == 0 and np.all(o == want), (tol, margin, o[:4])
    # per-candidate margins: 8 and 10 need a wider margin than 12 -> 12 at tolerance -9
    st, o = _predict(fmm, net, cand, 2.0, -10.0, -9.0, [0.0, 0.0, 4.0, 2.0, 0.5, 0.0])
    assert st == 0 and np.all(o == 12)
    # non-finite predictions fall back to the largest candidate
    net_nan = _constant_net([float("nan")] * 6)
    st, o = _predict(fmm, net_nan, cand, 2.0, -10.0, -6.0, 0.0)
    assert st == 0 and np.all(o == 16)
    # apply: box orders follow (every center at 10 -> every box with centers at 10)
    st, o = _predict(fmm, net, cand, 2.0, -10.0, -7.0, 0.5, apply=1)
    assert st == 0 and np.all(o == 10)
    from paper_1801_04070_amd import _lib
    rng = fmm.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE)
    owns = rng[:, 1] > rng[:, 0]
    assert np.all(fmm.box_orders()[owns] == 10)


def test_order_choice_errors():
    import torch
    from paper_1801_04070_amd import GQ_S
    g = gi.starfish_c1()
    fmm = _fmm(g, p_qbx=12)
    net = _constant_net([0.0] * 6)
    # candidate above p_qbx, unsorted candidates, wrong output count: GQ_EINVAL (-1)
    assert _predict(fmm, net, (4, 6, 8, 10, 12, 16), 1.0, 0.0, -6.0, 0.0)[0] == -1
    assert _predict(fmm, net, (6, 4, 8, 10, 11, 12), 1.0, 0.0, -6.0, 0.0)[0] == -1
    assert _predict(fmm, _constant_net([0.0] * 5), (4, 6, 8, 10, 12, 12), 1.0, 0.0, -6.0,
                    0.0)[0] == -1
    assert _predict(fmm, net, (2, 4, 6, 8, 10, 12), 1.0, float("inf"), -6.0, 0.0)[0] == -1
    assert _predict(fmm, net, (2, 4, 6, 8, 10, 12), 1.0, 0.0, -6.0,
                    [0, 0, float("nan"), 0, 0, 0])[0] == -1
    # the context is still usable after the rejected calls
    ones = torch.ones(g.src_w.shape[0], dtype=torch.float64, device="cuda:0")
    assert torch.isfinite(fmm.eval(GQ_S, ones)).all()
