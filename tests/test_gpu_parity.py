"""GPU parity: the HIP path (through the C ABI) against the CPU oracle (direct QBX, FP64).

Error measure: max_t |gpu_t - oracle_t| / max_t |oracle_t| over the compared targets.
Tolerances: the FMM error of Theorem 1 is bounded by C A (p_qbx + 1) max(sqrt 2/3, alpha)^(p_fmm+1)
with alpha = (t_f + sqrt 2)/(6 - sqrt 2) = 0.5046 at t_f = 0.9; the paper observes the actual
error about two orders of magnitude below the bound. Gates: 1e-10 at p_fmm = 30, 1e-7 at
p_fmm = 15; direct QBX on the GPU differs from the oracle by summation order only (1e-12).
"""
import copy

import numpy as np
import pytest

import gq_inputs as gi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _ctx(geom, **params):
    from paper_1801_04070_amd import QBXFMM
    q = QBXFMM(device=0)
    q.set_geometry_from(geom)
    stats = q.build(**params)
    return q, stats


def _densities(geom, seed):
    mu = gi.fourier_density(geom, seed=seed)
    mu2 = gi.fourier_density(geom, seed=seed + 1000)
    return mu, mu2


def _run(q, kind, mu, mu2, direct=False):
    out = q.eval(kind, _dev(mu), None if kind != 3 else _dev(mu2), direct=direct)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.fixture(scope="module")
def c1():
    return gi.starfish_c1()


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_direct_qbx_matches_oracle_c1(c1, kind):
    mu, mu2 = _densities(c1, 0)
    q, _ = _ctx(c1, p_qbx=8, p_fmm=15)
    gpu = _run(q, kind, mu, mu2, direct=True)
    ref = oracle.qbx_eval(c1, kind, mu, mu2 if kind == 3 else None, p_qbx=8)
    assert _rel(gpu, ref) < 1e-12


@pytest.mark.parametrize("kind", [1, 2, 3])
@pytest.mark.parametrize("p_fmm,tol", [(15, 1e-7), (30, 1e-10)])
def test_fmm_matches_oracle_c1(c1, kind, p_fmm, tol):
    mu, mu2 = _densities(c1, 0)
    q, _ = _ctx(c1, p_qbx=8, p_fmm=p_fmm)
    gpu = _run(q, kind, mu, mu2)
    ref = oracle.qbx_eval(c1, kind, mu, mu2 if kind == 3 else None, p_qbx=8)
    err = _rel(gpu, ref)
    print(f"C1 kind={kind} p_fmm={p_fmm} rel_err={err:.3e}")
    assert err < tol


@pytest.mark.parametrize("count_mode", [0, 1])
@pytest.mark.parametrize("kind", [1, 2, 3])
def test_fmm_matches_oracle_multi_curve(kind, count_mode):
    # 3 stars x 128 panels x 16 nodes = 6144 sources: several tree levels, suspended centers,
    # all list types; every target compared
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    mu, mu2 = _densities(g, 3)
    q, stats = _ctx(g, p_qbx=12, p_fmm=30, count_mode=count_mode)
    assert stats["n_list3_far"] > 0 and stats["n_list4_far"] > 0 and stats["n_list2"] > 0
    gpu = _run(q, kind, mu, mu2)
    ref = oracle.qbx_eval(g, kind, mu, mu2 if kind == 3 else None, p_qbx=12)
    err = _rel(gpu, ref)
    print(f"3 stars kind={kind} count_mode={count_mode} rel_err={err:.3e}")
    assert err < 1e-10


@pytest.mark.parametrize("p_fmm", [40, 63])
def test_fmm_deep_tree_high_order(p_fmm):
    """A deep tree (n_max 8) at high FMM orders: the downward pass shifts locals across many
    levels at once and runs the 3- and 4-tile forms of its matrix-core step."""
    g = gi.random_stars(n_curves=3, panels_per_curve=64, seed=21, box=12.0)
    mu, mu2 = _densities(g, 5)
    q, stats = _ctx(g, p_qbx=12, p_fmm=p_fmm, n_max=8)
    assert stats["n_levels"] >= 9, stats["n_levels"]
    gpu = _run(q, 3, mu, mu2)
    ref = oracle.qbx_eval(g, 3, mu, mu2, p_qbx=12)
    err = _rel(gpu, ref)
    print(f"deep tree levels={stats['n_levels']} p_fmm={p_fmm} rel_err={err:.3e}")
    assert err < 1e-12


def test_fmm_green_identity_c2_sampled():
    """Full-size 131072-source workload: Green's formula S(du/dn) - D(u) vs the oracle at
    sampled targets (the oracle evaluates them one by one) and vs u/2."""
    g = gi.config_geometry("c2")
    sig, tau, u = gi.green_test_field(g, (-5.0, -5.0))
    q, stats = _ctx(g, p_qbx=12, p_fmm=30)
    gpu = _run(q, 3, sig, tau)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(g.n_tgt, 192, replace=False))
    ref = oracle.qbx_eval(g, 3, sig, tau, p_qbx=12, tgt_xy=g.tgt_xy[idx], tgt_ctr=g.tgt_ctr[idx])
    err = _rel(gpu[idx], ref)
    print(f"C2 Green sampled rel_err vs oracle={err:.3e}")
    assert err < 1e-10
    # and the physics: u/2 up to QBX truncation/quadrature error at these orders
    assert np.abs(gpu - u / 2).max() / np.abs(u).max() < 1e-4


@pytest.mark.parametrize("kind", [1, 2])
def test_fmm_c2_sampled(kind):
    g = gi.config_geometry("c2")
    mu, mu2 = _densities(g, 2)
    q, _ = _ctx(g, p_qbx=12, p_fmm=30)
    gpu = _run(q, kind, mu, mu2)
    rng = np.random.default_rng(kind)
    idx = np.sort(rng.choice(g.n_tgt, 128, replace=False))
    ref = oracle.qbx_eval(g, kind, mu, None, p_qbx=12, tgt_xy=g.tgt_xy[idx], tgt_ctr=g.tgt_ctr[idx])
    err = _rel(gpu[idx], ref)
    print(f"C2 kind={kind} sampled rel_err={err:.3e}")
    assert err < 1e-10


def test_multi_density_and_determinism(c1):
    """Four densities in one call are bitwise reproducible and each row matches the oracle; a
    single density sums its direct part at the targets (every center here serves one target)
    while the 4-density call forms coefficient rows, so they agree to rounding."""
    q, _ = _ctx(c1, p_qbx=8, p_fmm=30)
    dens = np.stack([gi.fourier_density(c1, seed=s) for s in range(4)])
    out = q.eval(1, _dev(dens)).cpu().numpy()
    again = q.eval(1, _dev(dens)).cpu().numpy()
    assert np.array_equal(out, again), "evaluation is not bitwise deterministic"
    for j in range(4):
        single = q.eval(1, _dev(dens[j])).cpu().numpy()
        assert np.array_equal(single, q.eval(1, _dev(dens[j])).cpu().numpy())
        assert _rel(single, out[j]) < 1e-13
        ref = oracle.qbx_eval(c1, 1, dens[j], p_qbx=8)
        assert _rel(out[j], ref) < 1e-10


def test_one_sided_targets_and_jump(c1):
    # interior/exterior one-sided limits of D: D_- - D_+ = -mu (jump relation)
    mu, _ = _densities(c1, 5)
    vals = {}
    for side in (-1, 1):
        g = c1.one_sided(side)
        q, _ = _ctx(g, p_qbx=8, p_fmm=30)
        vals[side] = _run(q, 2, mu, None)
        ref = oracle.qbx_eval(g, 2, mu, p_qbx=8)
        assert _rel(vals[side], ref) < 1e-10
    assert np.abs((vals[-1] - vals[1]) + mu).max() < 1e-4 * np.abs(mu).max()


def test_small_and_ragged_geometries():
    # a single tiny panel set (root is a leaf), and a geometry whose node count is not a
    # multiple of anything convenient
    for g in (gi.unit_circle(4), gi.discretize([gi.StarCurve(amp=0.2, arms=3)], 37)):
        mu, _ = _densities(g, 7)
        q, _ = _ctx(g, p_qbx=8, p_fmm=30)
        gpu = _run(q, 1, mu, None)
        ref = oracle.qbx_eval(g, 1, mu, p_qbx=8)
        assert _rel(gpu, ref) < 1e-10


def test_empty_batch_and_errors(c1):
    from paper_1801_04070_amd import GQError, _lib
    q, _ = _ctx(c1, p_qbx=8, p_fmm=15)
    dens = torch.zeros((0, c1.n_src), dtype=torch.float64, device="cuda:0")
    out = q.eval(1, dens)
    assert out.shape == (0, c1.n_tgt)
    with pytest.raises(GQError) as e:
        q.eval(3, _dev(np.ones(c1.n_src)))  # S - D needs two densities
    assert e.value.status == _lib.GQ_EINVAL
    with pytest.raises(GQError) as e:
        _ctx(c1, p_qbx=7, p_fmm=15)  # no compiled kernel for this order
    assert e.value.status == _lib.GQ_EUNSUP


def test_density_batches_match_single_evaluations(c1):
    """134 densities (two launches of the batch dimension: 128, then 6), padded row strides, S - D
    kind: each row equals the single-density evaluation to rounding (a batch of 8 or more slots
    runs M2L and the Stage 7 gather as GEMMs over the slots, which sum in another order; a
    single density sums its direct part at the targets, the batches form coefficient rows), the
    batch is bitwise reproducible, and the last row matches the oracle within the gate."""
    q, _ = _ctx(c1, p_qbx=8, p_fmm=30)
    n, pad = 134, 7
    rng = np.random.default_rng(3)
    d1 = torch.zeros((n, c1.n_src + pad), dtype=torch.float64, device="cuda:0")
    d2 = torch.zeros((n, c1.n_src + pad), dtype=torch.float64, device="cuda:0")
    h1 = np.stack([gi.fourier_density(c1, seed=int(s)) for s in rng.integers(0, 10**6, n)])
    h2 = np.stack([gi.fourier_density(c1, seed=int(s)) for s in rng.integers(0, 10**6, n)])
    d1[:, :c1.n_src] = _dev(h1)
    d2[:, :c1.n_src] = _dev(h2)
    out = torch.full((n, c1.n_tgt + pad), np.nan, dtype=torch.float64, device="cuda:0")
    q.eval(3, d1[:, :c1.n_src], d2[:, :c1.n_src], out=out[:, :c1.n_tgt])
    res = out.cpu().numpy()
    assert np.isnan(res[:, c1.n_tgt:]).all(), "wrote outside the output rows"
    for j in (0, 33, 127, 128, 133):
        single = q.eval(3, _dev(h1[j]), _dev(h2[j])).cpu().numpy()
        assert _rel(res[j, :c1.n_tgt], single) < 1e-13
    again = torch.full_like(out, np.nan)
    q.eval(3, d1[:, :c1.n_src], d2[:, :c1.n_src], out=again[:, :c1.n_tgt])
    assert np.array_equal(again.cpu().numpy()[:, :c1.n_tgt], res[:, :c1.n_tgt])
    ref = oracle.qbx_eval(c1, 3, h1[133], h2[133], p_qbx=8)
    assert _rel(res[133, :c1.n_tgt], ref) < 1e-10
    ref = oracle.qbx_eval(c1, 3, h1[100], h2[100], p_qbx=8)
    assert _rel(res[100, :c1.n_tgt], ref) < 1e-10


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_density_groups_match_one_density_per_item(c1, kind):
    """The direct-interaction work items take 1, 2 or 4 densities at a time (shared pair geometry,
    each density's sums in the single-density order): 7 densities, so the last group of 2 and of 4
    is partial. Every group size gives the same rows bitwise; a size of 3 is rejected."""
    from paper_1801_04070_amd import GQError
    n = 7
    rng = np.random.default_rng(11)
    h1 = np.stack([gi.fourier_density(c1, seed=int(s)) for s in rng.integers(0, 10**6, n)])
    h2 = np.stack([gi.fourier_density(c1, seed=int(s)) for s in rng.integers(0, 10**6, n)])
    outs = {}
    for dg in (1, 2, 4):
        q, _ = _ctx(c1, p_qbx=12, p_fmm=30, near_dens_group=dg)
        outs[dg] = q.eval(kind, _dev(h1), _dev(h2) if kind == 3 else None).cpu().numpy()
        q.close()
    assert np.array_equal(outs[1], outs[2]) and np.array_equal(outs[1], outs[4])
    ref = oracle.qbx_eval(c1, kind, h1[n - 1], h2[n - 1] if kind == 3 else None, p_qbx=12)
    assert _rel(outs[4][n - 1], ref) < 1e-10
    with pytest.raises(GQError):
        _ctx(c1, p_qbx=12, p_fmm=30, near_dens_group=3)


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_mixed_precision_c1(c1, kind):
    """FP32 box expansions with power-of-two level scaling at p_fmm = 16 (one density: moments and
    P2L formed in FP64 and stored in FP32, M2L and the Stage 7 gather on the FP32 matrix cores)
    against the FP64 oracle: gate 1e-6."""
    from paper_1801_04070_amd import GQ_MIXED_FP32
    mu, mu2 = _densities(c1, 0)
    q, _ = _ctx(c1, p_qbx=8, p_fmm=16, precision=GQ_MIXED_FP32)
    gpu = _run(q, kind, mu, mu2)
    ref = oracle.qbx_eval(c1, kind, mu, mu2 if kind == 3 else None, p_qbx=8)
    err = _rel(gpu, ref)
    print(f"C1 mixed kind={kind} rel_err={err:.3e}")
    assert err < 1e-6


def test_mixed_and_high_order_c2_sampled():
    """Full-size workload: FP32 expansions at p_fmm = 16 (gate 1e-6) and all-FP64 at p_fmm = 40
    (gate 1e-12) against the oracle at sampled targets."""
    from paper_1801_04070_amd import GQ_MIXED_FP32
    g = gi.config_geometry("c2")
    mu, _ = _densities(g, 4)
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(g.n_tgt, 128, replace=False))
    ref = oracle.qbx_eval(g, 1, mu, None, p_qbx=12, tgt_xy=g.tgt_xy[idx], tgt_ctr=g.tgt_ctr[idx])
    q, _ = _ctx(g, p_qbx=12, p_fmm=16, precision=GQ_MIXED_FP32)
    err32 = _rel(_run(q, 1, mu, None)[idx], ref)
    q, _ = _ctx(g, p_qbx=12, p_fmm=40)
    err64 = _rel(_run(q, 1, mu, None)[idx], ref)
    print(f"C2 mixed p16 rel_err={err32:.3e}  fp64 p40 rel_err={err64:.3e}")
    assert err32 < 1e-6
    assert err64 < 1e-12


@pytest.mark.parametrize("kind", [1, 2])
def test_per_center_orders_match_oracle(kind):
    """Per-center QBX orders: every center runs at the smallest compiled order covering its own
    (the centers of a box regrouped by order); each target's value is the average of its two
    one-sided values at their centers' orders."""
    from paper_1801_04070_amd import _lib
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    mu, _ = _densities(g, 6)
    q, _ = _ctx(g, p_qbx=12, p_fmm=30)
    uniform = _run(q, kind, mu, None)
    orders = np.random.default_rng(0).choice([3, 4, 6, 8, 12], size=g.n_ctr).astype(np.int32)
    q.set_qbx_orders(orders)
    eff = q.center_orders()
    compiled = np.array([4, 6, 8, 10, 12])
    assert np.array_equal(eff, compiled[np.searchsorted(compiled, orders)])
    gpu = _run(q, kind, mu, None)
    ref = np.zeros(g.n_tgt)
    for col in (0, 1):
        cidx = g.tgt_ctr[:, col]
        for p in np.unique(eff[cidx]):
            sel = np.nonzero(eff[cidx] == p)[0]
            tc = np.full((len(sel), 2), -1, np.int32)
            tc[:, 0] = cidx[sel]
            ref[sel] += 0.5 * oracle.qbx_eval(g, kind, mu, p_qbx=int(p), tgt_xy=g.tgt_xy[sel],
                                               tgt_ctr=tc)
    err = _rel(gpu, ref)
    print(f"per-center orders kind={kind} rel_err={err:.3e}")
    assert err < 1e-10
    # the direct path uses the same effective orders
    assert _rel(_run(q, kind, mu, None, direct=True), ref) < 1e-12
    q.set_qbx_orders(None)
    assert np.array_equal(_run(q, kind, mu, None), uniform)


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_point_targets_match_oracle(kind):
    """Conventional (off-surface) targets next to QBX targets in one evaluation: point values
    (direct sum + M2P + L2P) against the oracle's plain sum of point potentials, QBX targets
    against the oracle's QBX."""
    g = gi.random_stars(n_curves=3, panels_per_curve=96, seed=21, box=10.0)
    mu, mu2 = _densities(g, 9)
    rng = np.random.default_rng(kind)
    pts = rng.uniform(g.src_xy.min(0) - 0.5, g.src_xy.max(0) + 0.5, size=(3000, 2))
    d = np.sqrt(((pts[:, None, :] - g.src_xy[None, ::7, :]) ** 2).sum(-1)).min(1)
    pts = pts[d > 1e-2][:2000]
    e = copy.copy(g)
    e.tgt_xy = np.concatenate([g.tgt_xy, pts])
    e.tgt_ctr = np.concatenate([g.tgt_ctr, np.full((len(pts), 2), -1, np.int32)])
    q, stats = _ctx(e, p_qbx=12, p_fmm=30)
    assert stats["n_point_targets"] == len(pts)
    d2 = mu2 if kind == 3 else None
    for direct, tol in ((False, 1e-10), (True, 1e-12)):
        gpu = _run(q, kind, mu, mu2, direct=direct)
        n = g.n_tgt
        ref_pt = oracle.point_potential(g, kind, mu, d2, tgt_xy=pts)
        ref_q = oracle.qbx_eval(g, kind, mu, d2, p_qbx=12)
        e_pt, e_q = _rel(gpu[n:], ref_pt), _rel(gpu[:n], ref_q)
        print(f"point targets kind={kind} direct={direct} rel_err={e_pt:.3e} qbx={e_q:.3e}")
        assert e_pt < tol and e_q < tol


@pytest.mark.parametrize("kind", [1, 2])
def test_point_targets_at_leaf_centers(kind):
    """Conventional targets placed exactly at the centers of sparse leaf boxes: each internal
    center then sits at t = 0 of its box local, where the local-to-center shift takes its plain
    Horner branch. Point values against the oracle's plain sums."""
    from paper_1801_04070_amd import QBXFMM, _lib
    g = gi.random_stars(n_curves=3, panels_per_curve=96, seed=21, box=10.0)
    h = QBXFMM(device=-1)
    h.set_geometry_from(g)
    st = h.build(p_qbx=12, p_fmm=30)
    level = h.tree_array(_lib.GQ_TREE_BOX_LEVEL)
    child = h.tree_array(_lib.GQ_TREE_BOX_CHILD)
    ij = h.tree_array(_lib.GQ_TREE_BOX_IJ)
    src = h.tree_array(_lib.GQ_TREE_BOX_SRC_RANGE)
    nsrc = src[:, 1] - src[:, 0]
    lo, side = st["root_lo"], st["root_side"]
    sz = side / 2.0 ** level  # box centers as the tree forms them
    cen = np.stack([lo[0] + (ij[:, 0] + 0.5) * sz, lo[1] + (ij[:, 1] + 0.5) * sz], 1)
    # inside the sources' bounding box (the root square stays the same) and few sources (the
    # extra particle splits nothing)
    inside = ((cen > g.src_xy.min(0)) & (cen < g.src_xy.max(0))).all(1)
    leaves = np.nonzero((child < 0).all(1) & (nsrc >= 1) & (nsrc <= 16) & (level >= 2)
                        & inside)[0][:40]
    assert len(leaves) >= 10
    pts = cen[leaves]
    h.close()
    e = copy.copy(g)
    e.tgt_xy = np.concatenate([g.tgt_xy, pts])
    e.tgt_ctr = np.concatenate([g.tgt_ctr, np.full((len(pts), 2), -1, np.int32)])
    q, stats = _ctx(e, p_qbx=12, p_fmm=30)
    assert stats["n_point_targets"] == len(pts)
    # the same root and boxes, and every internal center is owned by the leaf it sits on
    assert stats["root_lo"] == lo and stats["root_side"] == side
    assert np.array_equal(q.tree_array(_lib.GQ_TREE_BOX_IJ), ij)
    assert np.array_equal(q.tree_array(_lib.GQ_TREE_BOX_LEVEL), level)
    ctr = q.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE)
    order = q.tree_array(_lib.GQ_TREE_CTR_ORDER)
    for k, b in enumerate(leaves):
        owned = order[ctr[b, 0]:ctr[b, 1]]
        assert g.n_ctr + k in owned, (k, b)
    mu, mu2 = _densities(g, 5)
    gpu = _run(q, kind, mu, None)
    ref_pt = oracle.point_potential(g, kind, mu, None, tgt_xy=pts)
    err = _rel(gpu[g.n_tgt:], ref_pt)
    print(f"points at leaf centers kind={kind} rel_err={err:.3e}")
    assert err < 1e-10
    assert _rel(gpu[:g.n_tgt], oracle.qbx_eval(g, kind, mu, None, p_qbx=12)) < 1e-10


@pytest.mark.parametrize("kind", [1, 3, 4])
def test_graph_replays_match_eager(c1, kind):
    """A captured evaluation replayed several times, with other eager evaluations (sharing the
    workspace) and host synchronisations between replays, reproduces the eager result exactly;
    the graph goes stale when the buffers change, and a capture of more than one density batch
    is refused."""
    from paper_1801_04070_amd import GQError, _lib
    mu, mu2 = _densities(c1, 4)
    q, _ = _ctx(c1, p_qbx=8, p_fmm=20)
    d1 = _dev(np.stack([mu, 2 * mu]))
    d2 = _dev(np.stack([mu2, -mu2])) if kind == 3 else None
    eager = q.eval(kind, d1, d2).cpu().numpy()
    g, out = q.graph(kind, d1, d2)
    other = _dev(gi.fourier_density(c1, seed=77))
    for rep in range(4):
        out.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep
        # eager work between replays, on the same workspace
        q.eval(1, other)
        torch.cuda.synchronize()
    # the graph goes stale when the buffers change
    q.set_qbx_orders(np.full(c1.n_ctr, 4, np.int32))
    with pytest.raises(GQError) as e:
        g.launch()
    assert e.value.status == _lib.GQ_ESTATE
    g.close()
    big = _dev(np.tile(mu, (129, 1)))
    with pytest.raises(GQError) as e:
        q.graph(1, big)
    assert e.value.status == _lib.GQ_EUNSUP


def test_ragged_batch_matches_separate_contexts():
    """Independent geometries of very different sizes, overlapping in space, in one context:
    each geometry's potentials equal those of its own context (same trees, same work items),
    also with conventional targets, per-center orders and batched densities."""
    geoms = gi.ragged_star_batch(n_geoms=6, seed=200, min_nodes=256, max_nodes=16384)
    g2 = copy.copy(geoms[2])
    pts = np.array([[0.1, 0.2], [3.0, -1.0], [0.5, 0.5]])
    g2.tgt_xy = np.concatenate([g2.tgt_xy, pts])
    g2.tgt_ctr = np.concatenate([g2.tgt_ctr, np.full((3, 2), -1, np.int32)])
    geoms[2] = g2
    from paper_1801_04070_amd import QBXFMM
    kw = dict(p_qbx=12, p_fmm=30)
    qb = QBXFMM(0)
    qb.set_geometry_batch(geoms)
    qb.build(**kw)
    dens = [np.stack([gi.fourier_density(g, seed=40 + i), gi.fourier_density(g, seed=90 + i)])
            for i, g in enumerate(geoms)]
    dens2 = [np.stack([gi.fourier_density(g, seed=140 + i)] * 2) for i, g in enumerate(geoms)]
    db = _dev(np.concatenate(dens, axis=1))
    db2 = _dev(np.concatenate(dens2, axis=1))
    rng = np.random.default_rng(5)
    orders = [rng.choice([4, 6, 8, 12], size=g.n_ctr).astype(np.int32) for g in geoms]
    for kind in (1, 2, 3):
        for use_orders in (False, True):
            qb.set_qbx_orders(np.concatenate(orders) if use_orders else None)
            out = qb.eval(kind, db, db2 if kind == 3 else None).cpu().numpy()
            t0 = 0
            for i, g in enumerate(geoms):
                q = QBXFMM(0)
                q.set_geometry_from(g)
                q.build(**kw)
                if use_orders:
                    q.set_qbx_orders(orders[i])
                ref = q.eval(kind, _dev(dens[i]), _dev(dens2[i]) if kind == 3 else None)
                ref = ref.cpu().numpy()
                part = out[:, t0:t0 + g.n_tgt]
                err = np.abs(part - ref).max() / np.abs(ref).max()
                assert err <= 1e-14, (kind, use_orders, i, err)
                t0 += g.n_tgt
    # features: each center walks its own geometry's tree only
    from paper_1801_04070_amd.learned import center_features
    fb = center_features(qb).cpu().numpy()
    c0 = 0
    for g in geoms:
        q = QBXFMM(0)
        q.set_geometry_from(g)
        q.build(**kw)
        np.testing.assert_array_equal(fb[c0:c0 + g.n_ctr], center_features(q).cpu().numpy())
        c0 += g.n_ctr


@pytest.mark.parametrize("nd", [1, 8])
def test_forest_value_paths_match_separate_contexts(nd):
    """S and D summed at the targets on a forest: three star geometries in one context (one
    target per center, plus conventional targets with internal centers in one of them) against
    a context per geometry, for one density (the one-density value pass) and for 8 (the batched
    value passes, k_near_val_mfma and k_ctr_val): the same trees and work items, so the rows
    agree to rounding; and the first geometry against the oracle."""
    from paper_1801_04070_amd import GQ_S_AND_D, QBXFMM
    geoms = gi.ragged_star_batch(n_geoms=3, seed=300, min_nodes=512, max_nodes=4096)
    g1 = copy.copy(geoms[1])
    pts = np.array([[0.2, 0.1], [2.5, -1.5], [-0.4, 0.9]])
    g1.tgt_xy = np.concatenate([g1.tgt_xy, pts])
    g1.tgt_ctr = np.concatenate([g1.tgt_ctr, np.full((3, 2), -1, np.int32)])
    geoms[1] = g1
    kw = dict(p_qbx=12, p_fmm=30)
    qb = QBXFMM(0)
    qb.set_geometry_batch(geoms)
    qb.build(**kw)
    dens = [np.stack([gi.fourier_density(g, seed=70 + 10 * i + j) for j in range(nd)])
            for i, g in enumerate(geoms)]
    db = _dev(np.concatenate(dens, axis=1))
    out = qb.eval(GQ_S_AND_D, db if nd > 1 else db[0]).cpu().numpy().reshape(2, nd, -1)
    t0 = 0
    for i, g in enumerate(geoms):
        q = QBXFMM(0)
        q.set_geometry_from(g)
        q.build(**kw)
        ref = q.eval(GQ_S_AND_D, _dev(dens[i]) if nd > 1 else _dev(dens[i][0]))
        ref = ref.cpu().numpy().reshape(2, nd, -1)
        part = out[:, :, t0:t0 + g.n_tgt]
        err = np.abs(part - ref).max() / np.abs(ref).max()
        print(f"forest S_AND_D nd={nd} geometry {i}: {err:.2e} against its own context")
        assert err <= 1e-13, (i, err)
        if i == 0:
            for kind in (1, 2):
                o = oracle.qbx_eval(g, kind, dens[0][nd - 1], None, p_qbx=12)
                assert _rel(part[kind - 1, nd - 1], o) < 1e-10, kind
        t0 += g.n_tgt


def test_s_and_d_concurrent_matches_separate(c1):
    """GQ_S_AND_D (S and D of the same densities through one expansion pipeline over two
    workspace halves) against separate S and D evaluations: every center here serves one
    target, so the direct part of S and D is summed at the targets (by the real-coefficient
    recurrence; for a batch as a GEMM of pair weights and strengths) instead of formed as
    coefficients, and the rows agree to rounding, for a batch and for one density; the direct
    path exactly; a captured graph of it replays to the eager rows."""
    from paper_1801_04070_amd import GQ_S_AND_D
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    q, _ = _ctx(g, p_qbx=12, p_fmm=30)
    dens = _dev(np.stack([gi.fourier_density(g, seed=s) for s in (1, 2, 3)]))
    s_ref = q.eval(1, dens).cpu().numpy()
    d_ref = q.eval(2, dens).cpu().numpy()
    both = q.eval(GQ_S_AND_D, dens).cpu().numpy()
    assert both.shape == (6, g.n_tgt)
    eb_s, eb_d = _rel(both[:3], s_ref), _rel(both[3:], d_ref)
    print(f"3-density S and D against GQ_S / GQ_D: S {eb_s:.2e} D {eb_d:.2e}")
    assert eb_s < 1e-13 and eb_d < 1e-13
    one = q.eval(GQ_S_AND_D, dens[0]).cpu().numpy()
    es, ed = _rel(one[0], s_ref[0]), _rel(one[1], d_ref[0])
    print(f"one density S and D against GQ_S / GQ_D: S {es:.2e} D {ed:.2e}")
    assert es < 1e-13 and ed < 1e-13
    ref = oracle.qbx_eval(g, 2, dens[0].cpu().numpy(), None, p_qbx=12)
    assert _rel(one[1], ref) < 1e-10
    # direct path too
    bd = q.eval(GQ_S_AND_D, dens[:2], direct=True).cpu().numpy()
    assert np.array_equal(bd[:2], q.eval(1, dens[:2], direct=True).cpu().numpy())
    assert np.array_equal(bd[2:], q.eval(2, dens[:2], direct=True).cpu().numpy())
    # a captured GQ_S_AND_D evaluation replays to the eager rows
    gr, out = q.graph(GQ_S_AND_D, dens[1])
    gr.launch()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), q.eval(GQ_S_AND_D, dens[1]).cpu().numpy())
    gr.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_packed_list3_far_matches_per_box_items(precision):
    """Stage 5b packed across boxes (far_pairs_per_lane 1) against the per-box items (2, and
    the cost model 0): the same List 3 far sums in another order, so the potentials agree to
    rounding; S, D and S_AND_D over three densities (two slots), and the oracle for FP64."""
    from paper_1801_04070_amd import GQ_FP64, GQ_MIXED_FP32, GQ_S_AND_D
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    prec = GQ_FP64 if precision == "fp64" else GQ_MIXED_FP32
    dens = _dev(np.stack([gi.fourier_density(g, seed=40 + j) for j in range(3)]))
    res = {}
    for ppl in (1, 2, 0):
        q, st = _ctx(g, p_qbx=12, p_fmm=30 if precision == "fp64" else 16, precision=prec,
                     far_pairs_per_lane=ppl, far_chunk=5)
        assert (st["n_m2q_waves"] > 0) == (ppl == 1)
        res[ppl] = (q.eval(1, dens).cpu().numpy(), q.eval(2, dens).cpu().numpy(),
                    q.eval(GQ_S_AND_D, dens).cpu().numpy())
    tol = 1e-13 if precision == "fp64" else 1e-6
    for ppl in (2, 0):
        for a, b in zip(res[1], res[ppl]):
            assert _rel(a, b) < tol, ppl
    # S_AND_D sums its direct part at the targets (one target per center here): S to rounding
    assert _rel(res[1][2][:3], res[1][0]) < tol
    if precision == "fp64":
        mu = gi.fourier_density(g, seed=40)
        ref = oracle.qbx_eval(g, 1, mu, None, p_qbx=12)
        assert _rel(res[1][0][0], ref) < 1e-10


def test_autotune_picks_a_candidate_shape_and_keeps_results():
    """gq_autotune times candidate work-item shapes and keeps the fastest; the potentials stay
    those of the oracle (shapes change only how the direct and List 3 far sums are split)."""
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    mu, _ = _densities(g, 3)
    q, _ = _ctx(g, p_qbx=12, p_fmm=30)
    before = _run(q, 1, mu, None)
    params, ms = q.autotune(1, _dev(mu), reps=2)
    assert ms > 0
    shape = (params.near_chunk, params.far_chunk, params.far_pairs_per_lane)
    assert shape in {(1024, 16, 1), (512, 16, 1), (2048, 16, 1), (1024, 8, 1), (1024, 16, 2),
                     (1024, 32, 1), (4096, 16, 1)}
    after = _run(q, 1, mu, None)
    assert _rel(after, before) < 1e-13
    ref = oracle.qbx_eval(g, 1, mu, None, p_qbx=12)
    assert _rel(after, ref) < 1e-10
    from paper_1801_04070_amd import GQError
    with pytest.raises(GQError):
        q.autotune(3, _dev(mu))


@pytest.mark.parametrize("p_qbx,p_fmm", [(8, 30), (12, 30), (16, 30), (12, 40), (12, 63)])
def test_s_and_d_batch_on_matrix_cores(p_qbx, p_fmm):
    """GQ_S_AND_D over 20 densities: the direct interactions, the moments and P2L run on the
    matrix cores (one GEMM per center or box over its sources and a block of 64 densities, partly
    filled here) and M2L and the Stage 7 gather as GEMMs over the 40 slots, at FMM orders that
    take 2 to 4 row tiles per wavefront. Every S and D row matches the separate single-kind
    evaluation to rounding, the last density the oracle within the gate."""
    from paper_1801_04070_amd import GQ_S_AND_D
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    q, _ = _ctx(g, p_qbx=p_qbx, p_fmm=p_fmm)
    n = 20
    h = np.stack([gi.fourier_density(g, seed=300 + j) for j in range(n)])
    both = q.eval(GQ_S_AND_D, _dev(h)).cpu().numpy()
    assert both.shape == (2 * n, g.n_tgt)
    for j in (0, 7, 19):
        s = q.eval(1, _dev(h[j])).cpu().numpy()
        d = q.eval(2, _dev(h[j])).cpu().numpy()
        assert _rel(both[j], s) < 1e-13, j
        assert _rel(both[n + j], d) < 1e-13, j
    for kind, row in ((1, n - 1), (2, 2 * n - 1)):
        ref = oracle.qbx_eval(g, kind, h[n - 1], None, p_qbx=p_qbx)
        assert _rel(both[row], ref) < 1e-10, kind


def test_s_and_d_batch_mixed_precision():
    """FP32 box expansions for a batch of 20 densities of S and D: moments, P2L, M2L and the
    Stage 7 gather on the FP32 matrix cores (per-batch FP32 products summed in FP64), the direct
    pass on the FP64 matrix cores; against the oracle at the mixed-precision gate 1e-6, and the
    single-density mixed evaluation (vector-unit moments and P2L, FP32 matrix-core M2L and
    gather) to the same gate."""
    from paper_1801_04070_amd import GQ_MIXED_FP32, GQ_S_AND_D
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    q, _ = _ctx(g, p_qbx=12, p_fmm=16, precision=GQ_MIXED_FP32)
    n = 20
    h = np.stack([gi.fourier_density(g, seed=500 + j) for j in range(n)])
    both = q.eval(GQ_S_AND_D, _dev(h)).cpu().numpy()
    one = q.eval(GQ_S_AND_D, _dev(h[n - 1])).cpu().numpy()
    for kind, row, orow in ((1, n - 1, 0), (2, 2 * n - 1, 1)):
        ref = oracle.qbx_eval(g, kind, h[n - 1], None, p_qbx=12)
        e_b, e_1 = _rel(both[row], ref), _rel(one[orow], ref)
        print(f"mixed S_AND_D kind={kind}: batch {e_b:.3e} single {e_1:.3e}")
        assert e_b < 1e-6 and e_1 < 1e-6


@pytest.mark.parametrize("kind", [1, 2, 3])
def test_off_surface_targets_by_association(kind):
    """Targets anywhere in the plane (Sec. 2.2.2): pushed off the curve by up to 2.2 center radii
    along the normal, plus points all over the bounding box. gq_associate_targets gives each a
    center (inside its disk or within the 20 % slack) or leaves it to the conventional paths
    (point value: direct sum, multipole-to-point, local-to-point). One evaluation for all of them
    against the oracle's one-sided QBX at the associated centers and its plain point sums."""
    from paper_1801_04070_amd import associate_targets
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    rng = np.random.default_rng(40 + kind)
    i = rng.integers(0, g.n_src, 3000)
    near = g.src_xy[i] + rng.uniform(-2.2, 2.2, 3000)[:, None] * g.ctr_r[2 * i][:, None] * g.src_nrm[i]
    lo, hi = g.src_xy.min(0) - 1.0, g.src_xy.max(0) + 1.0
    tgt = np.concatenate([near, rng.uniform(lo, hi, (2000, 2))])
    tc, n_gap = associate_targets(g.ctr_xy, g.ctr_r, tgt, slack=0.2, far_factor=3.0)
    qbx = tc[:, 0] >= 0
    assert qbx.sum() > 1500 and (~qbx).sum() > 1500
    e = copy.copy(g)
    e.tgt_xy, e.tgt_ctr = tgt, tc
    q, stats = _ctx(e, p_qbx=12, p_fmm=30)
    assert stats["n_point_targets"] == (~qbx).sum()
    mu, mu2 = _densities(g, 8)
    d2 = mu2 if kind == 3 else None
    gpu = _run(q, kind, mu, mu2)
    ref_q = oracle.qbx_eval(g, kind, mu, d2, p_qbx=12, tgt_xy=tgt[qbx], tgt_ctr=tc[qbx])
    ref_p = oracle.point_potential(g, kind, mu, d2, tgt_xy=tgt[~qbx])
    e_q, e_p = _rel(gpu[qbx], ref_q), _rel(gpu[~qbx], ref_p)
    print(f"off-surface kind={kind}: qbx {qbx.sum()} ({e_q:.2e}), conventional {(~qbx).sum()} "
          f"({e_p:.2e}), gaps {n_gap}")
    assert e_q < 1e-10 and e_p < 1e-10


@pytest.mark.parametrize("nd,orders", [(1, False), (20, False), (20, True)])
def test_s_and_d_values_and_coefficient_paths(nd, orders):
    """GQ_S_AND_D sums the direct part at the targets only when every center serves at most one
    target, and for a batch of 8 or more densities also the box parts (L2QBXL, M2QBXL). The
    on-surface geometry (one target per center, value path) and the same geometry with
    off-surface targets added to its centers (several targets per center: the coefficient rows)
    agree with GQ_S and GQ_D at their common targets to rounding, and the latter with the oracle
    within the gate; also with per-center QBX orders (one pass per order group)."""
    from paper_1801_04070_amd import GQ_S_AND_D
    g = gi.random_stars(n_curves=3, panels_per_curve=64, seed=14, box=12.0)
    rng = np.random.default_rng(77)
    i = rng.integers(0, g.n_src, 400)
    c = 2 * i + rng.integers(0, 2, 400)   # one of the node's two centers
    extra = g.ctr_xy[c] + 0.5 * g.ctr_r[c][:, None] * rng.uniform(-1, 1, (400, 2)) / np.sqrt(2)
    e = copy.copy(g)
    e.tgt_xy = np.concatenate([g.tgt_xy, extra])
    e.tgt_ctr = np.concatenate([g.tgt_ctr, np.stack([c, np.full(400, -1)], 1)]).astype(np.int32)
    dens = np.stack([gi.fourier_density(g, seed=300 + j) for j in range(nd)])
    dd = _dev(dens if nd > 1 else dens[0])
    rows = {}
    po = np.random.default_rng(5).choice([4, 6, 8, 12], size=g.n_ctr).astype(np.int32)
    for name, geom in (("values", g), ("coefficients", e)):
        q, _ = _ctx(geom, p_qbx=12, p_fmm=30)
        if orders:
            q.set_qbx_orders(po)
        both = q.eval(GQ_S_AND_D, dd).cpu().numpy().reshape(2, nd, -1)
        s_ref = q.eval(1, dd).cpu().numpy().reshape(nd, -1)
        d_ref = q.eval(2, dd).cpu().numpy().reshape(nd, -1)
        es, ed = _rel(both[0], s_ref), _rel(both[1], d_ref)
        print(f"S_AND_D nd={nd} {name}: against GQ_S {es:.2e}, GQ_D {ed:.2e}")
        assert es < 1e-13 and ed < 1e-13, name
        rows[name] = both
    n = g.n_tgt
    assert _rel(rows["coefficients"][:, :, :n], rows["values"]) < 1e-13
    if orders:
        return  # the oracle runs one uniform order; GQ_S / GQ_D above hold the same orders
    j = nd - 1
    for kind in (1, 2):
        ref = oracle.qbx_eval(e, kind, dens[j], None, p_qbx=12)
        assert _rel(rows["coefficients"][kind - 1, j], ref) < 1e-10, kind


@pytest.mark.parametrize("tcr_shape,level_restrict", [(1, 0), (0, 1), (1, 1)])
def test_tree_variants_match_oracle(tcr_shape, level_restrict):
    """The disk-shaped TCR and the level-restricted tree give other lists; the potentials still
    match the oracle within the gate (S, D and S_AND_D, one and several densities)."""
    from paper_1801_04070_amd import GQ_S_AND_D
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    q, _ = _ctx(g, p_qbx=12, p_fmm=30, tcr_shape=tcr_shape, level_restrict=level_restrict)
    h = np.stack([gi.fourier_density(g, seed=700 + j) for j in range(10)])
    both = q.eval(GQ_S_AND_D, _dev(h)).cpu().numpy()
    one = q.eval(GQ_S_AND_D, _dev(h[9])).cpu().numpy()
    for kind, rows in ((1, (9, 0)), (2, (19, 1))):
        ref = oracle.qbx_eval(g, kind, h[9], None, p_qbx=12)
        assert _rel(both[rows[0]], ref) < 1e-10 and _rel(one[rows[1]], ref) < 1e-10, kind
