"""Tree and interaction lists (Stage 1, Sec. 4.3) checked by brute force on the host.

Runs through a host-only library context (no GPU): the builder is the library's own C++.
Checks, for every box that owns centers, that the sources reaching its centers through
  direct evaluation      List 1 U List 3 close U List 4 close (leaf sources),
  multipole -> QBX local List 3 far (subtree sources),
  box local expansions   List 2 and List 4 far of the box and all its ancestors
partition the source set exactly once; that every list entry satisfies its defining predicate
(Definitions 1-9); the list-size bounds of Sec. 4.6 (|List 2| <= 75, |List 4 close| <= 42,
|List 4 far| <= 63); and that every owned center's disk lies inside its box's target
confinement region.
"""
import copy
import json
import os

import numpy as np
import pytest

import gq_inputs as gi
from paper_1801_04070_amd import QBXFMM, _lib

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _build(geom, **kw):
    q = QBXFMM(device=-1)
    q.set_geometry_from(geom)
    stats = q.build(**kw)
    T = {
        "level": q.tree_array(_lib.GQ_TREE_BOX_LEVEL),
        "parent": q.tree_array(_lib.GQ_TREE_BOX_PARENT),
        "child": q.tree_array(_lib.GQ_TREE_BOX_CHILD),
        "ij": q.tree_array(_lib.GQ_TREE_BOX_IJ),
        "src": q.tree_array(_lib.GQ_TREE_BOX_SRC_RANGE),
        "ctr": q.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE),
        "src_order": q.tree_array(_lib.GQ_TREE_SRC_ORDER),
        "ctr_order": q.tree_array(_lib.GQ_TREE_CTR_ORDER),
    }
    T.update(q.lists())
    T["stats"] = stats
    lo = np.array(stats["root_lo"])
    side = stats["root_side"] / 2.0 ** T["level"]
    T["half"] = 0.5 * side
    T["center"] = lo[None, :] + (T["ij"] + 0.5) * side[:, None]
    T["leaf"] = (T["child"] < 0).all(axis=1)
    return q, T


def _row(T, name, b):
    st, ix = T[name]
    return ix[st[b]:st[b + 1]]


def _linf(T, a, b):
    return np.abs(T["center"][a] - T["center"][b]).max()


def _adjacent(T, a, b):
    return _linf(T, a, b) <= T["half"][a] + T["half"][b] * (1 + 1e-15) + 1e-300


def _ancestors(T, b):
    out = []
    while b >= 0:
        out.append(b)
        b = T["parent"][b]
    return out


GEOMS = {
    "c1": lambda: gi.starfish_c1(),
    "three_stars": lambda: gi.random_stars(n_curves=3, panels_per_curve=40, seed=4, box=8.0),
    "circle_small_boxes": lambda: gi.unit_circle(48),
}


def _dist2_sq(p, c, s):
    """Euclidean distance from point p to the closed square of radius s about c."""
    d = np.maximum(np.abs(np.asarray(p) - np.asarray(c)) - s, 0.0)
    return float(np.hypot(d[..., 0], d[..., 1]))


def _check_tree(geom, t_f=0.9, n_max=64, count_mode=0, w3=15, tcr_shape=0, level_restrict=0):
    q, T = _build(geom, p_qbx=8, p_fmm=10, t_f=t_f, n_max=n_max, count_mode=count_mode,
                  w3far_min_sources=w3, tcr_shape=tcr_shape, level_restrict=level_restrict)
    disk = tcr_shape == 1

    def dnorm(v):  # the TCR's norm of center offsets
        return np.hypot(v[..., 0], v[..., 1]) if disk else np.abs(v).max(axis=-1)

    def sep_d_tcr(d, b):  # d < TCR(b) (Definition 1 with the TCR's shape)
        if disk:
            return _dist2_sq(T["center"][b], T["center"][d], 3 * T["half"][d]) >= \
                T["half"][b] * (1 + t_f) * (1 - 1e-12)
        return _linf(T, d, b) >= (3 * T["half"][d] + T["half"][b] * (1 + t_f)) * (1 - 1e-12)

    def sep_tcr_d(b, d):  # TCR(b) < d
        if disk:
            return _dist2_sq(T["center"][b], T["center"][d],
                             T["half"][d] + 2 * T["half"][b] * (1 + t_f)) >= \
                T["half"][b] * (1 + t_f) * (1 - 1e-12)
        return _linf(T, d, b) >= (3 * T["half"][b] * (1 + t_f) + T["half"][d]) * (1 - 1e-12)
    nb = len(T["level"])
    ns = geom.n_src
    src = T["src"]
    # ---- particles: orders are permutations, box ranges consistent ----
    assert np.array_equal(np.sort(T["src_order"]), np.arange(ns))
    assert np.array_equal(np.sort(T["ctr_order"]), np.arange(geom.n_ctr))
    assert src[0, 0] == 0 and src[0, 1] == ns
    for b in range(nb):
        kids = [c for c in T["child"][b] if c >= 0]
        if kids:
            # non-leaf boxes own no sources: the subtree range is the union of the children's
            assert sum(src[c, 1] - src[c, 0] for c in kids) == src[b, 1] - src[b, 0]
    # every source lies in its leaf's closed square; every owned center disk fits the TCR
    xy = geom.src_xy[T["src_order"]]
    cxy = geom.ctr_xy[T["ctr_order"]]
    cr = geom.ctr_r[T["ctr_order"]]
    for b in range(nb):
        s0, s1 = src[b]
        if T["leaf"][b] and s1 > s0:
            d = np.abs(xy[s0:s1] - T["center"][b]).max()
            assert d <= T["half"][b] * (1 + 1e-12)
        c0, c1 = T["ctr"][b]
        if c1 > c0 and b != 0:
            reach = dnorm(cxy[c0:c1] - T["center"][b]) + cr[c0:c1]
            assert (reach <= T["half"][b] * (1 + t_f) * (1 + 1e-12)).all()
    # subdivision rule: a leaf owns at most n_max particles eligible for children (sources, and
    # centers whose disk would fit the TCR of the child containing them), unless at max depth
    for b in range(nb):
        if T["leaf"][b]:
            c0, c1 = T["ctr"][b]
            hc = 0.5 * T["half"][b]
            quad = (cxy[c0:c1] >= T["center"][b]).astype(float) * 2 - 1
            chc = T["center"][b] + quad * hc
            elig = (dnorm(cxy[c0:c1] - chc) + cr[c0:c1] <= hc * (1 + t_f)).sum()
            cnt = (src[b, 1] - src[b, 0]) + (elig if count_mode == 0 else 0)
            assert cnt <= n_max or T["level"][b] == T["stats"]["n_levels"] - 1
    if level_restrict:
        # Remark 2: no leaf has an adjacent source leaf (closed squares touching) two or more
        # levels coarser
        leaves = np.nonzero(T["leaf"])[0]
        sleaves = leaves[src[leaves, 1] > src[leaves, 0]]
        for a in leaves:
            near = sleaves[(np.abs(T["center"][sleaves] - T["center"][a]).max(axis=1)
                            <= (T["half"][sleaves] + T["half"][a]) * (1 + 1e-12))]
            assert (T["level"][near] >= T["level"][a] - 1).all(), a
    # ---- exact-once coverage and predicates for every box owning centers ----
    tf1 = 1 + t_f
    counts = {"list2": 0, "list4c": 0, "list4f": 0}
    for b in range(nb):
        for name in counts:
            counts[name] = max(counts[name], len(_row(T, name, b)))
        if T["ctr"][b, 1] == T["ctr"][b, 0]:
            continue
        ranges = []
        for name in ("list1", "list3c", "list4c"):
            for d in _row(T, name, b):
                assert T["leaf"][d], name
                ranges.append(tuple(src[d]))
        for d in _row(T, "list3f", b):
            ranges.append(tuple(src[d]))
        for w in _ancestors(T, b):
            for d in _row(T, "list2", w):
                ranges.append(tuple(src[d]))
            for d in _row(T, "list4f", w):
                ranges.append(tuple(src[d]))
        ranges = sorted(r for r in ranges if r[1] > r[0])
        assert ranges[0][0] == 0 and ranges[-1][1] == ns, "coverage does not span all sources"
        for r0, r1 in zip(ranges[:-1], ranges[1:]):
            assert r0[1] == r1[0], f"box {b}: gap or overlap between source ranges {r0} {r1}"
        # predicates
        for d in _row(T, "list1", b):
            assert _adjacent(T, b, d)
        for d in _row(T, "list3f", b):
            assert sep_d_tcr(d, b)
            assert not _adjacent(T, b, d) and T["level"][d] > T["level"][b]
        if w3 == 0:
            for d in _row(T, "list3c", b):
                assert not sep_d_tcr(d, b)
                assert not _adjacent(T, b, d)
        for d in _row(T, "list4c", b):
            assert not sep_tcr_d(b, d)
    for b in range(nb):
        for d in _row(T, "list2", b):
            assert T["level"][d] == T["level"][b]
            assert np.abs(T["ij"][d] - T["ij"][b]).max() in (3, 4, 5)  # 2-well-separated
        for d in _row(T, "list4f", b):
            assert sep_tcr_d(b, d)
            assert T["leaf"][d] and T["level"][d] <= T["level"][b]
            assert not _adjacent(T, b, d)
    return T, counts


@pytest.mark.parametrize("name", sorted(GEOMS))
@pytest.mark.parametrize("count_mode", [0, 1])
def test_lists_partition_sources(name, count_mode):
    _check_tree(GEOMS[name](), count_mode=count_mode)


@pytest.mark.parametrize("t_f", [0.0, 0.5, 0.9])
@pytest.mark.parametrize("n_max", [8, 32])
def test_lists_partition_deep_trees(t_f, n_max):
    # small n_max forces deep adaptive trees with many suspended centers
    _check_tree(gi.random_stars(n_curves=2, panels_per_curve=24, seed=9, box=6.0), t_f=t_f,
                n_max=n_max, w3=0)


@pytest.mark.parametrize("tcr_shape,level_restrict", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("n_max", [8, 64])
def test_tree_variants_partition_sources(tcr_shape, level_restrict, n_max):
    """The disk-shaped TCR and the level-restricted tree (Remark 2) keep the exact-once partition
    of the sources for every center, every list entry satisfies its relation for that TCR shape,
    and in the level-restricted tree no leaf has an adjacent source leaf two levels coarser."""
    g = gi.random_stars(n_curves=3, panels_per_curve=40, seed=4, box=8.0)
    T, counts = _check_tree(g, n_max=n_max, tcr_shape=tcr_shape, level_restrict=level_restrict)
    const = _golden()
    assert counts["list2"] <= const["max_list2"]["value"]
    assert counts["list4c"] <= const["max_list4_close"]["value"]
    assert counts["list4f"] <= const["max_list4_far"]["value"]


def test_level_restriction_on_full_size_tree(c2_tree):
    """Remark 2 on the 131072-source tree: the level-restricted tree has more boxes, and fewer
    direct (center, source) pairs and List 3 far pairs than the tree as built; the lists still
    meet the Sec. 4.6 size bounds."""
    g, T = c2_tree
    _, R = _build(g, p_qbx=12, p_fmm=30, level_restrict=1)
    a, b = T["stats"], R["stats"]
    assert b["n_boxes"] > a["n_boxes"]
    assert b["near_pairs"] < a["near_pairs"] and b["list3_far_pairs"] < a["list3_far_pairs"]
    const = _golden()
    assert b["max_list2"] <= const["max_list2"]["value"]
    assert b["max_list4"] <= const["max_list4"]["value"]
    assert b["max_list4_close"] <= const["max_list4_close"]["value"]
    assert b["max_list4_far"] <= const["max_list4_far"]["value"]


def test_remark1_demotion_keeps_partition():
    T0, _ = _check_tree(gi.starfish_c1(), n_max=16, w3=0)
    T1, _ = _check_tree(gi.starfish_c1(), n_max=16, w3=15)
    assert len(T1["list3f"][1]) <= len(T0["list3f"][1])


def test_list_size_bounds():
    with open(GOLDEN) as f:
        const = json.load(f)
    for name in GEOMS:
        _, counts = _check_tree(GEOMS[name]())
        assert counts["list2"] <= const["max_list2"]["value"]
        assert counts["list4c"] <= const["max_list4_close"]["value"]
        assert counts["list4f"] <= const["max_list4_far"]["value"]


def test_root_square_is_dyadic_and_covers_disks():
    g = gi.starfish_c1()
    q = QBXFMM(device=-1)
    q.set_geometry_from(g)
    s = q.build(p_qbx=8, p_fmm=10)
    side = s["root_side"]
    assert side == 2.0 ** round(np.log2(side))
    lo = np.array(s["root_lo"])
    assert (g.ctr_xy - g.ctr_r[:, None] >= lo).all()
    assert (g.ctr_xy + g.ctr_r[:, None] < lo + side).all()


def test_error_paths_host_context():
    from paper_1801_04070_amd import GQError
    g = gi.starfish_c1()
    q = QBXFMM(device=-1)
    with pytest.raises(GQError) as e:
        q.build(p_qbx=8, p_fmm=10)
    assert e.value.status == _lib.GQ_ESTATE
    bad = g.src_xy.copy()
    bad[3, 0] = np.nan
    with pytest.raises(GQError) as e:
        q.set_geometry(bad, g.src_nrm, g.src_w, g.ctr_xy, g.ctr_r, g.tgt_xy, g.tgt_ctr)
    assert e.value.status == _lib.GQ_EINVAL
    q.set_geometry_from(g)
    with pytest.raises(GQError) as e:
        q.build(p_qbx=8, p_fmm=10, n_max=0)
    assert e.value.status == _lib.GQ_EINVAL
    with pytest.raises(GQError) as e:
        q.build(p_qbx=8, p_fmm=99)
    assert e.value.status == _lib.GQ_EUNSUP
    # coincident particles stop at the depth guard instead of recursing forever
    n = 200
    same = np.zeros((n, 2))
    nrm = np.tile([1.0, 0.0], (n, 1))
    q2 = QBXFMM(device=-1)
    q2.set_geometry(same, nrm, np.ones(n), np.array([[0.5, 0.0]]), np.array([0.1]),
                    np.zeros((1, 2)), np.array([[0, -1]], np.int32))
    s = q2.build(p_qbx=8, p_fmm=10, n_max=8, max_levels=12)
    assert s["n_levels"] == 12


def test_box_orders_from_center_orders():
    """gq_set_qbx_orders: each box gets the smallest compiled order >= its centers' largest."""
    g = gi.starfish_c1()
    q = QBXFMM(device=-1)
    q.set_geometry_from(g)
    q.build(p_qbx=12, p_fmm=10)
    assert (q.box_orders() == 12).all()
    orders = np.random.default_rng(1).integers(0, 13, size=g.n_ctr).astype(np.int32)
    q.set_qbx_orders(orders)
    bo = q.box_orders()
    rng_c = q.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE)
    order_c = q.tree_array(_lib.GQ_TREE_CTR_ORDER)
    compiled = [4, 6, 8, 10, 12]
    for b, (c0, c1) in enumerate(rng_c):
        if c1 > c0:
            need = orders[order_c[c0:c1]].max()
            assert bo[b] == min(c for c in compiled if c >= need)
    from paper_1801_04070_amd import GQError
    with pytest.raises(GQError):
        q.set_qbx_orders(np.full(g.n_ctr, 13, np.int32))


def test_center_orders_regroup_centers_within_boxes():
    """Per-center orders: every center runs at the smallest compiled order >= its own; inside each
    box the centers are regrouped by that order (ascending, ties in their previous order), the
    set of centers per box and every list stay as built, and NULL restores the uniform order."""
    g = gi.random_stars(n_curves=3, panels_per_curve=40, seed=4, box=8.0)
    q = QBXFMM(device=-1)
    q.set_geometry_from(g)
    q.build(p_qbx=12, p_fmm=10)
    rng_c = q.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE)
    before = q.tree_array(_lib.GQ_TREE_CTR_ORDER)
    lists = q.lists()
    orders = np.random.default_rng(2).integers(0, 13, size=g.n_ctr).astype(np.int32)
    q.set_qbx_orders(orders)
    compiled = np.array([4, 6, 8, 10, 12])
    eff = compiled[np.searchsorted(compiled, orders)]
    np.testing.assert_array_equal(q.center_orders(), eff)
    after = q.tree_array(_lib.GQ_TREE_CTR_ORDER)
    for c0, c1 in rng_c:
        assert sorted(before[c0:c1]) == sorted(after[c0:c1])
        e = eff[after[c0:c1]]
        assert (np.diff(e) >= 0).all()
    for k, (st, ix) in q.lists().items():
        assert np.array_equal(st, lists[k][0]) and np.array_equal(ix, lists[k][1]), k
    q.set_qbx_orders(None)
    assert (q.center_orders() == 12).all()


def _with_point_targets(g, n_pt=300, seed=4):
    """Add conventional targets (both center slots -1) off the curve and around it."""
    rng = np.random.default_rng(seed)
    lo, hi = g.src_xy.min(0) - 0.3, g.src_xy.max(0) + 0.3
    pts = rng.uniform(lo, hi, size=(n_pt, 2))
    tgt_xy = np.concatenate([g.tgt_xy, pts])
    tgt_ctr = np.concatenate([g.tgt_ctr, np.full((n_pt, 2), -1, np.int32)])
    return pts, tgt_xy, tgt_ctr


def test_point_targets_match_explicit_tiny_centers():
    """A target with no center gets an internal center of radius 2^-40 * extent at its position,
    numbered after the caller's centers: the same tree as passing those centers explicitly."""
    g = gi.random_stars(n_curves=2, panels_per_curve=24, seed=9, box=6.0)
    pts, tgt_xy, tgt_ctr = _with_point_targets(g)
    q = QBXFMM(device=-1)
    q.set_geometry(g.src_xy, g.src_nrm, g.src_w, g.ctr_xy, g.ctr_r, tgt_xy, tgt_ctr)
    s = q.build(p_qbx=8, p_fmm=10, n_max=16)
    assert s["n_point_targets"] == len(pts) and s["n_ctr"] == g.n_ctr
    allxy = np.concatenate([g.src_xy, g.ctr_xy, tgt_xy])
    ext = (allxy.max(0) - allxy.min(0)).max()
    r_pt = np.ldexp(ext, -40)
    e = copy.copy(g)
    e.ctr_xy = np.concatenate([g.ctr_xy, pts])
    e.ctr_r = np.concatenate([g.ctr_r, np.full(len(pts), r_pt)])
    tc = tgt_ctr.copy()
    tc[len(g.tgt_xy):, 0] = g.n_ctr + np.arange(len(pts))
    e.tgt_xy, e.tgt_ctr = tgt_xy, tc
    q2 = QBXFMM(device=-1)
    q2.set_geometry_from(e)
    q2.build(p_qbx=8, p_fmm=10, n_max=16)
    for what in range(_lib.GQ_TREE_BOX_LEVEL, _lib.GQ_LIST4F + 1):
        assert np.array_equal(q.tree_array(what), q2.tree_array(what)), what
    T, _ = _check_tree(e, n_max=16)
    # every point target's center sits in a leaf that contains it
    owner = np.empty(e.n_ctr, np.int64)
    rng_c = q.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE)
    order_c = q.tree_array(_lib.GQ_TREE_CTR_ORDER)
    for b, (c0, c1) in enumerate(rng_c):
        owner[order_c[c0:c1]] = b
    assert all(T["leaf"][owner[g.n_ctr + j]] for j in range(len(pts)))
    # orders: point-target centers never raise a box's order
    q.set_qbx_orders(np.full(g.n_ctr, 4, np.int32))
    bo = q.box_orders()
    assert (bo[rng_c[:, 1] > rng_c[:, 0]] == 4).all()


def test_point_targets_only():
    g = gi.starfish_c1()
    pts = np.array([[0.0, 0.0], [3.0, 1.0], [0.2, -0.1]])
    q = QBXFMM(device=-1)
    q.set_geometry(g.src_xy, g.src_nrm, g.src_w, np.zeros((0, 2)), np.zeros(0), pts,
                   np.full((3, 2), -1, np.int32))
    s = q.build(p_qbx=4, p_fmm=10)
    assert s["n_ctr"] == 0 and s["n_point_targets"] == 3
    from paper_1801_04070_amd import GQError
    with pytest.raises(GQError):
        q.set_geometry(g.src_xy, g.src_nrm, g.src_w, np.zeros((0, 2)), np.zeros(0),
                       np.zeros((0, 2)), np.zeros((0, 2), np.int32))


def _boxes_by_tree(q):
    """Per forest box: (tree root, depth, i, j); roots found by following parents."""
    par = q.tree_array(_lib.GQ_TREE_BOX_PARENT)
    ij = q.tree_array(_lib.GQ_TREE_BOX_IJ)
    out = []
    for b in range(len(par)):
        d, r = 0, b
        while par[r] >= 0:
            r = par[r]
            d += 1
        out.append((r, d, int(ij[b, 0]), int(ij[b, 1])))
    return out


def test_forest_matches_separate_trees():
    """A batch of geometries (two of them overlapping in space) builds the same trees and lists
    as separate contexts, renumbered: boxes by (depth, i, j) within each tree, particles offset."""
    geoms = [gi.starfish_c1(), gi.unit_circle(24),
             gi.random_stars(n_curves=2, panels_per_curve=24, seed=9, box=6.0),
             gi.discretize([gi.StarCurve(amp=0.2, arms=3)], 40)]
    pts, tgt_xy, tgt_ctr = _with_point_targets(geoms[2], n_pt=50)
    g2 = copy.copy(geoms[2])
    g2.tgt_xy, g2.tgt_ctr = tgt_xy, tgt_ctr
    geoms[2] = g2
    kw = dict(p_qbx=8, p_fmm=10, n_max=16)
    qf = QBXFMM(device=-1)
    qf.set_geometry_batch(geoms)
    sf = qf.build(**kw)
    singles = []
    for g in geoms:
        q = QBXFMM(device=-1)
        q.set_geometry_from(g)
        singles.append((q, q.build(**kw)))
    for key in ("n_boxes", "n_leaves", "n_list1", "n_list2", "n_list3_close", "n_list3_far",
                "n_list4_close", "n_list4_far", "near_pairs", "n_point_targets"):
        assert sf[key] == sum(s[key] for _, s in singles), key
    fb = _boxes_by_tree(qf)
    roots = sorted({r for r, *_ in fb})
    assert len(roots) == len(geoms)
    so = np.concatenate([[0], np.cumsum([len(g.src_w) for g in geoms])])
    co = np.concatenate([[0], np.cumsum([len(g.ctr_r) for g in geoms])])
    f_src, f_ctr = qf.tree_array(_lib.GQ_TREE_SRC_ORDER), qf.tree_array(_lib.GQ_TREE_CTR_ORDER)
    f_lists = qf.lists()
    s_pos = c_pos = 0
    n_user = co[-1]
    pt_seen = 0
    for k, (q, st) in enumerate(singles):
        ns, nc_all = len(geoms[k].src_w), st["n_ctr"] + st["n_point_targets"]
        assert np.array_equal(f_src[s_pos:s_pos + ns], q.tree_array(_lib.GQ_TREE_SRC_ORDER) + so[k])
        c_single = q.tree_array(_lib.GQ_TREE_CTR_ORDER)
        want = np.where(c_single < st["n_ctr"], c_single + co[k],
                        n_user + pt_seen + (c_single - st["n_ctr"]))
        assert np.array_equal(f_ctr[c_pos:c_pos + nc_all], want)
        s_pos += ns
        c_pos += nc_all
        pt_seen += st["n_point_targets"]
        # lists, keyed by (depth, i, j) inside tree k
        sb = _boxes_by_tree(q)
        # roots are the first boxes of the depth-major numbering, in geometry order
        key_f = {b: (d, i, j) for b, (r, d, i, j) in enumerate(fb) if r == roots[k]}
        inv_f = {v: b for b, v in key_f.items()}
        s_lists = q.lists()
        for name in f_lists:
            fs, fi = f_lists[name]
            ss, si = s_lists[name]
            for b, (_, d, i, j) in enumerate(sb):
                fbx = inv_f[(d, i, j)]
                got = sorted(key_f[e] for e in fi[fs[fbx]:fs[fbx + 1]])
                exp = sorted(sb[e][1:] for e in si[ss[b]:ss[b + 1]])
                assert got == exp, (name, k, b)


@pytest.mark.parametrize("name", ["stars", "deep"])
def test_stage_work_counts(name):
    """The work the expansion stages are sized by, recomputed from the lists: direct moments for
    every box M2L (List 2) or M2QBXL (List 3 far) reads, split into 512-source items; the
    Stage 7 gather over every box owning centers and its ancestors with a List 2 or List 4 far
    row of their own."""
    if name == "stars":
        g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
        q, T = _build(g, p_qbx=12, p_fmm=30)
    else:
        g = gi.random_stars(n_curves=3, panels_per_curve=64, seed=21, box=12.0)
        q, T = _build(g, p_qbx=12, p_fmm=30, n_max=8)
    st = T["stats"]
    need = np.zeros(len(T["level"]), bool)
    need[T["list2"][1]] = True
    need[T["list3f"][1]] = True
    n = T["src"][:, 1] - T["src"][:, 0]
    assert st["n_moment_boxes"] == need.sum()
    assert st["n_moment_pairs"] == n[need].sum()
    big = need & (n > 512)
    assert st["n_moment_parts"] == np.ceil(n[big] / 512).sum()
    own = (np.diff(T["list2"][0]) > 0) | (np.diff(T["list4f"][0]) > 0)
    sinks = np.nonzero(T["ctr"][:, 1] > T["ctr"][:, 0])[0]
    pairs = 0
    for b in sinks:
        a = T["parent"][b]
        while a >= 0:
            pairs += own[a]
            a = T["parent"][a]
    assert st["n_l2l_sinks"] == len(sinks)
    assert st["n_l2l_pairs"] == pairs
    # every box read by M2L/M2QBXL has sources (its moments are not trivially zero)
    assert (n[need] > 0).all()


def _packed_far_waves(T, chunk=16, stage_rows=16):
    """Greedy packing of (center, List 3 far chunk) units, written from the rule: box order,
    whole units, at most 64 pairs and stage_rows staged far boxes per wavefront, a chunk staged
    once per wavefront that holds any of its units."""
    nc = T["ctr"][:, 1] - T["ctr"][:, 0]
    W = np.diff(T["list3f"][0])
    waves = units = 0
    lanes = staged = 0
    for b in np.nonzero(nc)[0]:
        for c0 in range(0, W[b], chunk):
            cl = min(chunk, W[b] - c0)
            in_wave = False
            for _ in range(nc[b]):
                if lanes + cl > 64 or (not in_wave and staged + cl > stage_rows):
                    waves += 1
                    lanes = staged = 0
                    in_wave = False
                if not in_wave:
                    staged += cl
                    in_wave = True
                lanes += cl
                units += 1
    return waves + (lanes > 0), units


@pytest.mark.parametrize("far_chunk", [16, 3])
def test_packed_list3_far_work(far_chunk):
    """Stage 5b packed across boxes: every (center, List 3 far box) pair once, one row per
    (center, far chunk), and the wavefront count of the packing rule, recomputed from the lists."""
    g = gi.random_stars(n_curves=3, panels_per_curve=128, seed=12, box=12.0)
    q, T = _build(g, p_qbx=12, p_fmm=30, far_chunk=far_chunk)
    st = T["stats"]
    nc = T["ctr"][:, 1] - T["ctr"][:, 0]
    W = np.diff(T["list3f"][0])
    assert st["list3_far_pairs"] > 0
    assert st["n_m2q_pairs"] == st["list3_far_pairs"] == (nc * W).sum()
    waves, units = _packed_far_waves(T, chunk=far_chunk)
    assert st["n_m2q_units"] == units == (nc * np.ceil(W / far_chunk)).sum()
    assert st["n_m2q_waves"] == waves
    assert waves >= np.ceil(st["n_m2q_pairs"] / 64)
    # items of one box's centers instead: no packed work
    q2, T2 = _build(g, p_qbx=12, p_fmm=30, far_chunk=far_chunk, far_pairs_per_lane=2)
    assert T2["stats"]["n_m2q_waves"] == T2["stats"]["n_m2q_pairs"] == 0


def test_packed_list3_far_work_forest():
    """The packed Stage 5b work of a ragged batch (one forest): every (center, List 3 far box)
    pair of every geometry once, one row per (center, far chunk), and the packing rule's
    wavefront count over the merged lists."""
    from paper_1801_04070_amd import QBXFMM
    geoms = gi.ragged_star_batch(n_geoms=4, seed=200)
    q = QBXFMM(device=-1)
    q.set_geometry_batch(geoms)
    st = q.build(p_qbx=12, p_fmm=30)
    T = {"ctr": q.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE)}
    T.update(q.lists())
    nc = T["ctr"][:, 1] - T["ctr"][:, 0]
    W = np.diff(T["list3f"][0])
    assert st["n_m2q_pairs"] == st["list3_far_pairs"] == (nc * W).sum() > 0
    waves, units = _packed_far_waves(T)
    assert st["n_m2q_units"] == units
    assert st["n_m2q_waves"] == waves


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _center_boxes(T):
    """Owning box of every tree-order center position (centers are numbered in pre-order)."""
    cbox = np.empty(T["ctr"][:, 1].max(), np.int64)
    for b, (c0, c1) in enumerate(T["ctr"]):
        cbox[c0:c1] = b
    return cbox


def _furthest_target(T, cxy, cr, cbox):
    """Per box b: max over the centers c owned by b or a descendant of |c - c_b| + r_c."""
    ft = np.zeros(len(T["level"]))
    b = cbox.copy()
    while (b >= 0).any():
        ok = b >= 0
        np.maximum.at(ft, b[ok], np.hypot(*(cxy[ok] - T["center"][b[ok]]).T) + cr[ok])
        nxt = b.copy()
        nxt[ok] = T["parent"][b[ok]]
        b = nxt
    return ft


@pytest.fixture(scope="module")
def c2_tree():
    g = gi.config_geometry("c2")
    q, T = _build(g, p_qbx=12, p_fmm=30)
    return g, T


def test_list_bounds_on_full_size_tree(c2_tree):
    """The Sec. 4.6 list-size bounds on the 131072-source tree: |List 2| <= 75, |List 4| <= 21,
    |List 4 close| <= 42, |List 4 far| <= 63 per box, and at most 64 List 3 far boxes per
    center (Lemma for Stage 5)."""
    g, T = c2_tree
    const = _golden()
    st = T["stats"]
    assert st["max_list2"] <= const["max_list2"]["value"]
    assert st["max_list4"] <= const["max_list4"]["value"]
    assert st["max_list4_close"] <= const["max_list4_close"]["value"]
    assert st["max_list4_far"] <= const["max_list4_far"]["value"]
    for name, key in (("list2", "max_list2"), ("list4c", "max_list4_close"),
                      ("list4f", "max_list4_far")):
        assert np.diff(T[name][0]).max() == st[key]
    owns = (T["ctr"][:, 1] - T["ctr"][:, 0]) > 0
    assert np.diff(T["list3f"][0])[owns].max() <= const["list3_far_per_center"]["value"]


def test_convergence_factors_on_full_size_tree(c2_tree):
    """Theorem 1's convergence factors as the geometric ratios of the separation figures, over
    every list entry of the 131072-source tree:
      List 2 (b, d): furthest target of b over closest point of d's circumscribed disk, at most
        alpha = (t_f + sqrt 2)/(6 - sqrt 2) (0.5046 at t_f = 0.9);
      List 3 far (c, d): radius of d's circumscribed disk over the distance from c_d to c's QBX
        disk, at most sqrt(2)/3;
      List 4 far (b, d): furthest target of b over the closest source of d, at most sqrt(2)/3.
    "Furthest target" is the largest |c - c_b| + r_c over the QBX centers below b."""
    g, T = c2_tree
    const = _golden()
    alpha = const["list2_convergence_factor_tf09"]["value"]
    far = const["list34_far_convergence_factor"]["value"]
    assert abs(alpha - (0.9 + 2 ** 0.5) / (6 - 2 ** 0.5)) < 1e-6
    cbox = _center_boxes(T)
    cxy, cr = g.ctr_xy[T["ctr_order"]], g.ctr_r[T["ctr_order"]]
    ft = _furthest_target(T, cxy, cr, cbox)
    nb = len(T["level"])
    cen, half = T["center"], T["half"]

    def pairs(name):
        st, ix = T[name]
        return np.repeat(np.arange(nb), np.diff(st)), ix

    b, d = pairs("list2")
    r2 = ft[b] / (np.hypot(*(cen[b] - cen[d]).T) - np.sqrt(2) * half[d])
    assert r2.max() <= alpha + 1e-9 and r2.max() > 0.45
    st3 = T["list3f"][0]
    n3 = np.diff(st3)[cbox]
    ci = np.repeat(np.arange(len(cbox)), n3)
    d3 = np.concatenate([T["list3f"][1][st3[x]:st3[x + 1]] for x in cbox])
    r3 = np.sqrt(2) * half[d3] / (np.hypot(*(cxy[ci] - cen[d3]).T) - cr[ci])
    assert len(r3) > 0 and r3.max() <= far + 1e-9
    b, d = pairs("list4f")
    ns = T["src"][d, 1] - T["src"][d, 0]
    pid = np.repeat(np.arange(len(b)), ns)
    src = np.concatenate([np.arange(T["src"][x, 0], T["src"][x, 1]) for x in d])
    y = g.src_xy[T["src_order"][src]]
    mind = np.full(len(b), np.inf)
    np.minimum.at(mind, pid, np.hypot(*(y - cen[b[pid]]).T))
    r4 = ft[b] / mind
    assert len(r4) > 0 and r4.max() <= far + 1e-9


@pytest.mark.parametrize("t_f", [0.9, 0.5, 0.0])
def test_mean_sources_near_centers_brute_force(t_f):
    """M_C (Sec. 4.6.1): the mean number of sources in the closed square of radius 8 r_c / t_f
    about each center, from the library's tree walk, against counting every (center, source)
    pair; t_f = 0 counts every source."""
    g = gi.random_stars(n_curves=3, panels_per_curve=40, seed=4, box=8.0)
    q = QBXFMM(device=-1)
    q.set_geometry_from(g)
    st = q.build(p_qbx=8, p_fmm=10, t_f=t_f)
    total = 0
    for c in range(g.n_ctr):
        if t_f == 0.0:
            total += g.n_src
        else:
            total += int((np.abs(g.src_xy - g.ctr_xy[c]).max(1) <= 8 * g.ctr_r[c] / t_f).sum())
    assert st["m_c_sum"] == total
    assert st["m_c"] == pytest.approx(total / g.n_ctr, rel=1e-15)


def test_fmm_order_from_accuracy():
    """Sec. 4.1: with p_fmm <= 0 the FMM order comes from the requested accuracy,
    p_fmm = ceil(|log2 eps|); eps outside (0, 1) is rejected."""
    from paper_1801_04070_amd import GQError
    g = gi.starfish_c1()
    q = QBXFMM(device=-1)
    q.set_geometry_from(g)
    for eps, p in ((0.5, 1), (1e-6, 20), (1e-10, 34), (2.0 ** -30, 30), (1e-30, 63)):
        q.build(p_qbx=8, p_fmm=0, eps=eps)
        assert q.params.p_fmm == p, (eps, q.params.p_fmm)
    q.build(p_qbx=8, p_fmm=15, eps=1e-10)
    assert q.params.p_fmm == 15
    for bad in (0.0, 1.0, -1e-3):
        with pytest.raises(GQError) as e:
            q.build(p_qbx=8, p_fmm=0, eps=bad)
        assert e.value.status == _lib.GQ_EINVAL


def _model_ops_from_lists(T, orders, n_user, p_fmm, n_src):
    """The per-list-entry cost model, center by center from the exported tree and lists: a QBX
    center of order p in box b costs p per source of List 1, List 3 close and List 4 close of b,
    p_FMM p per List 3 far box and p_FMM p for its own local (Stage 8); List 2 entries cost
    p_FMM^2, List 4 far entries p_FMM per source; forming multipoles p_FMM per source, and each
    upward (downward) shift p_FMM^2 for a non-root box with sources (with centers below it)."""
    ops = dict.fromkeys(_lib.GQ_OP_NAMES, 0)
    ns = T["src"][:, 1] - T["src"][:, 0]
    nb = len(T["level"])
    has_ctr = np.zeros(nb, bool)
    for b in range(nb):
        if T["ctr"][b, 1] > T["ctr"][b, 0]:
            a = b
            while a >= 0 and not has_ctr[a]:
                has_ctr[a] = True
                a = T["parent"][a]
    ops["multipoles"] = p_fmm * n_src
    for b in range(nb):
        if T["parent"][b] >= 0:
            ops["m2m"] += p_fmm ** 2 * (ns[b] > 0)
            ops["l2l"] += p_fmm ** 2 * has_ctr[b]
        ops["list2"] += p_fmm ** 2 * len(_row(T, "list2", b))
        ops["list4_far"] += p_fmm * int(ns[_row(T, "list4f", b)].sum())
        for k in range(T["ctr"][b, 0], T["ctr"][b, 1]):
            c = T["ctr_order"][k]
            if c >= n_user:
                continue
            p = int(orders[c])
            ops["list1"] += p * int(ns[_row(T, "list1", b)].sum())
            ops["list3_close"] += p * int(ns[_row(T, "list3c", b)].sum())
            ops["list4_close"] += p * int(ns[_row(T, "list4c", b)].sum())
            ops["list3_far"] += p_fmm * p * len(_row(T, "list3f", b))
            ops["l2qbxl"] += p_fmm * p
    return ops


def test_modeled_operation_counts():
    """gq_stats.model_ops against the cost model evaluated center by center from the exported
    lists, at the uniform order, after per-center orders, and with conventional targets (whose
    internal centers the model leaves out); under the uniform order the direct and far terms
    also equal the orders times the pair counts the stats report."""
    g = gi.random_stars(n_curves=3, panels_per_curve=64, seed=21, box=12.0)
    q, T = _build(g, p_qbx=12, p_fmm=30, n_max=8)
    st = T["stats"]
    exp = _model_ops_from_lists(T, np.full(g.n_ctr, 12), g.n_ctr, 30, g.n_src)
    assert st["model_ops"] == exp
    assert st["model_ops_total"] == sum(exp.values())
    near = exp["list1"] + exp["list3_close"] + exp["list4_close"]
    assert near == 12 * st["near_pairs"]
    assert exp["list3_far"] == 30 * 12 * st["list3_far_pairs"]
    assert exp["list4_far"] == 30 * st["list4_far_sources"]
    assert exp["list2"] == 30 ** 2 * st["n_list2"]
    assert exp["l2qbxl"] == 30 * 12 * g.n_ctr
    # Table 2's bounds: Stage 4 <= 75 N_B p_FMM^2, Stage 7 <= 4 N_B p_FMM^2 (one shift per box)
    assert exp["list2"] <= 75 * st["n_boxes"] * 30 ** 2
    assert exp["l2l"] <= st["n_boxes"] * 30 ** 2 and exp["m2m"] <= st["n_boxes"] * 30 ** 2

    orders = np.random.default_rng(3).integers(0, 13, size=g.n_ctr).astype(np.int32)
    q.set_qbx_orders(orders)
    got = q.stats()["model_ops"]
    assert got == _model_ops_from_lists(T, q.center_orders(), g.n_ctr, 30, g.n_src)
    assert got["list2"] == exp["list2"] and got["list1"] < exp["list1"]

    pts, tgt_xy, tgt_ctr = _with_point_targets(g)
    q2 = QBXFMM(device=-1)
    q2.set_geometry(g.src_xy, g.src_nrm, g.src_w, g.ctr_xy, g.ctr_r, tgt_xy, tgt_ctr)
    s2 = q2.build(p_qbx=8, p_fmm=10, n_max=16)
    T2 = {"level": q2.tree_array(_lib.GQ_TREE_BOX_LEVEL),
          "parent": q2.tree_array(_lib.GQ_TREE_BOX_PARENT),
          "src": q2.tree_array(_lib.GQ_TREE_BOX_SRC_RANGE),
          "ctr": q2.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE),
          "ctr_order": q2.tree_array(_lib.GQ_TREE_CTR_ORDER)}
    T2.update(q2.lists())
    exp2 = _model_ops_from_lists(T2, np.full(g.n_ctr, 8), g.n_ctr, 10, g.n_src)
    assert s2["model_ops"] == exp2
    assert exp2["l2qbxl"] == 10 * 8 * g.n_ctr
