"""Operator-level checks of the HIP stages (the box expansions read back with
gq_get_expansions), against brute force and the paper's translation properties:

  * multipoles: every box's multipole equals the brute-force expansion (eq. (multipole)) of its
    subtree sources about its center, to roundoff (the direct moments are the multipoles the M2M
    chain of eq. (m2m) would build: in 2-D it keeps the first p + 1 moments exact);
  * the downward pass: every complete local equals the box's own local plus every ancestor's own
    local shifted exactly (eq. (l2l), m = 0..p) to its center, to roundoff ("the FMM forgets
    intermediate translations", Sec. 3.2);
  * M2L and P2L: a box's own local, evaluated at its QBX centers and on their disks, matches the
    direct potential of its List 2 and List 4 far sources within the Lemma-type bound
    A rho^(p+1)/(1 - rho) with rho = (sqrt 2 + t_f)/(6 - sqrt 2) for List 2 and sqrt(2)/3 for
    List 4 far (Sec. 3.2, Theorem 1's factors), and the error falls as p grows.
"""
import math
from types import SimpleNamespace

import numpy as np
import pytest

import gq_inputs as gi
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

T_F = 0.9
ALPHA = (math.sqrt(2) + T_F) / (6 - math.sqrt(2))
BETA = math.sqrt(2) / 3


def _setup(p_fmm, n_max=32, seed=5):
    from paper_1801_04070_amd import GQ_S, QBXFMM, _lib
    g = gi.random_stars(n_curves=3, panels_per_curve=64, seed=seed)
    mu = gi.fourier_density(g, seed=seed)
    q = QBXFMM(device=0)
    q.set_geometry_from(g)
    st = q.build(p_qbx=8, p_fmm=p_fmm, n_max=n_max, t_f=T_F)
    q.eval(GQ_S, torch.as_tensor(mu, device="cuda:0"))
    torch.cuda.synchronize()
    lvl = q.tree_array(_lib.GQ_TREE_BOX_LEVEL)
    side = st["root_side"] / 2.0 ** lvl
    ij = q.tree_array(_lib.GQ_TREE_BOX_IJ)
    lo = np.array(st["root_lo"])
    cen = lo[None, :] + (ij + 0.5) * side[:, None]
    T = SimpleNamespace(
        g=g, mu=mu, q=q, side=side, cz=cen[:, 0] + 1j * cen[:, 1],
        parent=q.tree_array(_lib.GQ_TREE_BOX_PARENT),
        child=q.tree_array(_lib.GQ_TREE_BOX_CHILD),
        src=q.tree_array(_lib.GQ_TREE_BOX_SRC_RANGE), ctr=q.tree_array(_lib.GQ_TREE_BOX_CTR_RANGE),
        src_order=q.tree_array(_lib.GQ_TREE_SRC_ORDER),
        ctr_order=q.tree_array(_lib.GQ_TREE_CTR_ORDER), lists=q.lists(), p=p_fmm)
    return T


def _row(T, name, b):
    st, ix = T.lists[name]
    return ix[st[b]:st[b + 1]]


def _subtree_sources(T, b):
    s0, s1 = T.src[b]
    return T.src_order[s0:s1]


def _leaf_sources(T, d):
    """Sources a box owns directly (List 4 far boxes contribute their own sources)."""
    return _subtree_sources(T, d)


def test_multipoles_equal_brute_force():
    from paper_1801_04070_amd import _lib
    T = _setup(p_fmm=16)
    M = T.q.expansions(_lib.GQ_EXP_MULTIPOLE)
    read = np.unique(np.concatenate([T.lists["list2"][1], T.lists["list3f"][1]]))
    assert len(read) > 20
    worst = 0.0
    for b in read:
        idx = _subtree_sources(T, b)
        sub = SimpleNamespace(src_xy=T.g.src_xy[idx], src_nrm=T.g.src_nrm[idx],
                              src_w=T.g.src_w[idx])
        a = oracle.multipole(sub, oracle.S, T.mu[idx], None, (T.cz[b].real, T.cz[b].imag), T.p)
        got = M[b] * T.side[b] ** np.arange(T.p + 1)
        worst = max(worst, float(np.abs(got - a).max() / np.abs(a).max()))
    print(f"multipoles of {len(read)} boxes: max rel diff {worst:.2e}")
    assert worst < 1e-12


def test_complete_locals_are_exact_shifts_of_own_locals():
    from paper_1801_04070_amd import _lib
    T = _setup(p_fmm=16)
    L = T.q.expansions(_lib.GQ_EXP_LOCAL)
    Lf = T.q.expansions(_lib.GQ_EXP_LOCAL_COMPLETE)
    P = T.p
    k = np.arange(P + 1)
    C = np.array([[math.comb(kk, m) if kk >= m else 0 for m in range(P + 1)] for kk in range(P + 1)],
                 dtype=float)
    owners = [b for b in range(len(T.parent)) if T.ctr[b][1] > T.ctr[b][0]]
    has_own = {b for b in range(len(T.parent))
               if len(_row(T, "list2", b)) or len(_row(T, "list4f", b))}
    worst, n_chain = 0.0, 0
    for b in owners:
        ref = L[b] / T.side[b] ** k if b in has_own else np.zeros(P + 1, complex)
        scale = np.abs(ref).copy()
        a = T.parent[b]
        while a >= 0:
            if a in has_own:
                Ba = L[a] / T.side[a] ** k               # unscaled local of a about c_a
                d = T.cz[b] - T.cz[a]
                terms = C * (Ba[:, None] * d ** np.maximum(k[:, None] - k[None, :], 0))
                terms = np.where(k[:, None] >= k[None, :], terms, 0)
                ref = ref + terms.sum(0)
                scale = scale + np.abs(terms).sum(0)
                n_chain += 1
            a = T.parent[a]
        got = Lf[b] / T.side[b] ** k
        worst = max(worst, float((np.abs(got - ref) / np.maximum(scale, 1e-300)).max()))
    print(f"complete locals of {len(owners)} boxes over {n_chain} ancestor shifts: "
          f"max diff {worst:.2e} of the summed magnitudes")
    assert n_chain > 20
    assert worst < 1e-12


def _own_local_errors(T):
    from paper_1801_04070_amd import _lib
    L = T.q.expansions(_lib.GQ_EXP_LOCAL)
    k = np.arange(T.p + 1)
    out = []
    for b in range(len(T.parent)):
        c0, c1 = T.ctr[b]
        v, x4 = _row(T, "list2", b), _row(T, "list4f", b)
        if c1 <= c0 or (len(v) == 0 and len(x4) == 0):
            continue
        # the box's own centers and points on their disks
        ci = T.ctr_order[c0:c1]
        cz = T.g.ctr_xy[ci, 0] + 1j * T.g.ctr_xy[ci, 1]
        pts = np.concatenate([cz] + [cz + T.g.ctr_r[ci] * np.exp(1j * t)
                                     for t in (0.0, 2.1, 4.2)])
        B = L[b] / T.side[b] ** k
        u = -(0.5 / np.pi) * np.real(np.polyval(B[::-1], pts - T.cz[b]))
        sv = np.concatenate([_subtree_sources(T, d) for d in v]) if len(v) else np.zeros(0, int)
        sx = np.concatenate([_leaf_sources(T, d) for d in x4]) if len(x4) else np.zeros(0, int)
        idx = np.concatenate([sv, sx])
        y = T.g.src_xy[idx, 0] + 1j * T.g.src_xy[idx, 1]
        qv = T.g.src_w[idx] * T.mu[idx]
        ref = -(0.5 / np.pi) * (qv[None, :] * np.log(np.abs(pts[:, None] - y[None, :]))).sum(1)
        av = np.abs(T.g.src_w[sv] * T.mu[sv]).sum() / (2 * np.pi)
        ax = np.abs(T.g.src_w[sx] * T.mu[sx]).sum() / (2 * np.pi)
        bound = ((T.p + 2) * av * ALPHA ** (T.p + 1) / (1 - ALPHA)
                 + (T.p + 2) * ax * BETA ** (T.p + 1) / (1 - BETA))
        out.append((float(np.abs(u - ref).max()), bound))
    return out


@pytest.mark.parametrize("p_fmm", [8, 14])
def test_own_locals_within_translation_bounds(p_fmm):
    T = _setup(p_fmm=p_fmm)
    errs = _own_local_errors(T)
    assert len(errs) > 20
    ratio = max(e / b for e, b in errs)
    print(f"p_fmm {p_fmm}: {len(errs)} boxes, max error {max(e for e, _ in errs):.2e}, "
          f"max error/bound {ratio:.2e}")
    assert ratio <= 1.0


def test_own_local_error_falls_with_order():
    e8 = max(e for e, _ in _own_local_errors(_setup(p_fmm=8)))
    e14 = max(e for e, _ in _own_local_errors(_setup(p_fmm=14)))
    print(f"max own-local error: p 8 {e8:.2e}, p 14 {e14:.2e}")
    assert e14 < e8 * ALPHA ** 4
