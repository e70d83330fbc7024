"""Algorithmic work per kernel launch, from the tree/list statistics.

Counting convention (floating-point operations of the method's formulas, not of the generated
code): complex multiply 6, complex add 2, real x complex multiply-add 4, complex multiply-add
8, real multiply-add 2, reciprocal / division / logarithm 1 each. Source-to-expansion steps use
the power recurrences of eqs. (multipole)/(local); translations use the factored forms
(M2L: diag(o^-m) B diag(o^-k); L2QBXL: repeated Horner).

Bytes are the algorithmic HBM traffic of one launch: each operand the kernel must read once and
each result it writes once (source records 24 B for charges, 32 B for dipoles, 40 B for both;
complex coefficients 16 B).
"""
from __future__ import annotations

MI355X_PEAKS = {
    "fp64_vector_tflops": 78.6,   # 256 CU x 2.4 GHz x 128 FP64 flop/clk/CU
    "fp32_vector_tflops": 157.3,
    "fp64_mfma_tflops": 78.6,
    "hbm_gbs": 8000.0,
}


def _near_pair_flops(kind: int, q: int) -> int:
    # z = y - c (2; the sums run in z^-m and take the factor r^m once per center), 1/z (6);
    # charge: log|z| term (3), q-1 powers (6 each), q accumulations (4)
    f = 2 + 6
    if kind == 4:
        # S and D of one density in one pass: z, 1/z and the powers 1/z^m (m <= q+1) once;
        # charge: log term (3), q accumulations (4); dipole: q+1 complex multiply-adds (8)
        return f + 3 + 6 * q + 4 * q + 8 * (q + 1)
    if kind & 1:
        f += 3 + 6 * (q - 1) + 4 * q
    if kind & 2:
        # e = d/z (6), q powers (6 each), q+1 complex adds (2)
        f += 6 + 6 * q + 2 * (q + 1)
    return f


def _m2qbxl_flops(q: int, p: int) -> int:
    # y, 1/y, w = s/y, u = -r/y, log|y|; a_0 terms; a_k w^k; sum_k C(m+k-1,k-1) T_k for all m;
    # output scaling by u^m and accumulation
    return 16 + 10 * q + 12 * p + 4 * (q + 1) * p + 6 * q + 8 * (q + 1)


def _l2qbxl_flops(q: int, p: int) -> int:
    # t, 1/t, t^p (binary powers, ~2 log2 p products); per k: a_k = b_k t^k and the next power
    # (2 complex products), q+1 complex adds of the Horner in (1 + h); r/(c - c_b) and its q powers
    # applied to the q coefficients (2q products)
    logp = max(p, 1).bit_length()
    return 12 + 6 * 2 * logp + (p + 1) * (12 + 2 * (q + 1)) + 12 * q


def _qbxl2p_flops(q: int) -> int:
    return 5 + 8 * q


def stage_work(stats: dict, kind: int, p_qbx: int, p_fmm: int, n_slots: int,
               near_values: bool = False) -> dict:
    """Algorithmic flops and HBM bytes of one launch of each stage for one density; kind 4 (S and
    D of the same density, one pipeline) is the sum of the two kinds except for the direct
    interactions, whose pair geometry is formed once. The flops are the method's (coefficient
    formation and evaluation) whatever the kernel's formulation; near_values: the direct pass and
    the List 3 far pass write one double per (center, chunk) row and kind instead of the
    coefficient row, and the center stage reads those (every center serving one target)."""
    if kind == 4:
        s = stage_work(stats, 1, p_qbx, p_fmm, n_slots, near_values)
        d = stage_work(stats, 2, p_qbx, p_fmm, n_slots, near_values)
        out = {k: {"flops": s[k]["flops"] + d[k]["flops"], "bytes": s[k]["bytes"] + d[k]["bytes"],
                   "bound": s[k]["bound"]} for k in s}
        row = (p_qbx + 1) * 16
        P1 = p_fmm + 1
        out["p2m"] = {"flops": stats.get("n_moment_pairs", 0) * (4 + 6 * p_fmm + 12 * P1),
                      "bytes": stats.get("n_moment_pairs", 0) * 40
                               + 2 * stats.get("n_moment_boxes", 0) * P1 * 16, "bound": "alu"}
        out["near"] = {"flops": stats["near_pairs"] * _near_pair_flops(4, p_qbx),
                       "bytes": stats["near_sources"] * (40 + 4) + stats["n_ctr"] * 24
                                + 2 * stats["n_ctr"] * (8 if near_values else row),
                       "bound": "alu"}
        return out
    q, p = p_qbx, p_fmm
    P1, Q1 = p + 1, q + 1
    src_rec = {1: 24, 2: 32, 3: 40}[kind]
    row = 8 if near_values else Q1 * 16  # a row: one value at the target, or the coefficients
    n_rows_near = stats["n_ctr"]  # at least one direct row per center
    out = {}
    out["near"] = {
        "flops": stats["near_pairs"] * _near_pair_flops(kind, q),
        "bytes": stats["near_sources"] * (src_rec + 4) + stats["n_ctr"] * 24 + n_rows_near * row,
        "bound": "alu"}
    out["m2qbxl"] = {
        "flops": stats["list3_far_pairs"] * _m2qbxl_flops(q, p),
        "bytes": stats["n_list3_far"] * (P1 * 16 + 20) + stats["list3_far_pairs"] // 8 * row,
        "bound": "alu"}
    out["qbx_center"] = {
        "flops": stats["n_ctr"] * _l2qbxl_flops(q, p) + n_slots * _qbxl2p_flops(q),
        "bytes": stats["n_ctr"] * (24 + 4 + row) + stats["n_target_boxes"] * P1 * 16
                 + n_slots * 24,
        "bound": "alu"}
    per_pair = 6 * P1 + 4 * P1 * P1 + 8 * P1
    p2l = 4 + 6 + 6 * p + 4 * P1 + 3
    out["m2l_p2l"] = {
        "flops": stats["n_list2"] * per_pair + stats["list4_far_sources"] * p2l,
        "bytes": stats["n_list2"] * (P1 * 16 + 8) + stats["n_local_boxes"] * P1 * 16,
        "bound": "alu"}
    tri = P1 * (P1 + 1) // 2
    # Stage 2 as direct moments (k_p2m_all): per (box, subtree source) pair y (4), p powers (6
    # each) and the accumulations (S: 4 per order, D: 8); "m2m" is the sum of split boxes' partials
    nk = 2 if kind == 3 else 1
    out["m2m"] = {"flops": stats.get("n_moment_parts", 0) * P1 * 2 * nk,
                  "bytes": stats.get("n_moment_parts", 0) * P1 * 16 * nk
                           + stats.get("n_moment_parts", 0) // 2 * P1 * 16, "bound": "latency"}
    # Stage 7 as a gather: per (box, ancestor) pair t^j a_j (6 per term), the binomial sum
    # (real x complex multiply-add, 4 per term of the triangle), u^-m (6) and the sum (2)
    out["l2l"] = {"flops": stats.get("n_l2l_pairs", 0) * (6 * P1 + 4 * tri + 8 * P1)
                           + stats.get("n_l2l_sinks", 0) * 2 * P1,
                  "bytes": stats.get("n_l2l_pairs", 0) * (P1 * 16 + 36)
                           + 2 * stats.get("n_l2l_sinks", 0) * P1 * 16, "bound": "alu"}
    p2m = 4 + 6 * p + (4 * P1 if kind & 1 else 0) + (8 * P1 if kind & 2 else 0)
    out["p2m"] = {"flops": stats.get("n_moment_pairs", 0) * p2m,
                  "bytes": stats.get("n_moment_pairs", 0) * src_rec
                           + stats.get("n_moment_boxes", 0) * P1 * 16, "bound": "alu"}
    out["gather"] = {"flops": stats["n_src"] * 3, "bytes": stats["n_src"] * (8 + 8 + 16 + 4 + src_rec - 16),
                     "bound": "hbm"}
    out["finalize"] = {"flops": stats["n_tgt"] * 2, "bytes": stats["n_tgt"] * (16 + 8 + 8), "bound": "hbm"}
    return out


def center_kernel(stats: dict, kind: int, p_qbx: int, p_fmm: int, n_slots: int) -> dict:
    """Flops and bytes of one launch of the per-center kernel (Stages 3, 5, 6a, 8 + QBXL2P)."""
    q, p = p_qbx, p_fmm
    flops = (stats["near_pairs"] * _near_pair_flops(kind, q)
             + stats["list3_far_pairs"] * _m2qbxl_flops(q, p)
             + stats["n_ctr"] * _l2qbxl_flops(q, p)
             + n_slots * _qbxl2p_flops(q))
    src_rec = {1: 24, 2: 32, 3: 40}[kind]
    nbytes = (stats["n_ctr"] * (16 + 8 + 4 + 8)          # center xy, r, box, target-slot index
              + n_slots * (16 + 8)                        # target xy, slot value written
              + stats["n_target_boxes"] * (p + 1) * 16    # box local read once per box
              + stats["n_list3_far"] * (p + 1) * 16       # List 3 far multipoles per box entry
              + stats["near_sources"] * src_rec)     # near sources, once per target box
    return {"flops": flops, "bytes": nbytes}


def m2l_kernel(stats: dict, kind: int, p_fmm: int) -> dict:
    P1 = p_fmm + 1
    per_pair = 6 * P1 + 4 * P1 * P1 + 8 * P1
    p2l = 4 + 6 + 6 * p_fmm + 4 * P1 + 3
    flops = stats["n_list2"] * per_pair + stats["list4_far_sources"] * p2l
    nbytes = stats["n_list2"] * (P1 * 16 + 8) + stats["n_local_boxes"] * P1 * 16
    return {"flops": flops, "bytes": nbytes}
