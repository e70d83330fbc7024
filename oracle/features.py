"""Brute-force per-center geometry features -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may import
this module. It shares nothing with the library's feature kernel: every center looks at every
source (no tree), in FP64 numpy, with the definitions written out one by one.

For a center c with radius r, over the sources y with |y - c| < 4 r (weight w, unit normal n):
  0: sum of w over |y - c| < 2 r, divided by 4 r
  1: sum of w over |y - c| < 4 r, divided by 8 r
  2: min over all sources of |y - c|, divided by r (4 when no source lies within 4 r)
  3: log2(r * count / sum of w)  (0 when the disk holds no source)
  4: |sum w n| / sum w
  5: sqrt(weighted variance of o = (y - c).n / r)
  6: weighted mean of o
  7: min |y - c| over sources whose normal has a negative dot product with the normal of the
     nearest source, divided by 4 r (1 when there is none inside the disk)
The features are the inputs of the order-prediction network, an addition to the method; they
have no counterpart in the paper, so their pins are closed forms on circles (see the tests).
"""
from __future__ import annotations

import numpy as np


def center_features(src_xy, src_nrm, src_w, ctr_xy, ctr_r) -> np.ndarray:
    src_xy = np.asarray(src_xy, np.float64)
    src_nrm = np.asarray(src_nrm, np.float64)
    src_w = np.asarray(src_w, np.float64)
    out = np.zeros((len(ctr_r), 8))
    for c, (x, r) in enumerate(zip(np.asarray(ctr_xy, np.float64), np.asarray(ctr_r, np.float64))):
        e = src_xy - x
        d = np.hypot(e[:, 0], e[:, 1])
        R = 4.0 * r
        near = d < R
        if not near.any():
            out[c] = [0, 0, 4.0, 0, 0, 0, 0, 1.0]
            continue
        k0 = np.argmin(np.where(near, d, np.inf))
        n0 = src_nrm[k0]
        w, n, ee, dd = src_w[near], src_nrm[near], e[near], d[near]
        a2 = w[dd < 2.0 * r].sum()
        a4 = w.sum()
        o = (ee * n).sum(1) / r
        mean_o = (w * o).sum() / a4
        var_o = max((w * o * o).sum() / a4 - mean_o ** 2, 0.0)
        opp = (n @ n0) < 0
        out[c] = [a2 / r / 4, a4 / r / 8, d[k0] / r, np.log2(max(r * near.sum() / a4, 1e-3)),
                  np.hypot(*(w[:, None] * n).sum(0)) / a4, np.sqrt(var_o), mean_o,
                  (dd[opp].min() if opp.any() else R) / R]
    return out
