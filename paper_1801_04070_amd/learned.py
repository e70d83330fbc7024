"""Learned per-center QBX orders (an addition to the method; the paper uses one uniform order).

Sec. 4.1 ties the QBX error at a center to its expansion radius, the distance to the nearest
singular part of the field, and how well the quadrature resolves the density near the center.
``gq_center_features`` measures those quantities for every center; a small network
(``include/gigaqbx_mlp.h``) maps them to the predicted log10 QBX error at each candidate order,
and every center takes the lowest order whose prediction, plus a calibrated safety margin, meets
the tolerance. Without a trained model the evaluation keeps the uniform build order.

All arithmetic (features, network, order choice, evaluation) runs in the HIP library; this
module marshals arguments, and its trainer drives the library's own kernels:

* training data: for random 2 x 2 lattices of stars (``gq_inputs.order_training_geometry``,
  sources upsampled to 64 Gauss nodes per 16-node panel, as QBX needs) the library's FMM
  (p_fmm 40) evaluates Green's formula S(du/dn) - D(u) for u = log|x - x0| (x0 outside the
  lattice), one target per center at its own node, at every candidate order.
  The exact one-sided limits are u on the interior side and 0 on the exterior side, so the
  label of (center, order) is the log10 of its true error relative to max |u| at the targets;
* training: Adam on the weighted squared error of the scaled log10 errors;
* calibration: per candidate order j and tolerance, the margin m_j is the smallest (in steps of
  0.05) for which no held-out center with prediction_j + m_j <= tol has a true error above the
  tolerance (calibrated at log10 tolerances -8, -10 and -12).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import GQ_S_MINUS_D, QBXFMM, GQError, library, _ptr, _lib

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "order_mlp.npz")

CANDIDATES = (4, 6, 8, 10, 12, 16)
OUT_SCALE, OUT_SHIFT = 4.0, -10.0      # predicted log10 error = OUT_SCALE * y + OUT_SHIFT
LOG10_FLOOR = -13.0                    # labels below 1e-13 carry only rounding noise
N_HIDDEN = 64
CAL_TOLS = (-8.0, -10.0, -12.0)


def center_features(fmm: QBXFMM):
    """(n_ctr, 8) FP32 device tensor of per-center features (caller's center order)."""
    import torch
    f = torch.empty((fmm.n_ctr, _lib.GQ_N_FEATURES), dtype=torch.float32,
                    device=f"cuda:{fmm.device}")
    fmm._check(fmm._L.gq_center_features(fmm._h, _ptr(f)))
    return f


class OrderModel:
    """Trained network weights with the output scaling and the calibrated margins."""

    def __init__(self, params, n_hidden=N_HIDDEN, candidates=CANDIDATES, out_scale=OUT_SCALE,
                 out_shift=OUT_SHIFT, margins=None, meta=None):
        self.params = np.asarray(params, dtype=np.float32)
        self.n_hidden = int(n_hidden)
        self.candidates = tuple(int(c) for c in candidates)
        self.out_scale, self.out_shift = float(out_scale), float(out_shift)
        self.margins = dict(margins or {})
        self.meta = dict(meta or {})
        self._nets = {}

    @classmethod
    def load(cls, path: str = WEIGHTS) -> "OrderModel":
        z = np.load(path, allow_pickle=False)
        meta = json.loads(str(z["meta"]))
        return cls(z["params"], int(z["n_hidden"]), tuple(z["candidates"].tolist()),
                   float(z["out_scale"]), float(z["out_shift"]),
                   {float(k): [float(x) for x in v] for k, v in meta.pop("margins").items()},
                   meta)

    def save(self, path: str = WEIGHTS) -> None:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        meta = dict(self.meta)
        meta["margins"] = {str(k): v for k, v in self.margins.items()}
        np.savez(path, params=self.params, n_hidden=self.n_hidden,
                 candidates=np.array(self.candidates, np.int32), out_scale=self.out_scale,
                 out_shift=self.out_shift, meta=json.dumps(meta, sort_keys=True))

    def network(self, device: int = 0):
        from .mlp import MLP
        if device not in self._nets:
            net = MLP(_lib.GQ_N_FEATURES, self.n_hidden, len(self.candidates), device=device)
            net.set_params(self.params)
            self._nets[device] = net
        return self._nets[device]

    def margin(self, log10_tol: float) -> list:
        """Per-candidate margins calibrated at this tolerance; for another tolerance those of the
        nearest calibrated one at or below it (the tightest if none is below)."""
        n = len(self.candidates)
        if not self.margins:
            return [1.0] * n
        ks = sorted(self.margins)
        below = [k for k in ks if k <= log10_tol + 1e-9]
        return list(self.margins[below[-1] if below else ks[0]])

    def predict_log10_errors(self, fmm: QBXFMM):
        """(n_ctr, n_candidates) FP32 device tensor of predicted log10 QBX errors."""
        y = self.network(fmm.device).forward(center_features(fmm))
        return y * self.out_scale + self.out_shift

    def choose_orders(self, fmm: QBXFMM, log10_tol: float, margin=None, apply: bool = True):
        """Per-center orders (int32 device tensor); applied to ``fmm`` unless apply=False."""
        import torch
        m = np.asarray(self.margin(log10_tol) if margin is None else
                       np.broadcast_to(margin, (len(self.candidates),)), dtype=np.float64).copy()
        net = self.network(fmm.device)
        cand = np.array(self.candidates, np.int32)
        out = torch.empty(fmm.n_ctr, dtype=torch.int32, device=f"cuda:{fmm.device}")
        fmm._check(fmm._L.gq_orders_predict(fmm._h, net._h, cand.ctypes.data, len(cand),
                                            self.out_scale, self.out_shift, float(log10_tol),
                                            m.ctypes.data, _ptr(out), int(apply)))
        return out


def load_default() -> OrderModel | None:
    """The shipped model, or None (callers then keep uniform orders)."""
    try:
        return OrderModel.load(WEIGHTS)
    except (OSError, KeyError, ValueError):
        return None


def choose_orders(fmm: QBXFMM, log10_tol: float, model: OrderModel | None = None):
    """Learned orders for ``fmm`` (built with p_qbx >= the largest candidate), or the uniform
    build order when no model is available. Returns the orders tensor or None (uniform)."""
    model = model if model is not None else load_default()
    if model is None or fmm.params.p_qbx < max(model.candidates):
        fmm.set_qbx_orders(None)
        return None
    return model.choose_orders(fmm, log10_tol)


# ----------------------------------------------------------------------------- training ----

def error_table(geom, x0, device: int = 0, p_fmm: int = 40):
    """Features (n_ctr, 8) and true log10 errors (n_ctr, n_candidates) of one geometry.

    One target per center at its own node; Green's formula with u = log|x - x0| gives the exact
    one-sided limits u (interior centers, even index) and 0 (exterior centers, odd index)."""
    import torch
    import gq_inputs as gi
    g = gi.per_center_targets(geom)
    fmm = QBXFMM(device)
    fmm.set_geometry_from(g)
    fmm.build(p_qbx=max(CANDIDATES), p_fmm=p_fmm)
    feat = center_features(fmm)
    dudn, u, u_tgt = gi.green_test_field(g, x0)
    dev = f"cuda:{device}"
    d1 = torch.from_numpy(dudn).to(dev)
    d2 = torch.from_numpy(u).to(dev)
    want = torch.from_numpy(u_tgt).to(dev)
    want[1::2] = 0.0
    scale = float(np.abs(u_tgt).max())
    errs = []
    for p in CANDIDATES:
        fmm.set_qbx_orders(np.full(fmm.n_ctr, p, np.int32))
        v = fmm.eval(GQ_S_MINUS_D, d1, d2)
        errs.append(((v - want).abs() / scale).clamp_min(10.0 ** LOG10_FLOOR).log10())
    fmm.close()
    return feat, torch.stack(errs, dim=1).float()


def dataset(seeds, device: int = 0, log=None):
    import torch
    import gq_inputs as gi
    xs, ts = [], []
    for s in seeds:
        geom, x0 = gi.order_training_geometry(int(s))
        f, e = error_table(geom, x0, device)
        xs.append(f)
        ts.append(e)
        if log:
            q = torch.quantile(e, torch.tensor([0.1, 0.5, 0.9], device=e.device), dim=0)
            log(f"seed {s}: {f.shape[0]} centers; log10 order error by order, 10/50/90%: "
                + " ".join("/".join(f"{float(v):.1f}" for v in q[:, j]) for j in range(e.shape[1])))
    return torch.cat(xs), torch.cat(ts)


def calibrate(pred, true, tols=CAL_TOLS, step=0.05, max_margin=6.0):
    """Per-candidate margins: for each tolerance and order j the smallest m (multiple of `step`)
    such that no held-out row with pred_j + m <= tol has true_j > tol."""
    out = {}
    for tol in tols:
        ms = []
        for j in range(pred.shape[1]):
            p, t = pred[:, j], true[:, j]
            m = 0.0
            while m < max_margin:
                sel = p + m <= tol
                if not bool((t[sel] > tol).any()):
                    break
                m = round(m + step, 10)
            ms.append(round(m, 2))
        out[float(tol)] = ms
    return out


def choice_report(pred, true, margins, candidates=CANDIDATES):
    """On held-out rows, per tolerance: among rows whose largest candidate meets the tolerance,
    the miss rate and worst log10 error of the chosen orders; the share of rows no candidate can
    meet; the mean chosen order, the mean of the smallest order that truly meets the tolerance,
    and the smallest uniform order whose worst error meets it."""
    import torch
    cand = torch.tensor(candidates, device=pred.device)
    rep = {}
    for tol, m in margins.items():
        fits = pred + torch.tensor(m, device=pred.device) <= tol
        last = torch.full_like(fits[:, 0], len(candidates) - 1, dtype=torch.long)
        j = torch.where(fits.any(1), fits.float().argmax(1), last)
        err = true.gather(1, j[:, None])[:, 0]
        ok = true <= tol
        best = torch.where(ok.any(1), ok.float().argmax(1), last)
        feas = ok[:, -1]
        uni = [c for c, col in zip(candidates, true.T) if bool((col[feas] <= tol).all())]
        rep[str(tol)] = {"miss_rate": float((err[feas] > tol).float().mean()),
                         "worst_log10_err": round(float(err[feas].max()), 2),
                         "infeasible_rate": float((~feas).float().mean()),
                         "mean_order": round(float(cand[j].float().mean()), 3),
                         "mean_best_order": round(float(cand[best].float().mean()), 3),
                         "uniform_order": uni[0] if uni else None}
    return rep


def train(train_seeds=range(1000, 1180), val_seeds=range(1180, 1200), steps: int = 4000,
          batch: int = 16384, lr: float = 2e-3, seed: int = 7, device: int = 0, log=print):
    """Train the order network on the GPU with the library's kernels; returns (model, report)."""
    import torch
    from .mlp import MLP
    t0 = time.time()
    x, e = dataset(train_seeds, device, log)
    xv, ev = dataset(val_seeds, device, log)
    t_data = time.time() - t0
    tgt = (e - OUT_SHIFT) / OUT_SCALE
    net = MLP(_lib.GQ_N_FEATURES, N_HIDDEN, len(CANDIDATES), seed=seed, device=device)
    gen = torch.Generator(device=f"cuda:{device}")
    gen.manual_seed(seed)
    n = x.shape[0]
    hist = []
    t1 = time.time()
    for it in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), device=x.device, generator=gen)
        rate = lr * 0.5 * (1.0 + np.cos(np.pi * it / steps))   # cosine decay
        want = it % 500 == 0 or it == steps - 1
        loss = net.train_step(x[idx], tgt[idx], lr=rate, want_loss=want)
        if want:
            hist.append((it, loss))
            log(f"step {it}: loss {loss:.5f}")
    torch.cuda.synchronize()
    t_train = time.time() - t1
    model = OrderModel(net.get_params(), N_HIDDEN, CANDIDATES, OUT_SCALE, OUT_SHIFT)
    pv = net.forward(xv) * OUT_SCALE + OUT_SHIFT
    model.margins = calibrate(pv, ev)
    choice = choice_report(pv, ev, model.margins)
    rmse = ((pv - ev) ** 2).mean(0).sqrt().tolist()
    report = {"train_rows": int(n), "val_rows": int(xv.shape[0]), "steps": steps,
              "batch": batch, "lr": lr, "seconds_data": round(t_data, 1),
              "seconds_train": round(t_train, 1), "val_rmse_log10": [round(v, 3) for v in rmse],
              "margins": model.margins, "validation_choice": choice, "loss_history": hist,
              "train_seeds": [int(min(train_seeds)), int(max(train_seeds))],
              "val_seeds": [int(min(val_seeds)), int(max(val_seeds))]}
    model.meta = {k: v for k, v in report.items() if k != "loss_history"}
    return model, report


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="train the per-center QBX order network on the GPU")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--report", default=None)
    ap.add_argument("--train-seeds", type=int, nargs=2, default=(1000, 1180))
    ap.add_argument("--val-seeds", type=int, nargs=2, default=(1180, 1200))
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=2e-3)
    a = ap.parse_args(argv)
    library()
    model, report = train(range(*a.train_seeds), range(*a.val_seeds), a.steps, a.batch, a.lr,
                          log=lambda s: print(s, flush=True))
    model.save(a.out)
    print(json.dumps(report), flush=True)
    if a.report:
        with open(a.report, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
