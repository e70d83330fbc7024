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
  (p_fmm 40) evaluates Green's formula S(du/dn) - D(u) for u = log|x - x0| (x0 outside every
  curve, often close to one), one target per center at its own node, at every candidate order.
  The exact one-sided limits are u on the interior side and 0 on the exterior side, so the
  label of (center, order) is the log10 of its true error relative to max |u| at the targets;
* training: Adam on the weighted squared error of the scaled log10 errors;
* calibration: the margin is the smallest one for which, on held-out geometries, no center's
  chosen order exceeds the tolerance (checked at log10 tolerances -6, -8 and -10).
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
LOG10_FLOOR = -16.0
N_HIDDEN = 64
CAL_TOLS = (-6.0, -8.0, -10.0)


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
                   {float(k): float(v) for k, v in meta.pop("margins").items()}, meta)

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

    def margin(self, log10_tol: float) -> float:
        """Calibrated margin at this tolerance, else the largest calibrated one (1 if none)."""
        if not self.margins:
            return 1.0
        for k, v in self.margins.items():
            if abs(k - log10_tol) < 1e-6:
                return v
        return max(self.margins.values())

    def predict_log10_errors(self, fmm: QBXFMM):
        """(n_ctr, n_candidates) FP32 device tensor of predicted log10 QBX errors."""
        y = self.network(fmm.device).forward(center_features(fmm))
        return y * self.out_scale + self.out_shift

    def choose_orders(self, fmm: QBXFMM, log10_tol: float, margin: float | None = None,
                      apply: bool = True):
        """Per-center orders (int32 device tensor); applied to ``fmm`` unless apply=False."""
        import torch
        m = self.margin(log10_tol) if margin is None else float(margin)
        net = self.network(fmm.device)
        cand = np.array(self.candidates, np.int32)
        out = torch.empty(fmm.n_ctr, dtype=torch.int32, device=f"cuda:{fmm.device}")
        fmm._check(fmm._L.gq_orders_predict(fmm._h, net._h, cand.ctypes.data, len(cand),
                                            self.out_scale, self.out_shift, float(log10_tol), m,
                                            _ptr(out), int(apply)))
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


def calibrate(pred, true, tols=CAL_TOLS, candidates=CANDIDATES):
    """Smallest margin (0.05 steps) with no held-out center whose chosen order misses the
    tolerance, among centers whose largest candidate order meets it."""
    import torch
    out = {}
    for tol in tols:
        ok_at_max = true[:, -1] <= tol
        p, t = pred[ok_at_max], true[ok_at_max]
        m = 0.0
        while m < 6.0:
            fits = p + m <= tol
            first = torch.where(fits.any(1), fits.float().argmax(1),
                                torch.full_like(fits[:, 0], len(candidates) - 1, dtype=torch.long))
            miss = t.gather(1, first[:, None])[:, 0] > tol
            if not bool(miss.any()):
                break
            m += 0.05
        out[float(tol)] = round(m, 2)
    return out


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
    rmse = ((pv - ev) ** 2).mean(0).sqrt().tolist()
    report = {"train_rows": int(n), "val_rows": int(xv.shape[0]), "steps": steps,
              "batch": batch, "lr": lr, "seconds_data": round(t_data, 1),
              "seconds_train": round(t_train, 1), "val_rmse_log10": [round(v, 3) for v in rmse],
              "margins": model.margins, "loss_history": hist,
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
