"""Throughput of the GIGAQBX FMM hot path on one MI355X.

Headline workload: 16 random star curves, 8192 panels x 16 Gauss-Legendre nodes = 131072 sources,
two QBX centers per node (radius = half the panel arclength), 131072 on-surface targets,
p_qbx = 12, p_fmm = 30, n_max = 64, t_f = 0.9, FP64. One step evaluates the single-layer and the
double-layer potential of a Fourier-mode density (all FMM stages, densities resident in HBM) with
one gq_eval(GQ_S_AND_D) call (one expansion pipeline for both kinds, the direct interactions of
both kinds in one pass);
targets/s = 2 x 131072 / step time. Tree and list build is excluded and reported as build_ms.

Variants on the same geometry (reported under "variants", each with its own error against the
FP64 oracle at sampled targets):
  sequential_s_then_d  S and D as two calls on one stream (no overlap between the kinds)
  batched_64      64 densities per call (a block of right-hand sides), FP64, p_fmm 30
  mixed_fp32_p16  FP32 box expansions at p_fmm 16 (tolerance 1e-6)
  fp64_p16        all-FP64 at p_fmm 16, the equal-accuracy reference for mixed_fp32_p16
  fp64_p40        all-FP64 at p_fmm 40 (tolerance 1e-12)
  ragged_32       32 independent stars (1024..65536 nodes) in one batched context (one forest)
                  against 32 contexts evaluated one after another
  learned_orders_1e-10, _1e-12
                  per-center QBX orders from the shipped network on an 8 x 8 lattice of nearly
                  touching wavy curves (196608 targets), against the smallest uniform order
                  meeting the same tolerance (true error via Green's formula)

The JSON line also carries:
  roofline      the dominant kernel's achieved rate (algorithmic flops per launch / average launch
                time from HIP events recorded on the library's streams during the timed steps)
                against the FP64 vector peak;
  cpu_baseline  the CPU oracle (direct QBX, FP64) timed on a bounded sample of the same targets
                on this host; the same oracle values give the GPU-vs-oracle error of this run.

Usage: python bench.py [--gpus 1] [--steps 100] [--warmup 20] [--no-cpu-baseline] [--no-variants]
       python bench.py --copy-mib 256      (plain copy kernel, for HBM counter calibration)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QBX-FMM targets/s at 1e-10 rel err, plain vs batched/mixed/learned, 1 GPU"
GATE = 1e-10
# kernels of each stage in a GQ_S_AND_D evaluation of one density
KERNEL_OF_STAGE = {"near": "k_near_sd_t<4, 12>", "m2qbxl": "k_m2qbxl_packed", "qbx_center": "k_qbx_center",
                   "m2l_p2l": "k_m2l_mb", "m2m": "k_m_reduce", "l2l": "k_l2l_gather",
                   "p2m": "k_p2m_all", "gather": "k_gather", "finalize": "k_finalize"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def copy_calibration(mib: int, reps: int = 5):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} copies of {mib} MiB")


class Timer:
    """Times K steps with events on torch's current stream (the library's stream)."""

    def __init__(self):
        import torch
        self.torch = torch
        self.a = torch.cuda.Event(enable_timing=True)
        self.b = torch.cuda.Event(enable_timing=True)

    def run(self, q, step, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        q.stage_times()
        q.set_profiling(True)
        torch.cuda.synchronize()
        self.a.record()
        for _ in range(steps):
            step()
        self.b.record()
        torch.cuda.synchronize()
        ms = self.a.elapsed_time(self.b) / steps
        stages = q.stage_times()
        q.set_profiling(False)
        return ms, stages

    def run_plain(self, step, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        self.a.record()
        for _ in range(steps):
            step()
        self.b.record()
        torch.cuda.synchronize()
        return self.a.elapsed_time(self.b) / steps


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` (mean over its template instances) from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when the kernel sources have changed since
    the counters were taken."""
    from paper_1801_04070_amd import profsummary
    path = os.path.join(ROOT, "profiles", "hbm_traffic_c2.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except OSError:
        return None, "no counter summary"
    if t.get("kernel_sources_sha256") != profsummary.sources_sha256():
        return None, "kernel sources changed since the counters were taken"
    ks = [d for k, d in t["kernels"].items() if k.startswith(kernel + "<") or k == kernel]
    if not ks:
        return None, "kernel not in the counter summary"
    n = sum(d["dispatches"] for d in ks)
    return (round(sum(d["hbm_bytes"] * d["dispatches"] for d in ks) / n),
            "profiles/hbm_traffic_c2.json (FETCH_SIZE + WRITE_SIZE, copy-calibrated)")


def ragged_variant(timer, steps, warmup, n_geoms=32, p_qbx=12, p_fmm=30):
    """32 separate star geometries with log-uniform node counts 1024..65536 (seed 200): one
    batched context (a forest: every stage launched once for all geometries) against one context
    per geometry evaluated one after another. One step: S and D of one density per geometry."""
    import numpy as np
    import torch
    import gq_inputs as gi
    from paper_1801_04070_amd import GQ_D, GQ_S, QBXFMM
    geoms = gi.ragged_star_batch(n_geoms=n_geoms, seed=200)
    dens = [gi.fourier_density(g, seed=200 + i) for i, g in enumerate(geoms)]
    kw = dict(p_qbx=p_qbx, p_fmm=p_fmm)
    qb = QBXFMM(0)
    qb.set_geometry_batch(geoms)
    t0 = time.perf_counter()
    qb.build(**kw)
    build_s = time.perf_counter() - t0
    db = torch.as_tensor(np.concatenate(dens), device="cuda:0")
    ob = torch.empty((2, 1, qb.n_tgt), dtype=torch.float64, device="cuda:0")

    def step_b():
        qb.eval(GQ_S, db, out=ob[0])
        qb.eval(GQ_D, db, out=ob[1])

    ms_b = timer.run_plain(step_b, steps, warmup)
    _, st_b = timer.run(qb, step_b, min(steps, 5), 1)
    _, bd = per_stage(st_b, min(steps, 5))
    sep = []
    for g, d in zip(geoms, dens):
        q = QBXFMM(0)
        q.set_geometry_from(g)
        q.build(**kw)
        dd = torch.as_tensor(d, device="cuda:0")
        sep.append((q, dd, torch.empty((2, 1, g.n_tgt), dtype=torch.float64, device="cuda:0")))

    def step_s():
        for q, dd, o in sep:
            q.eval(GQ_S, dd, out=o[0])
            q.eval(GQ_D, dd, out=o[1])

    ms_s = timer.run_plain(step_s, steps, warmup)
    ref = torch.cat([o[:, 0] for _, _, o in sep], dim=1)
    diff = float((ob[:, 0] - ref).abs().max() / ref.abs().max())
    n_t = qb.n_tgt
    for q, _, _ in sep:
        q.close()
    qb.close()
    return {"value": round(2 * n_t / (ms_b * 1e-3), 1), "unit": "targets/s",
            "ms_per_step": round(ms_b, 4), "separate_ms_per_step": round(ms_s, 4),
            "separate_value": round(2 * n_t / (ms_s * 1e-3), 1),
            "speedup_vs_separate": round(ms_s / ms_b, 3), "max_rel_diff_vs_separate": diff,
            "n_geoms": n_geoms, "n_tgt": n_t, "build_s": round(build_s, 2), "steps": steps,
            "stage_ms_per_step": bd,
            "workload": f"{n_geoms} stars, 1024..65536 nodes each (log-uniform, seed 200), "
                        f"{n_t} targets, S and D, FP64, p_qbx {p_qbx}, p_fmm {p_fmm}"}


def learned_variant(timer, steps, warmup, log10_tol=-10.0, p_fmm=30, panels=192):
    """Learned per-center QBX orders against the smallest uniform order meeting the tolerance
    (found by trying the candidates against the exact solution) and against the configured
    uniform order p_qbx 12.

    Workload: 8 x 8 lattice of wavy curves (seed 300) whose neighbours nearly touch (gap of four
    expansion radii), `panels` panels x 16 nodes per curve (192: 196608 on-surface targets and
    393216 centers), sources upsampled to 64 nodes per panel (786432 sources). One step evaluates
    Green's formula S(du/dn) - D(u), u = log|x - x0| with x0 outside the lattice; the exact value
    at the targets is u / 2, so every error here is the true error relative to max |u|. (At 1024
    panels per curve the uniform order 4 already reaches 1e-12, leaving no order to save.)"""
    import numpy as np
    import torch
    import gq_inputs as gi
    from paper_1801_04070_amd import GQ_S_MINUS_D, QBXFMM, learned
    model = learned.load_default()
    if model is None:
        return {"status": "no shipped order model"}
    g = gi.wavy_lattice(nx=8, ny=8, panels_per_curve=panels, seed=300, gap_in_radii=4.0,
                        src_order=64)
    lo, hi = g.src_xy.min(0), g.src_xy.max(0)
    x0 = (lo[0] - 0.7, 0.3 * lo[1] + 0.7 * hi[1])
    sig, tau, u = gi.green_test_field(g, x0)
    q = QBXFMM(0)
    q.set_geometry_from(g)
    t0 = time.perf_counter()
    stats = q.build(p_qbx=max(model.candidates), p_fmm=p_fmm)
    build_s = time.perf_counter() - t0
    d1 = torch.as_tensor(sig, device="cuda:0")
    d2 = torch.as_tensor(tau, device="cuda:0")
    out = torch.empty((1, g.n_tgt), dtype=torch.float64, device="cuda:0")
    scale = float(np.abs(u).max())
    half_u = torch.as_tensor(0.5 * u, device="cuda:0")

    def step():
        q.eval(GQ_S_MINUS_D, d1, d2, out=out)

    def log10_err():
        step()
        return float(torch.log10((out[0] - half_u).abs().max() / scale))

    uniform = {}
    p_u = None
    for p in model.candidates:
        q.set_qbx_orders(np.full(g.n_ctr, p, np.int32))
        uniform[p] = round(log10_err(), 2)
        if uniform[p] <= log10_tol:
            p_u = p
            break
    if p_u is None:
        return {"status": "no uniform candidate order meets the tolerance", "uniform": uniform}
    ms_u = timer.run_plain(step, steps, warmup)
    _, st_u = timer.run(q, step, steps, 1)
    # the configured uniform order of the method (p_qbx 12, as in the 16-star workload), which a
    # user without the network runs; the smallest uniform order above needs the exact solution
    q.set_qbx_orders(np.full(g.n_ctr, 12, np.int32))
    e_12 = round(log10_err(), 2)
    ms_12 = timer.run_plain(step, steps, warmup)
    t0 = time.perf_counter()
    orders = learned.choose_orders(q, log10_tol, model)
    torch.cuda.synchronize()
    choose_s = time.perf_counter() - t0
    e_l = round(log10_err(), 2)
    ms_l = timer.run_plain(step, steps, warmup)
    _, st_l = timer.run(q, step, steps, 1)
    hist = torch.bincount(orders.long(), minlength=max(model.candidates) + 1).cpu().numpy()
    _, bd_u = per_stage(st_u, steps)
    _, bd_l = per_stage(st_l, steps)
    q.close()
    v_u = g.n_tgt / (ms_u * 1e-3)
    v_l = g.n_tgt / (ms_l * 1e-3)
    return {"value": round(v_l, 1), "unit": "targets/s", "ms_per_step": round(ms_l, 4),
            "uniform_value": round(v_u, 1), "uniform_ms_per_step": round(ms_u, 4),
            "speedup_vs_uniform": round(v_l / v_u, 3), "log10_tol": log10_tol,
            "configured_order_value": round(g.n_tgt / (ms_12 * 1e-3), 1),
            "configured_order_ms_per_step": round(ms_12, 4), "configured_order_log10_err": e_12,
            "speedup_vs_configured_order": round(ms_12 / ms_l, 3),
            "p_uniform": p_u, "uniform_log10_err": uniform, "learned_log10_err": e_l,
            "status": "ok" if e_l <= log10_tol else "FAILED",
            "learned_order_histogram": {int(p): int(hist[p]) for p in model.candidates},
            "choose_orders_s": round(choose_s, 3), "build_s": round(build_s, 1),
            "stage_ms_per_step_uniform": bd_u, "stage_ms_per_step_learned": bd_l,
            "steps": steps, "p_fmm": p_fmm,
            "learned_mean_order": round(float(orders.float().mean()), 3),
            "workload": f"8x8 wavy lattice (gap 4 radii), {panels} panels per curve, "
                        f"{g.n_tgt} targets, {g.n_ctr} centers, {g.n_src} upsampled sources, "
                        "Green's formula, FP64"}


def neumann_variant(timer, geom, n_rhs=8, p_qbx=12, p_fmm=30, tol=1e-10):
    """The exterior Neumann integral equation of Sec. 1 (-mu/2 + S' mu = g) on the 16-star
    workload: n_rhs manufactured problems (25 point charges inside every star, seeds 20..,
    Table 5's construction) solved together by GMRES, each iteration one batched GQ_SP
    evaluation of all right-hand sides; then S mu at the check points outside every star (a
    second context, point targets) against the manufactured field. Timed: the whole solve."""
    import copy as _copy
    import numpy as np
    import torch
    import gq_inputs as gi
    from paper_1801_04070_amd import GQ_S, QBXFMM
    from paper_1801_04070_amd.bie import gmres, neumann_operator
    probs = [gi.neumann_test_problem(geom, seed=20 + j) for j in range(n_rhs)]
    rhs = torch.as_tensor(np.stack([p[0] for p in probs]), device="cuda:0")
    q = QBXFMM(0)
    q.set_geometry_from(geom)
    q.build(p_qbx=p_qbx, p_fmm=p_fmm)
    q.set_target_normals(geom.src_nrm)
    op = neumann_operator(q)
    gmres(op, rhs, tol=tol, maxiter=3)  # warm-up (workspace, first launches)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, its, res = gmres(op, rhs, tol=tol, maxiter=60)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    ev = _copy.copy(geom)
    ev.tgt_xy = probs[0][1]
    ev.tgt_ctr = np.full((len(ev.tgt_xy), 2), -1, dtype=np.int32)
    qe = QBXFMM(0)
    qe.set_geometry_from(ev)
    qe.build(p_qbx=p_qbx, p_fmm=p_fmm)
    u = qe.eval(GQ_S, x).cpu().numpy()
    errs = [float(np.abs(u[j] - probs[j][2]).max() / np.abs(probs[j][2]).max())
            for j in range(n_rhs)]
    n_it = int(its.max())
    q.close()
    qe.close()
    return {"value": round(n_rhs * n_it * geom.n_tgt / sec, 1), "unit": "targets/s",
            "ms_per_solve": round(sec * 1e3, 2), "n_rhs": n_rhs,
            "gmres_iterations": [int(i) for i in its], "final_residuals": [float(r) for r in res],
            "bvp_rel_errors": errs, "n_check_points": int(len(ev.tgt_xy)),
            "workload": f"exterior Neumann equation, {n_rhs} right-hand sides by batched GMRES "
                        f"to {tol:g}, S' by GQ_SP (p_qbx {p_qbx}, p_fmm {p_fmm}); value = "
                        "right-hand sides x iterations x targets / solve time"}


def offsurface_variant(timer, geom, dens_h, args, n_side=384, p_qbx=12, p_fmm=30):
    """Targets on a regular grid over the 16-star workload's bounding box (n_side^2 points)
    instead of on the curves: gq_associate_targets (Sec. 2.2.2, 20 % slack, conventional beyond
    three radii) makes the grid points near the curves one-sided QBX targets and leaves the rest
    to the conventional paths (direct sum, multipole-to-point, local-to-point). One step: S and D
    of one density for all grid points. Parity: the oracle's QBX at the associated centers and
    its plain point sums at a sample."""
    import copy as _copy
    import numpy as np
    import torch
    import oracle
    from paper_1801_04070_amd import GQ_S_AND_D, QBXFMM, associate_targets
    lo, hi = geom.src_xy.min(0) - 0.5, geom.src_xy.max(0) + 0.5
    xs = np.linspace(lo[0], hi[0], n_side)
    ys = np.linspace(lo[1], hi[1], n_side)
    tgt = np.stack(np.meshgrid(xs, ys, indexing="ij"), -1).reshape(-1, 2)
    t0 = time.perf_counter()
    tc, n_gap = associate_targets(geom.ctr_xy, geom.ctr_r, tgt, slack=0.2, far_factor=3.0)
    assoc_s = time.perf_counter() - t0
    g = _copy.copy(geom)
    g.tgt_xy, g.tgt_ctr = tgt, tc
    q = QBXFMM(0)
    q.set_geometry_from(g)
    t0 = time.perf_counter()
    q.build(p_qbx=p_qbx, p_fmm=p_fmm)
    build_s = time.perf_counter() - t0
    d = torch.as_tensor(dens_h, device="cuda:0")
    out = torch.empty((2, len(tgt)), dtype=torch.float64, device="cuda:0")

    def step():
        q.eval(GQ_S_AND_D, d, out=out)

    ms = timer.run_plain(step, args.steps, args.warmup)
    _, st = timer.run(q, step, min(args.steps, 5), 1)
    _, bd = per_stage(st, min(args.steps, 5))
    res = out.cpu().numpy()
    q.close()
    qbx = tc[:, 0] >= 0
    r = {"value": round(2 * len(tgt) / (ms * 1e-3), 1), "unit": "targets/s",
         "ms_per_step": round(ms, 4), "steps": args.steps, "n_targets": int(len(tgt)),
         "n_qbx_targets": int(qbx.sum()), "n_conventional_targets": int((~qbx).sum()),
         "n_gap_targets": int(n_gap), "associate_s": round(assoc_s, 3),
         "build_s": round(build_s, 3), "stage_ms_per_step": bd,
         "workload": f"{n_side}x{n_side} grid over the 16-star workload, S and D, FP64, "
                     f"p_qbx {p_qbx}, p_fmm {p_fmm}"}
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(11)
        iq = rng.choice(np.nonzero(qbx)[0], 256, replace=False)
        ip = rng.choice(np.nonzero(~qbx)[0], 256, replace=False)
        err = {}
        for kind, row in ((1, 0), (2, 1)):
            ref_q = oracle.qbx_eval(geom, kind, dens_h, p_qbx=p_qbx, tgt_xy=tgt[iq], tgt_ctr=tc[iq])
            ref_p = oracle.point_potential(geom, kind, dens_h, tgt_xy=tgt[ip])
            err["SD"[kind - 1]] = max(float(np.abs(res[row, iq] - ref_q).max() / np.abs(ref_q).max()),
                                     float(np.abs(res[row, ip] - ref_p).max() / np.abs(ref_p).max()))
        err.update({"gate": GATE, "n_sampled_targets": 512})
        if max(err["S"], err["D"]) > GATE:
            err["status"] = "FAILED"
        r["parity"] = err
    return r


def per_stage(stages, steps):
    agg = {}
    for (kind, name), (ms, cnt) in stages.items():
        agg.setdefault(name, [0.0, 0])
        agg[name][0] += ms
        agg[name][1] += cnt
    return agg, {k: round(v[0] / steps, 4) for k, v in agg.items()}


def oracle_sample(geom, dens, budget_s: float, seed=123):
    """Oracle values (S and D) at a bounded random sample of targets, and the time it took."""
    import numpy as np
    import oracle
    from paper_1801_04070_amd import GQ_D, GQ_S

    order = np.random.default_rng(seed).permutation(geom.n_tgt)
    probe = order[:16]
    t0 = time.perf_counter()
    oracle.qbx_eval(geom, GQ_S, dens, p_qbx=12, tgt_xy=geom.tgt_xy[probe], tgt_ctr=geom.tgt_ctr[probe])
    per_target = (time.perf_counter() - t0) / len(probe)
    n = int(min(geom.n_tgt, max(64, budget_s / (2.5 * per_target))))
    idx = np.sort(order[:n])
    t0 = time.perf_counter()
    ref_s = oracle.qbx_eval(geom, GQ_S, dens, p_qbx=12, tgt_xy=geom.tgt_xy[idx],
                            tgt_ctr=geom.tgt_ctr[idx])
    ref_d = oracle.qbx_eval(geom, GQ_D, dens, p_qbx=12, tgt_xy=geom.tgt_xy[idx],
                            tgt_ctr=geom.tgt_ctr[idx])
    dt = time.perf_counter() - t0
    return {"idx": idx, "S": ref_s, "D": ref_d, "seconds": dt, "threads": oracle.num_threads()}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_errors(sample, out_s, out_d):
    import numpy as np
    i = sample["idx"]
    es = float(np.abs(out_s[i] - sample["S"]).max() / np.abs(sample["S"]).max())
    ed = float(np.abs(out_d[i] - sample["D"]).max() / np.abs(sample["D"]).max())
    return {"S": es, "D": ed, "n_sampled_targets": int(len(i))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the device reaches its steady clock only after some tens of steps: 20 untimed steps, then
    # 100 timed ones (about 40 ms)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--only", default="", help="comma-separated variant names: run only these")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--batch", type=int, default=64, help="densities of the batched variant")
    ap.add_argument("--overlap", type=int, default=1, choices=(0, 1),
                    help="run direct and List 3 far work on a second stream")
    ap.add_argument("--near-chunk", type=int, default=0, help="direct sources per work item")
    ap.add_argument("--far-chunk", type=int, default=0, help="List 3 far boxes per work item")
    ap.add_argument("--far-ppl", type=int, default=None,
                    help="List 3 far pairs per lane (gq_params.far_pairs_per_lane; default: the "
                         "library's, 1 = pairs packed across boxes)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_mib:
        copy_calibration(args.copy_mib)
        return

    import gq_inputs as gi
    from paper_1801_04070_amd import GQ_D, GQ_MIXED_FP32, GQ_S, GQ_S_AND_D, QBXFMM, perfmodel

    p_qbx, p_fmm = 12, 30
    log("bench: building the 16-star workload (131072 sources)")
    geom = gi.config_geometry("c2")
    dens_h = gi.fourier_density(geom, seed=2)
    dens = torch.as_tensor(dens_h, dtype=torch.float64, device="cuda:0")
    timer = Timer()

    def context(**kw):
        q = QBXFMM(device=0)
        q.set_geometry_from(geom)
        params = dict(p_qbx=p_qbx, p_fmm=p_fmm, n_max=64, count_mode=0, t_f=0.9,
                      w3far_min_sources=15, overlap=args.overlap, near_chunk=args.near_chunk,
                      far_chunk=args.far_chunk)
        if args.far_ppl is not None:
            params["far_pairs_per_lane"] = args.far_ppl
        params.update(kw)
        return q, q.build(**params)

    def sd_step(q, d, out):
        # S and D of the same densities in one call (the library runs the kinds concurrently);
        # out rows: S of every density, then D of every density
        def step():
            q.eval(GQ_S_AND_D, d, out=out)
        return step

    # ---- headline: plain FP64 ----
    q, stats = context()
    out = torch.empty((2, geom.n_tgt), dtype=torch.float64, device="cuda:0")
    # timed without stage events (they cost launches of their own); the stage breakdown and the
    # roofline come from a second timed region of the same steps with the ABI's stage profiling
    ms_per_step = timer.run_plain(sd_step(q, dens, out), args.steps, args.warmup)
    log(f"bench: plain {args.steps} steps, {ms_per_step:.3f} ms/step")
    ms_profiled, stages = timer.run(q, sd_step(q, dens, out), args.steps, 1)
    log(f"bench: with stage profiling {ms_profiled:.3f} ms/step")
    agg, breakdown = per_stage(stages, args.steps)
    n_slots = int((geom.tgt_ctr >= 0).sum())
    # each stage interval of a GQ_S_AND_D step covers the work of both kinds (kind 4 below)
    used = geom.tgt_ctr[geom.tgt_ctr >= 0]
    one_target = used.size == 0 or int(np.bincount(used).max()) <= 1
    work = perfmodel.stage_work(stats, 4, p_qbx, p_fmm, n_slots, near_values=one_target)
    dom = max(agg, key=lambda n: agg[n][0])
    ms_dom, n_dom = agg[dom]
    avg_ms = ms_dom / n_dom
    flops = work[dom]["flops"]
    nbytes = work[dom]["bytes"]
    peak = perfmodel.MI355X_PEAKS["fp64_vector_tflops"]
    achieved = flops / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": KERNEL_OF_STAGE[dom] + " (S and D of one density)",
                "timed_region": f"{args.steps} profiled steps (stage events on), "
                                f"{ms_profiled:.4f} ms/step",
                "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": int(flops),
                "algorithmic_bytes_per_launch": int(nbytes),
                "achieved_hbm_gbs": round(nbytes / (avg_ms * 1e-3) / 1e9, 1)}
    roofline["traffic"], roofline["traffic_source"] = measured_traffic(KERNEL_OF_STAGE[dom])
    # the same kernels with nothing else on the device: no side stream, one kernel at a time
    q_iso, _ = context(overlap=0)
    out_iso = torch.empty_like(out)
    _, st_iso = timer.run(q_iso, sd_step(q_iso, dens, out_iso), args.steps, 1)
    agg_iso, breakdown_iso = per_stage(st_iso, args.steps)
    q_iso.close()
    if dom in agg_iso:
        ms_i, n_i = agg_iso[dom]
        ach_i = flops / (ms_i / n_i * 1e-3) / 1e12
        roofline["isolated"] = {"timed_region": f"{args.steps} profiled steps, no side "
                                                "stream (one kernel at a time)",
                                "avg_launch_ms": round(ms_i / n_i, 4),
                                "achieved": round(ach_i, 3), "frac": round(ach_i / peak, 4)}
    stage_rates = {}
    for name, (ms, cnt) in agg.items():
        if name in work and cnt:
            stage_rates[name] = round(work[name]["flops"] / (ms / cnt * 1e-3) / 1e12, 3)
    value = 2 * geom.n_tgt / (ms_per_step * 1e-3)
    plain_out = out.cpu().numpy()
    # S then D as two calls on one stream (no concurrency between the kinds)
    out_seq = torch.empty_like(out)

    def seq_step():
        q.eval(GQ_S, dens, out=out_seq[0:1])
        q.eval(GQ_D, dens, out=out_seq[1:2])

    ms_seq = timer.run_plain(seq_step, args.steps, args.warmup)
    o_seq = out_seq.cpu().numpy()
    seq_diff = float(np.abs(o_seq - plain_out).max() / np.abs(plain_out).max())
    log(f"bench: S then D sequential {ms_seq:.3f} ms/step (max rel diff {seq_diff:.1e})")
    q.close()

    # ---- variants ----
    variants = {
                "sequential_s_then_d": {"value": round(2 * geom.n_tgt / (ms_seq * 1e-3), 1),
                                        "unit": "targets/s", "ms_per_step": round(ms_seq, 4),
                                        "steps": args.steps,
                                        "vs_plain": round(ms_per_step / ms_seq, 3),
                                        "max_rel_diff_to_plain": seq_diff,
                                        "workload": "S then D as two calls on one stream"}}
    outputs = {}
    if not args.no_variants:
        def want(name):
            return not args.only or name in args.only.split(",")

        def variant(name, workload, nd=1, graph=False, **kw):
            if not want(name):
                return
            qv, _ = context(**kw)
            if nd == 1:
                dv = dens
            else:
                hb = np.stack([gi.fourier_density(geom, seed=100 + j) for j in range(nd)])
                dv = torch.as_tensor(hb, dtype=torch.float64, device="cuda:0")
                outputs[name + "_density"] = hb[nd - 1]
            ov = torch.empty((2 * nd, geom.n_tgt), dtype=torch.float64, device="cuda:0")
            steps = max(2, args.steps // 4) if nd > 1 else args.steps
            # the stage breakdown from eager steps with stage events
            _, st = timer.run(qv, sd_step(qv, dv, ov), min(steps, 5), 1)
            _, bd = per_stage(st, min(steps, 5))
            if graph:
                # the evaluation captured once as a HIP graph and replayed (gq_graph_create)
                gr, ov = qv.graph(GQ_S_AND_D, dv)
                ms = timer.run_plain(gr.launch, steps, max(1, args.warmup))
            else:
                ms = timer.run_plain(sd_step(qv, dv, ov), steps, max(1, args.warmup))
            v = 2 * nd * geom.n_tgt / (ms * 1e-3)
            variants[name] = {"value": round(v, 1), "unit": "targets/s", "ms_per_step": round(ms, 4),
                              "steps": steps, "workload": workload, "hip_graph": graph,
                              "vs_plain": round(v / value, 3), "stage_ms_per_step": bd}
            torch.cuda.synchronize()
            outputs[name] = ov[[nd - 1, 2 * nd - 1]].cpu().numpy()
            if graph:
                gr.close()
            qv.close()
            log(f"bench: {name}: {ms:.3f} ms/step")

        nb = args.batch
        variant(f"batched_{nb}", f"{nb} seeded densities per call, S and D, FP64, p_fmm 30, "
                "replayed as a captured HIP graph", nd=nb, graph=True)
        variant(f"batched_{nb}_mixed_fp32_p16", f"{nb} densities, S and D, FP32 box expansions "
                "(FP32 matrix-core moments, P2L, M2L, gather), p_fmm 16, tolerance 1e-6, HIP graph",
                nd=nb, graph=True, p_fmm=16, precision=GQ_MIXED_FP32)
        variant(f"batched_{nb}_fp64_p16", f"{nb} densities, S and D, all FP64, p_fmm 16 "
                "(equal-accuracy reference), HIP graph", nd=nb, graph=True, p_fmm=16)
        variant("mixed_fp32_p16", "FP32 box expansions (FP32 matrix-core M2L and gather), p_fmm 16, "
                "tolerance 1e-6", p_fmm=16, precision=GQ_MIXED_FP32)
        variant("fp64_p16", "all FP64, p_fmm 16 (equal-accuracy reference for mixed_fp32_p16)",
                p_fmm=16)
        variant("fp64_p40", "all FP64, p_fmm 40, tolerance 1e-12", p_fmm=40)
        variant("level_restricted", "the tree refined until no leaf has an adjacent source leaf "
                "two levels coarser (Remark 2), S and D, FP64, p_fmm 30", level_restrict=1)
        variant("disk_tcr", "disk-shaped target confinement regions (the corrigendum's first "
                "experiments), S and D, FP64, p_fmm 30", tcr_shape=1)
        if want("offsurface"):
            log("bench: off-surface targets")
            variants["offsurface"] = offsurface_variant(timer, geom, dens_h, args)
            log(f"bench: offsurface: {variants['offsurface']['ms_per_step']} ms/step")
        if want("neumann_bie"):
            log("bench: exterior Neumann equation by batched GMRES")
            variants["neumann_bie"] = neumann_variant(timer, geom)
            log(f"bench: neumann_bie: {variants['neumann_bie']['ms_per_solve']} ms per solve, "
                f"{max(variants['neumann_bie']['gmres_iterations'])} iterations")
        if want("ragged_32"):
            log("bench: ragged batch of 32 geometries")
            variants["ragged_32"] = ragged_variant(timer, args.steps, args.warmup)
            log(f"bench: ragged batch: {variants['ragged_32']['speedup_vs_separate']}x vs separate")
        for tol in (-10.0, -12.0):
            name = f"learned_orders_1e{int(tol)}"
            if not want(name):
                continue
            log(f"bench: learned orders on the wavy lattice, tolerance 1e{int(tol)}")
            variants[name] = learned_variant(timer, max(2, args.steps // 4), max(1, args.warmup),
                                             log10_tol=tol)
            log(f"bench: {name}: {variants[name].get('speedup_vs_uniform')}x")
        # the learned-order workload as specified: 8 x 8 wavy curves, 1024 panels each
        # (1048576 targets, 2097152 centers, 4194304 upsampled sources), tolerance 1e-8
        if want("learned_orders_1e-8_1m"):
            log("bench: learned orders, 1048576-target wavy lattice, tolerance 1e-8")
            variants["learned_orders_1e-8_1m"] = learned_variant(timer, 3, 1, log10_tol=-8.0,
                                                                 panels=1024)
            log(f"bench: learned_orders_1e-8_1m: "
                f"{variants['learned_orders_1e-8_1m'].get('speedup_vs_uniform')}x")

    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "targets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain FP64 GIGAQBX, S and D, 16 random stars, 8192 panels x 16 "
                               "nodes = 131072 sources, p_qbx 12, p_fmm 30, n_max 64, t_f 0.9",
                   "variant": "plain", "n_src": geom.n_src, "n_tgt": geom.n_tgt,
                   "n_ctr": geom.n_ctr, "p_qbx": p_qbx, "p_fmm": p_fmm,
                   "boxes": stats["n_boxes"], "levels": stats["n_levels"],
                   "list2_pairs": stats["n_list2"], "near_pairs": stats["near_pairs"],
                   "list3_far_pairs": stats["list3_far_pairs"], "overlap": args.overlap,
                   "build_ms": round(stats["build_ms"], 1)},
        "variants": variants,
        "stage_ms_per_step": breakdown,
        "stage_ms_per_step_isolated": breakdown_iso,
        "stage_tflops": stage_rates,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        smp = oracle_sample(geom, dens_h, args.cpu_budget)
        n = len(smp["idx"])
        result["cpu_baseline"] = {
            "value": round(2 * n / smp["seconds"], 2), "unit": "targets/s",
            "cores": smp["threads"], "kind": "oracle",
            "host_cpus": os.cpu_count(), "cpu_model": cpu_model(),
            "sample": f"{n} random on-surface targets of the same workload, S and D, direct QBX "
                      f"(FP64, compensated sums, OpenMP over targets, {smp['threads']} threads "
                      f"as OMP_NUM_THREADS allows of {os.cpu_count()} host CPUs); "
                      f"{smp['seconds']:.1f} s"}
        par = rel_errors(smp, plain_out[0], plain_out[1])
        par["gate"] = GATE
        if max(par["S"], par["D"]) > GATE:
            par["status"] = "FAILED"
        result["parity"] = par
        gates = {"mixed_fp32_p16": 1e-6, "fp64_p16": 1e-6, "fp64_p40": 1e-12,
                 "level_restricted": GATE, "disk_tcr": GATE}
        for name, gate in gates.items():
            if name in outputs:
                e = rel_errors(smp, outputs[name][0], outputs[name][1])
                e["gate"] = gate
                if max(e["S"], e["D"]) > gate:
                    e["status"] = "FAILED"
                variants[name]["parity"] = e
        bname = f"batched_{args.batch}"
        if bname in outputs:
            # every batched variant's last density is the same seeded density
            smp_b = oracle_sample(geom, outputs[bname + "_density"], args.cpu_budget / 4, seed=7)
            for name, gate in ((bname, GATE), (bname + "_mixed_fp32_p16", 1e-6),
                               (bname + "_fp64_p16", 1e-6)):
                if name not in outputs:
                    continue
                e = rel_errors(smp_b, outputs[name][0], outputs[name][1])
                e["gate"] = gate
                if max(e["S"], e["D"]) > gate:
                    e["status"] = "FAILED"
                variants[name]["parity"] = e
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
