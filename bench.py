"""Throughput of the GIGAQBX FMM hot path on one MI355X.

Workload (default): 16 random star curves, 8192 panels x 16 Gauss-Legendre nodes = 131072
sources, two QBX centers per node (radius = half the panel arclength), 131072 on-surface targets,
p_qbx = 12, p_fmm = 30, n_max = 64, t_f = 0.9, FP64. One step evaluates the single-layer and the
double-layer potential of a Fourier-mode density (all FMM stages, densities resident in HBM);
targets/s = 2 x 131072 / step time. Tree and list build is excluded and reported as build_ms.

The JSON line also carries:
  roofline      the dominant kernel's achieved rate (algorithmic flops per launch / average launch
                time from HIP events recorded on the library's stream during the timed steps)
                against the FP64 vector peak;
  cpu_baseline  the CPU oracle (direct QBX, FP64) timed on a bounded sample of the same targets
                on this host, whose values also give the GPU-vs-oracle error of this run.

Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu-baseline]
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
KERNEL_OF_STAGE = {"near": "k_near", "m2qbxl": "k_m2qbxl", "qbx_center": "k_qbx_center",
                   "m2l_p2l": "k_far_local", "m2m": "k_m2m", "l2l": "k_l2l", "p2m": "k_p2m",
                   "gather": "k_gather", "finalize": "k_finalize"}


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


def cpu_baseline(geom, dens, gpu_out, budget_s: float):
    """Oracle on a bounded sample of targets: throughput on this host and GPU parity there."""
    import numpy as np
    import oracle
    from paper_1801_04070_amd import GQ_D, GQ_S

    rng = np.random.default_rng(123)
    order = rng.permutation(geom.n_tgt)
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
    err_s = float(np.abs(gpu_out[0][idx] - ref_s).max() / np.abs(ref_s).max())
    err_d = float(np.abs(gpu_out[1][idx] - ref_d).max() / np.abs(ref_d).max())
    cpu = {"value": 2 * n / dt, "unit": "targets/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{n} random on-surface targets of the same workload, S and D, direct QBX "
                     f"(FP64, compensated sums, OpenMP over targets); {dt:.1f} s"}
    return cpu, {"S": err_s, "D": err_d, "n_sampled_targets": n, "gate": GATE}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--batch", type=int, default=64, help="densities of the batched variant")
    ap.add_argument("--overlap", type=int, default=1, choices=(0, 1),
                    help="run direct and List 3 far work on a second stream")
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
    from paper_1801_04070_amd import GQ_D, GQ_S, QBXFMM, perfmodel

    p_qbx, p_fmm = 12, 30
    log("bench: building C2 workload (16 stars, 131072 sources)")
    geom = gi.config_geometry("c2")
    dens_h = gi.fourier_density(geom, seed=2)
    q = QBXFMM(device=0)
    q.set_geometry_from(geom)
    stats = q.build(p_qbx=p_qbx, p_fmm=p_fmm, n_max=64, count_mode=0, t_f=0.9,
                    w3far_min_sources=15, overlap=args.overlap)
    dens = torch.as_tensor(dens_h, dtype=torch.float64, device="cuda:0")
    out = torch.empty((2, geom.n_tgt), dtype=torch.float64, device="cuda:0")

    def step():
        q.eval(GQ_S, dens, out=out[0:1])
        q.eval(GQ_D, dens, out=out[1:2])

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    q.stage_times()
    q.set_profiling(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(stop) / args.steps
    stages = q.stage_times()
    q.set_profiling(False)
    log(f"bench: {args.steps} steps, {ms_per_step:.3f} ms/step")

    # dominant kernel and its roofline: algorithmic work per launch / average launch time
    per_stage = {}
    for (kind, name), (ms, cnt) in stages.items():
        per_stage.setdefault(name, [0.0, 0])
        per_stage[name][0] += ms
        per_stage[name][1] += cnt
    breakdown = {k: round(v[0] / args.steps, 4) for k, v in per_stage.items()}
    n_slots = int((geom.tgt_ctr >= 0).sum())
    work = {k: perfmodel.stage_work(stats, k, p_qbx, p_fmm, n_slots) for k in (GQ_S, GQ_D)}
    dom = max(per_stage, key=lambda n: per_stage[n][0])
    ms_dom, n_dom = per_stage[dom]
    avg_ms = ms_dom / n_dom
    flops = (work[GQ_S][dom]["flops"] + work[GQ_D][dom]["flops"]) / 2
    nbytes = (work[GQ_S][dom]["bytes"] + work[GQ_D][dom]["bytes"]) / 2
    peak = perfmodel.MI355X_PEAKS["fp64_vector_tflops"]
    achieved = flops / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": KERNEL_OF_STAGE[dom] + " (S and D launches)",
                "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": None,
                "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": int(flops),
                "algorithmic_bytes_per_launch": int(nbytes),
                "achieved_hbm_gbs": round(nbytes / (avg_ms * 1e-3) / 1e9, 1)}
    stage_rates = {}
    for name, (ms, cnt) in per_stage.items():
        if name in work[GQ_S] and cnt:
            f = (work[GQ_S][name]["flops"] + work[GQ_D][name]["flops"]) / 2
            stage_rates[name] = round(f / (ms / cnt * 1e-3) / 1e12, 3)

    value = 2 * geom.n_tgt / (ms_per_step * 1e-3)
    gpu_out = out.cpu().numpy()

    # batched variant: 64 seeded densities in one call per kind (a block right-hand-side batch)
    variants = {}
    if args.batch > 1:
        nb = args.batch
        hb = np.stack([gi.fourier_density(geom, seed=100 + j) for j in range(nb)])
        db = torch.as_tensor(hb, dtype=torch.float64, device="cuda:0")
        ob = torch.empty((2, nb, geom.n_tgt), dtype=torch.float64, device="cuda:0")

        def bstep():
            q.eval(GQ_S, db, out=ob[0])
            q.eval(GQ_D, db, out=ob[1])

        bsteps = max(2, args.steps // 4)
        for _ in range(max(1, args.warmup)):
            bstep()
        torch.cuda.synchronize()
        q.stage_times()
        q.set_profiling(True)
        start.record()
        for _ in range(bsteps):
            bstep()
        stop.record()
        torch.cuda.synchronize()
        bms = start.elapsed_time(stop) / bsteps
        bstages = {}
        for (kind, name), (ms, cnt) in q.stage_times().items():
            bstages[name] = round(bstages.get(name, 0.0) + ms / bsteps, 3)
        q.set_profiling(False)
        variants[f"batched_{nb}"] = {
            "value": round(2 * nb * geom.n_tgt / (bms * 1e-3), 1), "unit": "targets/s",
            "ms_per_step": round(bms, 4), "steps": bsteps,
            "workload": f"same geometry, {nb} seeded densities per call, S and D",
            "vs_plain": round(2 * nb * geom.n_tgt / (bms * 1e-3) / value, 3),
            "stage_ms_per_step": bstages}
        log(f"bench: batched {nb}: {bms:.3f} ms/step")
        batched_out = (ob[0, nb - 1].cpu().numpy(), ob[1, nb - 1].cpu().numpy(), hb[nb - 1])
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
        "stage_tflops": stage_rates,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a sample")
        cpu, parity = cpu_baseline(geom, dens_h, gpu_out, args.cpu_budget)
        result["cpu_baseline"] = cpu
        result["parity"] = parity
        if max(parity["S"], parity["D"]) > GATE:
            result["parity"]["status"] = "FAILED"
        if variants:
            _, bpar = cpu_baseline(geom, batched_out[2], batched_out[:2], args.cpu_budget / 4)
            key = next(iter(variants))
            variants[key]["parity"] = bpar
            if max(bpar["S"], bpar["D"]) > GATE:
                variants[key]["parity"]["status"] = "FAILED"
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
