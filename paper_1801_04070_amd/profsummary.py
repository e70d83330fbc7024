"""Summaries of rocprofv3 CSV output: per-kernel launch statistics and HBM traffic per dispatch.

Usage (after the profiling runs, from the repo root):
  python -m paper_1801_04070_amd.profsummary stats  <kernel_stats.csv> [--top 20]
  python -m paper_1801_04070_amd.profsummary pmc    <counter_collection.csv> [--top 20]
  python -m paper_1801_04070_amd.profsummary traffic --fetch F.csv --write W.csv \
        --copy-fetch CF.csv --copy-write CW.csv --copy-mib 256 --out traffic.json
  python -m paper_1801_04070_amd.profsummary mfma --trace <kernel_trace.csv> \
        --pmc <counter_collection.csv> [--after KERNEL]
  python -m paper_1801_04070_amd.profsummary window <kernel_trace.csv> --after KERNEL [--top 20]

``mfma`` reads SQ_INSTS_VALU_MFMA_MOPS_F64 / _F32 (units of 512 flops) per dispatch from one run
and the launch durations from a kernel trace of the same workload in another, and prints the
executed matrix-core flops and rate of every kernel that has them. With --after, only the
dispatches after the last one of KERNEL count in either file (a later phase of the run).

FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch. ``traffic`` calibrates them with a plain
device copy of known size (bytes read = bytes written = copy size): the factors are
copy bytes / counter bytes of the copy kernel, applied to every other kernel. The JSON records
the SHA-256 of the kernel sources at the time, so a reader can tell when the numbers are stale.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "kernels.hpp",
                                                           "cplx.hpp", "mlp.hip", "orders.hip")]


def sources_sha256() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """'void gq::(anonymous namespace)::k_near<1, 12>(int, ...)' -> 'k_near<1, 12>'."""
    n = name.strip().strip('"')
    n = re.sub(r"^void\s+", "", n)
    depth, cut = 0, len(n)
    for i, ch in enumerate(n):            # drop the argument list (first '(' outside <...>)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and not n[i:].startswith("(anonymous"):
            cut = i
            break
    n = n[:cut]
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"^(gq::|at::native::)", "", n)
    return n


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(f"none of {names} in {list(row)}")


def kernel_stats(path):
    out = []
    for r in _rows(path):
        out.append({"kernel": short_name(_col(r, "Name", "KernelName", "Kernel_Name")),
                    "calls": int(_col(r, "Calls")),
                    "total_ms": float(_col(r, "TotalDurationNs")) * 1e-6,
                    "avg_us": float(_col(r, "AverageNs")) * 1e-3,
                    "pct": float(_col(r, "Percentage"))})
    return sorted(out, key=lambda d: -d["total_ms"])


def counter_per_kernel(path, counter: str):
    """{kernel: (mean value per dispatch, dispatches)} for one counter (summed over agents)."""
    per = defaultdict(lambda: defaultdict(float))
    for r in _rows(path):
        if _col(r, "Counter_Name") != counter:
            continue
        k = short_name(_col(r, "Kernel_Name"))
        per[k][_col(r, "Dispatch_Id")] += float(_col(r, "Counter_Value"))
    return {k: (sum(v.values()) / len(v), len(v)) for k, v in per.items()}


def _copy_kernel(d):
    cands = [k for k in d if "copy" in k.lower() or "elementwise" in k.lower()]
    if not cands:
        raise SystemExit("no copy kernel in the calibration run")
    return max(cands, key=lambda k: d[k][0] * d[k][1])


def traffic(fetch, write, copy_fetch, copy_write, copy_mib):
    f, w = counter_per_kernel(fetch, "FETCH_SIZE"), counter_per_kernel(write, "WRITE_SIZE")
    cf, cw = counter_per_kernel(copy_fetch, "FETCH_SIZE"), counter_per_kernel(copy_write,
                                                                             "WRITE_SIZE")
    nbytes = copy_mib * (1 << 20)
    kf, kw = _copy_kernel(cf), _copy_kernel(cw)
    sf = nbytes / (cf[kf][0] * 1024.0)
    sw = nbytes / (cw[kw][0] * 1024.0)
    kernels = {}
    for k in sorted(set(f) | set(w)):
        fk = f.get(k, (0.0, 0))[0] * 1024.0 * sf
        wk = w.get(k, (0.0, 0))[0] * 1024.0 * sw
        kernels[k] = {"fetch_bytes": round(fk), "write_bytes": round(wk),
                      "hbm_bytes": round(fk + wk),
                      "dispatches": max(f.get(k, (0, 0))[1], w.get(k, (0, 0))[1])}
    return {"fetch_scale": sf, "write_scale": sw, "copy_kernel": kf, "copy_mib": copy_mib,
            "kernel_sources_sha256": sources_sha256(), "kernels": kernels}


PEAK_TFLOPS = {"SQ_INSTS_VALU_MFMA_MOPS_F64": 78.6, "SQ_INSTS_VALU_MFMA_MOPS_F32": 157.3}


def _after(rows, kernel, key):
    """Rows whose key (dispatch id or start time) follows the last dispatch of ``kernel``."""
    if not kernel:
        return rows
    last = max((int(_col(r, key)) for r in rows if short_name(_col(r, "Kernel_Name")) == kernel),
               default=-1)
    return [r for r in rows if int(_col(r, key)) > last]


def mfma_rates(trace, pmc, after=None):
    tr = _after(_rows(trace), after, "Start_Timestamp")
    dur = defaultdict(list)
    for r in tr:
        dur[short_name(_col(r, "Kernel_Name"))].append(
            (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) * 1e-9)
    per = defaultdict(lambda: defaultdict(float))
    for r in _after(_rows(pmc), after, "Dispatch_Id"):
        cn = _col(r, "Counter_Name")
        if cn in PEAK_TFLOPS:
            per[(short_name(_col(r, "Kernel_Name")), cn)][_col(r, "Dispatch_Id")] += \
                float(_col(r, "Counter_Value"))
    out = []
    for (k, cn), v in per.items():
        fl = sum(v.values()) / len(v) * 512.0
        if fl == 0 or not dur.get(k):
            continue
        d = sum(dur[k]) / len(dur[k])
        out.append({"kernel": k, "counter": cn, "launches": len(dur[k]), "avg_ms": d * 1e3,
                    "gflop": fl / 1e9, "tflops": fl / d / 1e12,
                    "frac": fl / d / 1e12 / PEAK_TFLOPS[cn]})
    return sorted(out, key=lambda x: -x["gflop"] * x["launches"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--top", type=int, default=25)
    b = sub.add_parser("pmc")
    b.add_argument("csv")
    b.add_argument("--counter", default=None)
    b.add_argument("--top", type=int, default=25)
    c = sub.add_parser("traffic")
    for n in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--out"):
        c.add_argument(n, required=True)
    c.add_argument("--copy-mib", type=int, required=True)
    wdw = sub.add_parser("window")
    wdw.add_argument("csv")
    wdw.add_argument("--after", required=True)
    wdw.add_argument("--top", type=int, default=25)
    m = sub.add_parser("mfma")
    m.add_argument("--trace", required=True)
    m.add_argument("--pmc", required=True)
    m.add_argument("--after", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        rows = kernel_stats(args.csv)
        print(f"{'kernel':58s} {'calls':>6s} {'total ms':>10s} {'avg us':>9s} {'%':>6s}")
        for d in rows[:args.top]:
            print(f"{d['kernel'][:58]:58s} {d['calls']:6d} {d['total_ms']:10.3f} "
                  f"{d['avg_us']:9.2f} {d['pct']:6.2f}")
    elif args.cmd == "pmc":
        names = {r["Counter_Name"] for r in _rows(args.csv)}
        for cn in sorted(names if args.counter is None else [args.counter]):
            d = counter_per_kernel(args.csv, cn)
            print(f"== {cn} (mean per dispatch)")
            for k, (v, n) in sorted(d.items(), key=lambda kv: -kv[1][0] * kv[1][1])[:args.top]:
                print(f"{k[:58]:58s} {v:14.1f} x{n}")
    elif args.cmd == "window":
        per = defaultdict(list)
        for r in _after(_rows(args.csv), args.after, "Start_Timestamp"):
            per[short_name(_col(r, "Kernel_Name"))].append(
                (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) * 1e-6)
        tot = sum(sum(v) for v in per.values())
        print(f"{'kernel':58s} {'calls':>6s} {'total ms':>10s} {'avg us':>9s} {'%':>6s}")
        for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:args.top]:
            print(f"{k[:58]:58s} {len(v):6d} {sum(v):10.3f} {sum(v) / len(v) * 1e3:9.2f} "
                  f"{100 * sum(v) / tot:6.2f}")
    elif args.cmd == "mfma":
        print(f"{'kernel':50s} {'launches':>8s} {'avg ms':>8s} {'GFLOP':>8s} {'TF/s':>7s} "
              f"{'of peak':>7s}")
        for d in mfma_rates(args.trace, args.pmc, args.after):
            prec = "f64" if d["counter"].endswith("F64") else "f32"
            print(f"{d['kernel'][:46]:46s} {prec} {d['launches']:8d} {d['avg_ms']:8.3f} "
                  f"{d['gflop']:8.2f} {d['tflops']:7.1f} {d['frac']:7.3f}")
    else:
        t = traffic(args.fetch, args.write, args.copy_fetch, args.copy_write, args.copy_mib)
        with open(args.out, "w") as f:
            json.dump(t, f, indent=1, sort_keys=True)
        print(f"fetch scale {t['fetch_scale']:.3f}, write scale {t['write_scale']:.3f}")
        for k, d in sorted(t["kernels"].items(), key=lambda kv: -kv[1]["hbm_bytes"])[:20]:
            print(f"{k[:58]:58s} fetch {d['fetch_bytes'] / 1e6:10.2f} MB  write "
                  f"{d['write_bytes'] / 1e6:10.2f} MB  x{d['dispatches']}")


if __name__ == "__main__":
    sys.exit(main())
