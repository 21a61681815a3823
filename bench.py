"""Benchmark: tree-build particles/s at N = 2^24 (Plummer, n_leaf 16, FP64 moments)
and the achieved HBM bandwidth of the dominant kernel against the MI355X peak.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision fp64|mixed]

One step = one complete build (keys, sort, leaves, parents, moments) of a
resident synthetic particle set.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
METRIC = "tree-build particles/sec at N=2^24 + achieved HBM GB/s fraction of peak"

WORKLOADS = {
    "plummer16m": "N=2^24 Plummer sphere (a=1, r<50) normalised into the unit cube, equal masses, "
                  "n_leaf=16",
    "uniform64k": "N=65,536 uniform in the unit cube, equal masses, n_leaf=16",
    "clustered64m": "N=2^26 clustered (70% in 2000 NFW halos, 30% uniform), periodic unit box, "
                    "n_leaf=8",
    "mixed16m": "N=2^24 clustered set with log-normal masses, n_leaf=8",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer16m", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--sort-config", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 22,
                    help="particles of the workload the oracle builds for the CPU baseline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of 256 MiB (to scale HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """Five plain device-to-device copies of 2^28 bytes each: a kernel whose HBM
    traffic is known exactly (2^28 read + 2^28 written per launch), to scale the
    FETCH_SIZE / WRITE_SIZE counters of the build kernels."""
    import torch
    src = torch.empty(1 << 26, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": 1 << 28, "launches": 5}))


def algorithmic_bytes(n: int, cells: int, leaves: int, passes: int, precision: str) -> dict:
    """Bytes each stage must move (reads + writes), not counter traffic.

    keygen      read pos 12 + write key 8 per particle
    sort_pass   read key 8 (+ payload 4 after the first pass) + write key 8 + payload 4
    cell_count  read sorted key 8
    cell_emit   read sorted key 8 + perm 4 + gathered pos/mass 16 per particle; write
                key 8 + depth 1 + first 4 + child 8 per cell and count 4 + moments per leaf
    parents     per internal cell: read its children's key 8 + count 4 + moments,
                write its own count 4 + child count 4 + moments
    """
    mom = 80 if precision == "fp64" else 40
    inner = cells - leaves
    return {
        "keygen": 20 * n,
        "sort_pass": (20 + 24 * (passes - 1)) * n,
        "cell_count": 8 * n,
        "cell_emit": 28 * n + 21 * cells + (4 + mom) * leaves,
        "parents": (12 + mom) * max(cells - 1, 0) + (8 + mom) * inner,
    }


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2312_06102_amd import datagen as dg
    from paper_2312_06102_amd import treebuild as tb

    t_gen = time.time()
    pos_np, mass_np, n_leaf = dg.workload(args.workload)
    n = pos_np.shape[0]
    print(f"[bench] generated {args.workload} N={n} in {time.time() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    mass = torch.from_numpy(mass_np).to(dev)
    box = ((0.0, 0.0, 0.0), 1.0)
    b = tb.Builder(n, n_leaf, args.precision, args.sort_config, dev)
    passes = (63 + tb.tb_sort_configs()[args.sort_config][0] - 1) // tb.tb_sort_configs()[args.sort_config][0]

    for _ in range(args.warmup):
        b.launch(pos, mass, box)
    res = b.result()
    cells = res["n_cells"]
    leaves = int((res["child_ptr"][:, 0] < 0).sum().item())

    # timed region: K complete builds
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.launch(pos, mass, box)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    print(f"[bench] {args.steps} builds, {sec * 1e3:.3f} ms/build", file=sys.stderr, flush=True)

    # per-kernel durations from HIP events recorded on the build stream
    tb.tb_trace_enable(True)
    for _ in range(args.steps):
        b.launch(pos, mass, box)
    torch.cuda.synchronize()
    trace = tb.tb_trace_read()
    tb.tb_trace_enable(False)

    alg = algorithmic_bytes(n, cells, leaves, passes, args.precision)
    kernels = {}
    for name, (launches, total_ms) in sorted(trace.items()):
        per_build_ms = total_ms / args.steps
        k = {"ms_per_build": round(per_build_ms, 4), "launches_per_build": launches // args.steps,
             "avg_launch_ms": round(total_ms / max(launches, 1), 5)}
        if name in alg:
            k["alg_bytes_per_build"] = alg[name]
            k["alg_GBps"] = round(alg[name] / (per_build_ms * 1e-3) / 1e9, 1)
        kernels[name] = k
    sp = trace["sort_pass"]
    sort_avg_ms = sp[1] / sp[0]
    sort_bytes_per_launch = alg["sort_pass"] / passes
    achieved = sort_bytes_per_launch / (sort_avg_ms * 1e-3) / 1e9
    total_alg = sum(alg.values())
    traced_ms = sum(v[1] for v in trace.values()) / args.steps

    line = {
        "metric": METRIC,
        "value": n / sec,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 keys + f64 moments" if args.precision == "fp64" else "u64 keys + f32 moments",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "N": n,
                   "n_leaf": n_leaf, "precision": args.precision, "box": "unit cube",
                   "sort_config": list(tb.tb_sort_configs()[args.sort_config]),
                   "cells": cells, "leaves": leaves},
        "roofline": {"kernel": "sort_pass (radix scatter pass, one launch per digit)",
                     "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None,
                     "alg_bytes_per_launch": sort_bytes_per_launch,
                     "avg_launch_ms": round(sort_avg_ms, 5)},
        "build_alg_GBps": round(total_alg / sec / 1e9, 1),
        "build_alg_frac": round(total_alg / sec / 1e9 / HBM_PEAK_GBPS, 4),
        "traced_ms_per_build": round(traced_ms, 4),
        "kernels": kernels,
    }

    if not args.no_cpu_baseline:
        import oracle
        m = min(args.cpu_sample, n)
        sub_p = np.ascontiguousarray(pos_np[:m])
        sub_m = np.ascontiguousarray(mass_np[:m])
        oracle.load()
        tc0 = time.perf_counter()
        oracle.build(sub_p, sub_m, n_leaf)
        tc1 = time.perf_counter()
        line["cpu_baseline"] = {
            "value": m / (tc1 - tc0), "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} particles of the same workload, full oracle build "
                      f"(keys, top-down insertion, perm, canonical order, direct FP64 moments), "
                      f"{tc1 - tc0:.2f} s on {platform.processor() or platform.machine()} "
                      f"(host nproc={os.cpu_count()})"}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
