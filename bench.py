"""Benchmark: tree-build particles/s at N = 2^24 (Plummer, n_leaf 16, FP64 moments)
and the achieved HBM bandwidth of the dominant kernel against the MI355X peak.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--precision fp64|mixed]

One step = one complete build (keys, sort, leaves, parents, moments) of a
resident synthetic particle set; for the batched workload one step = one build
of all 4,096 sets.  Prints one JSON line.

Workloads
  plummer16m    N = 2^24 Plummer, n_leaf 16, FP64 (default: the headline line)
  uniform64k    N = 65,536 uniform, n_leaf 16 (latency-bound; parity size)
  clustered64m  N = 2^26 clustered halos, n_leaf 8
  mixed16m      N = 2^24 clustered, log-normal masses, n_leaf 8: the mixed-precision
                path timed, beside the FP64 path on the same data, with the
                per-moment error of mixed against FP64
  batched4096   4,096 Plummer sets, sizes log-uniform in [256, 262144], n_leaf 16:
                one graph-captured batch per step, beside eager batches and 4,096
                sequential single-set builds; the sort shape comes from the autotuner
  disk16m       N = 2^24 thin exponential disk, n_leaf 16

    python bench.py --sim plummer|disk [--sim-n N] [--steps K]

runs leapfrog steps instead (build, reorder, walk, kick-drift per step; the
paper's own methodology) and reports per-phase times with the particles
reordered every step and every tenth step.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
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
    "mixed16m": "N=2^24 clustered set (2000 NFW halos + 30% uniform) with log-normal masses, "
                "n_leaf=8, mixed-precision moments vs FP64",
    "disk16m": "N=2^24 exponential disk (scale length h, sech^2 height 0.1 h, R < 10 h) "
               "normalised into the unit cube, equal masses, n_leaf=16",
    "batched4096": "4096 independent Plummer sets, sizes floor(exp(U(ln 256, ln 262144))), each in "
                   "its own unit cube, masses 1/n_b, n_leaf=16, one graph-captured batch",
}

# profiles/pmc_<workload>.json holds per-launch HBM counter bytes measured with
# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, scaled by a copy-kernel calibration,
# together with a hash of the kernel sources they were taken on.
PROFILES = os.path.join(ROOT, "profiles")
SOURCES = sorted(glob.glob(os.path.join(ROOT, "paper_2312_06102_amd", "csrc", "*"))) + \
    [os.path.join(ROOT, "include", "treebuild.h")]

def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="plummer16m", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: mixed for mixed16m, fp64 otherwise")
    ap.add_argument("--sort-config", type=int, default=None,
                    help="sort shape index (default: 0; the autotuner's choice for batched4096)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true",
                    help="batched4096: skip the 4096 sequential single-set builds")
    ap.add_argument("--no-compare", action="store_true",
                    help="mixed16m: skip the FP64 build on the same data; single sets: skip "
                         "timing the subtree-rooted cell build on the same data")
    ap.add_argument("--sort-counted", action="store_true",
                    help="count the tiles' digits in every radix pass (TB_SORT_COUNTED)")
    ap.add_argument("--sort-lookback", action="store_true",
                    help="keep the decoupled look-back in every radix pass (TB_SORT_LOOKBACK)")
    ap.add_argument("--curve", default="morton", choices=["morton", "hilbert"],
                    help="particle keys: Morton (default) or Peano-Hilbert (TB_HILBERT)")
    ap.add_argument("--subtrees", action="store_true",
                    help="time the subtree-rooted cell build (TB_SUBTREES) as the step")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="particles of the workload the oracle builds for the CPU baseline "
                         "(default: all of a single set up to 2^24, the first 2^24 of a larger "
                         "one, whole sets up to 2^22 particles of a batch)")
    ap.add_argument("--sim", choices=["plummer", "disk"], default=None,
                    help="time leapfrog steps of an N-body run (build + walk per step) instead")
    ap.add_argument("--sim-n", type=int, default=1 << 22, help="particles of the --sim run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of 256 MiB (to scale HBM byte counters)")
    ap.add_argument("--gather-calibration", action="store_true",
                    help="only run random-row gathers of 16-B and of 128-B rows (2^28 bytes each), "
                         "to check the counter scale on gathers")
    ap.add_argument("--summarize-trace", metavar="CSV",
                    help="write profiles/build_<workload>_kernel_trace.md from a rocprofv3 "
                         "--kernel-trace CSV (with --profile-command and --builds)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH", "WRITE", "COPYF", "COPYW"),
                    help="write profiles/pmc_<workload>.json and its .md from rocprofv3 --pmc "
                         "FETCH_SIZE / WRITE_SIZE CSVs of the build and of --copy-calibration")
    ap.add_argument("--summarize-sq", metavar="CSV",
                    help="write profiles/sort_<workload>_sq_counters.md from a rocprofv3 --pmc CSV "
                         "of SQ counters (with --profile-command)")
    ap.add_argument("--gather-csv", default=None,
                    help="with --summarize-pmc: FETCH_SIZE CSV of --gather-calibration")
    ap.add_argument("--profile-command", default="", help="command line recorded in a summary")
    ap.add_argument("--builds", type=int, default=0, help="builds in the profiled run")
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


def gather_calibration():
    """Random-row gathers of 2^28 bytes, rows of 16 B (as the reorder's records)
    and of 128 B (one cache line each), five of each: the first shows the line
    amplification of 16-byte gathers, the second checks the counter scale on
    random whole-line reads."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(7)
    for width in (4, 32):
        rows = (1 << 26) // width
        src = torch.rand((rows, width), device="cuda:0")
        idx = torch.randperm(rows, generator=g).to("cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            torch.index_select(src, 0, idx, out=dst)
        torch.cuda.synchronize()
        del src, dst, idx
    print(json.dumps({"gather_calibration_bytes_per_launch": 1 << 28, "row_bytes": [16, 128],
                      "launches": 5}))


def _short_kernel(name: str) -> str:
    """'void tb::k_onesweep<8, 11, 512, 2, 2, false>(...)' -> 'k_onesweep<8, 11, 512, 2, 2, false>'."""
    n = name.split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    return n.replace("tb::", "").strip()


STAGE_OF = [("k_onesweep", "sort_pass"), ("k_tile_count", "sort_pass"),
            ("k_tile_scan", "sort_pass"), ("k_keygen", "keygen"), ("k_hist_reduce", "hist_reduce"),
            ("k_set_base", "hist_reduce"), ("k_set_sums", "cell_scan"),
            ("k_reorder", "reorder"), ("k_cell_emit", "cell_emit"), ("k_cell_scan", "cell_scan"),
            ("k_set_scan", "cell_scan"), ("k_parents", "parents"), ("k_init", "init"),
            ("k_setup", "setup"), ("k_tile_map", "setup"), ("k_bbox", "bbox"),
            ("k_blocks", "blocks"), ("k_block_build", "block_build"), ("k_upper", "upper")]


def _stage(kernel: str):
    for prefix, st in STAGE_OF:
        if kernel.startswith(prefix):
            return st
    return None


def _read_csv(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


SQ_CLOCK_GHZ = 2.4  # MI355X engine clock; SQ_WAVE_CYCLES counts in units of 4 cycles


def summarize_sq(args):
    """Markdown table of SQ instruction counters per library kernel: the mean per
    dispatch of every counter, and per wave the VALU and LDS instructions and the
    wave's life (SQ_WAVE_CYCLES x 4 cycles over the waves, at 2.4 GHz)."""
    rows = _read_csv(args.summarize_sq)
    per = {}
    for r in rows:
        k = _short_kernel(r["Kernel_Name"])
        if _stage(k) is None:
            continue
        d = per.setdefault(k, {"dispatches": set(), "waves": {}, "ctr": {}})
        did = r["Dispatch_Id"]
        d["dispatches"].add(did)
        d["waves"][did] = int(r["Grid_Size"]) // 64
        d["ctr"].setdefault(r["Counter_Name"], {})[did] = float(r["Counter_Value"])
    names = sorted({c for d in per.values() for c in d["ctr"]})
    out = [f"# SQ instruction counters: {args.workload}", "",
           "Command (on the GPU host, repository root as `<repo>`):", "",
           f"    {args.profile_command}", "",
           "Mean per dispatch (values summed over the chip as rocprofv3 reports them); per "
           "wave: the mean over dispatches of counter / waves of the dispatch; wave life = "
           f"SQ_WAVE_CYCLES x 4 cycles / waves at {SQ_CLOCK_GHZ} GHz.", "",
           "| kernel | dispatches | " + " | ".join(n.replace("SQ_", "") for n in names)
           + " | VALU / wave | LDS / wave | wave life us |",
           "|---|---|" + "---|" * len(names) + "---|---|---|"]
    order = sorted(per.items(), key=lambda kv: -sum(kv[1]["ctr"].get("SQ_WAVE_CYCLES", {}).values()))
    for k, d in order:
        disp = sorted(d["dispatches"])
        means = [sum(d["ctr"].get(n, {}).values()) / len(disp) for n in names]

        def per_wave(name):
            v = d["ctr"].get(name, {})
            xs = [v[i] / d["waves"][i] for i in disp if i in v and d["waves"][i]]
            return sum(xs) / len(xs) if xs else float("nan")
        life = per_wave("SQ_WAVE_CYCLES") * 4 / (SQ_CLOCK_GHZ * 1e3)
        out.append(f"| {k} | {len(disp)} | " + " | ".join(f"{m:.3g}" for m in means)
                   + f" | {per_wave('SQ_INSTS_VALU'):.0f} | {per_wave('SQ_INSTS_LDS'):.0f} | "
                   f"{life:.2f} |")
    path = os.path.join(PROFILES, f"sort_{args.workload}_sq_counters.md")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print(path)


def summarize_trace(args):
    """Markdown table of a rocprofv3 kernel trace: library kernels only."""
    rows = _read_csv(args.summarize_trace)
    agg = {}
    for r in rows:
        k = _short_kernel(r["Kernel_Name"])
        if _stage(k) is None:
            continue
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0
        a = agg.setdefault(k, {"calls": 0, "tot": 0.0, "min": 1e30, "max": 0.0, "grid": 0,
                               "wg": 0, "lds": 0, "vgpr": 0})
        a["calls"] += 1
        a["tot"] += d
        a["min"] = min(a["min"], d)
        a["max"] = max(a["max"], d)
        wg = int(r.get("Workgroup_Size_X") or r.get("Workgroup_Size") or 0)
        grid = int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)
        a["wg"] = wg
        a["grid"] = max(a["grid"], grid // max(wg, 1))
        a["lds"] = int(r.get("Group_Segment_Size") or r.get("LDS_Block_Size") or 0)
        a["vgpr"] = int(r.get("Arch_VGPR_Count") or r.get("VGPR_Count") or 0)
    total = sum(a["tot"] for a in agg.values())
    # one key-generation launch per build
    b = args.builds or sum(a["calls"] for k, a in agg.items() if k.startswith("k_keygen")) or 1
    args.builds = b
    lines = [f"# Kernel trace: {args.workload} ({WORKLOADS.get(args.workload, '')})", "",
             "Command (on the GPU host, repository root as `<repo>`):", "",
             f"    {args.profile_command}", "",
             f"{args.builds} builds traced. Durations in microseconds; library kernels only "
             "(grid: the largest launch, in workgroups).", "",
             "| kernel | stage | calls | per build | total us | avg us | min us | max us | share "
             "| grid (WGs) | WG | static LDS B | VGPR |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["tot"]):
        lines.append(f"| {k} | {_stage(k)} | {a['calls']} | {a['calls'] / b:g} | {a['tot']:.1f} | "
                     f"{a['tot'] / a['calls']:.2f} | {a['min']:.2f} | {a['max']:.2f} | "
                     f"{100 * a['tot'] / total:.1f}% | {a['grid']} | {a['wg']} | {a['lds']} | "
                     f"{a['vgpr']} |")
    st = {}
    for k, a in agg.items():
        st[_stage(k)] = st.get(_stage(k), 0.0) + a["tot"]
    lines += ["", "Per build by stage (us): " + ", ".join(
        f"{k} {v / b:.1f}" for k, v in sorted(st.items(), key=lambda kv: -kv[1])) + ".",
              f"Sum of library kernel time per build: {total / b:.1f} us."]
    if "sort_pass" in st:
        n_pass = sum(a["calls"] for k, a in agg.items() if k.startswith("k_onesweep")
                     and _stage(k) == "sort_pass") / b
        lines.append(f"Sort passes (scatter + the count and scan of counted passes): "
                     f"{st['sort_pass'] / b:.1f} us per build, {st['sort_pass'] / b / max(n_pass, 1):.1f} "
                     f"us per pass over {n_pass:g} passes.")
    out = os.path.join(PROFILES, f"build_{args.workload}_kernel_trace.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def summarize_pmc(args):
    """Per-stage HBM bytes per launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
    scaled by the same counters on --copy-calibration (2^28 bytes read and written)."""
    fetch, write, copyf, copyw = (_read_csv(p) for p in args.summarize_pmc)

    def per_kernel(rows, counter):
        out = {}
        for r in rows:
            if r.get("Counter_Name") != counter:
                continue
            k = _short_kernel(r["Kernel_Name"])
            out.setdefault(k, []).append(float(r["Counter_Value"]) * 1024.0)
        return out

    def copy_bytes(rows, counter):
        vals = [float(r["Counter_Value"]) * 1024.0 for r in rows if r.get("Counter_Name") == counter
                and "copy" in r["Kernel_Name"].lower()]
        vals = sorted(vals)[len(vals) // 2:] if vals else []  # the large copies
        return sum(vals) / max(len(vals), 1)

    cal = 1 << 28
    fs = cal / copy_bytes(copyf, "FETCH_SIZE")
    ws = cal / copy_bytes(copyw, "WRITE_SIZE")
    fk, wk = per_kernel(fetch, "FETCH_SIZE"), per_kernel(write, "WRITE_SIZE")
    # one key-generation launch per build
    b = args.builds or sum(len(v) for k, v in fk.items() if k.startswith("k_keygen")) or 1
    stages = {}
    for k in set(fk) | set(wk):
        st = _stage(k)
        if st is None:
            continue
        e = stages.setdefault(st, {"fetch": 0.0, "write": 0.0, "launches": 0, "names": set()})
        e["fetch"] += sum(fk.get(k, [])) * fs
        e["write"] += sum(wk.get(k, [])) * ws
        if k.startswith("k_onesweep") or st != "sort_pass":
            e["launches"] += len(fk.get(k, []))
        e["names"].add(k)
    kernels = {}
    for st, e in stages.items():
        n = max(e["launches"], 1)
        kernels[st] = {"fetch_bytes_per_launch": e["fetch"] / n, "write_bytes_per_launch":
                       e["write"] / n, "bytes_per_launch": (e["fetch"] + e["write"]) / n,
                       "launches_per_build": e["launches"] / b,
                       "rocprof_names": sorted(e["names"])}
    gather = None
    if args.gather_csv:
        # raw FETCH_SIZE per useful byte of the two gathers (16-B rows first, then 128-B rows)
        g = [float(r["Counter_Value"]) * 1024.0 / (1 << 28) for r in _read_csv(args.gather_csv)
             if r.get("Counter_Name") == "FETCH_SIZE" and "gather" in r["Kernel_Name"]]
        if len(g) >= 2:
            h = len(g) // 2
            gather = {"what": "raw FETCH_SIZE per useful byte of random-row gathers of 2^28 "
                              "bytes (bench.py --gather-calibration)",
                      "rows_16B": sum(g[:h]) / h, "rows_128B": sum(g[h:]) / (len(g) - h)}
    prof = {"workload": args.workload, "builds_profiled": b, "command": args.profile_command,
            "gather_check": gather,
            "calibration": {"what": "FETCH_SIZE / WRITE_SIZE (KiB) of a 2^28-byte device copy",
                            "copy_bytes_per_launch": cal, "fetch_scale": fs, "write_scale": ws},
            "source_sha256": source_hash(), "kernels": kernels,
            "file": f"profiles/pmc_{args.workload}.json"}
    out = os.path.join(PROFILES, f"pmc_{args.workload}.json")
    with open(out, "w") as f:
        json.dump(prof, f, indent=1, sort_keys=True)
    lines = [f"# HBM traffic per stage: {args.workload}", "",
             f"Counters: FETCH_SIZE x {fs:.4f} and WRITE_SIZE x {ws:.4f} (the same counters on a "
             "plain copy of 2^28 bytes); means per launch over the profiled builds.", "",
             "Command (repository root as `<repo>`):", "", f"    {args.profile_command}", "",
             "| stage | launches / build | fetch MB / launch | write MB / launch | total MB / build |",
             "|---|---|---|---|---|"]
    for st, k in sorted(kernels.items(), key=lambda kv: -kv[1]["bytes_per_launch"] *
                        kv[1]["launches_per_build"]):
        lines.append(f"| {st} | {k['launches_per_build']:g} | {k['fetch_bytes_per_launch'] / 1e6:.1f} | "
                     f"{k['write_bytes_per_launch'] / 1e6:.1f} | "
                     f"{k['bytes_per_launch'] * k['launches_per_build'] / 1e6:.1f} |")
    tot = sum(k["bytes_per_launch"] * k["launches_per_build"] for k in kernels.values())
    lines += ["", f"Total per build: {tot / 1e9:.3f} GB."]
    if gather:
        lines += ["", "Scale check on gathers (`bench.py --gather-calibration`): a random gather of "
                  f"128-byte rows reads {gather['rows_128B']:.2f} raw FETCH_SIZE bytes per byte, a "
                  f"random gather of 16-byte rows {gather['rows_16B']:.2f}, against 0.50 for the "
                  "streaming copy. Random whole-line reads count in full where streaming reads count "
                  "half, so the copy's x2 overstates a gather: the reorder's fetch figure above is "
                  "between its value and half of it (one 128-byte line per 16-byte record is "
                  "about 2.1 GB per build at N = 2^24)."]
    with open(os.path.join(PROFILES, f"build_{args.workload}_hbm_counters.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def code_text(src: str) -> str:
    """C/C++/HIP source without its comments, trailing spaces and blank lines:
    what a counter profile depends on (string and character literals kept)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).splitlines())
    return "\n".join(ln for ln in lines if ln)


def source_hash() -> str:
    """SHA-256 of the kernel and boundary sources' code (comments do not count)."""
    h = hashlib.sha256()
    for p in SOURCES:
        h.update(os.path.basename(p).encode())
        with open(p, encoding="utf-8") as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()


def counter_traffic(workload: str) -> dict | None:
    """Per-launch HBM bytes by kernel from the committed counter profile, or None
    when there is none or the kernels changed since it was taken."""
    path = os.path.join(PROFILES, f"pmc_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    if prof.get("source_sha256") != source_hash():
        return None
    return prof


def kernel_bytes(n: int, cells: int, leaves: int, key_passes: int, precision: str,
                 index_bits: int = 0) -> dict:
    """Bytes each traced stage must read + write for what it computes (its
    compulsory traffic), per build.

    keygen      read pos 12 + mass 4; write key 8 + packed (x, y, z, m) record 16
    sort_pass   per pass, what its element format moves in and out (sort_forms):
                key 8 + index 4 while the key is 64-bit (pass 0 reads the key alone:
                its index is the position), then one packed word of 8 or 4 bytes;
                the last pass writes the index alone, 4
                (counted passes also read their elements a second time to count
                their tiles' digits, not counted here)
    reorder     read perm 4 + gathered record 16; write the record in key order 16, its
                key 8 and its (a_i, D_i) 2
    cell_emit   read sorted keys 8 + sorted records 16 + (a_i, D_i) 2 per particle; write
                key 8, depth 1, first 4, child link 8, head_parent 4 per cell, count 4 +
                moments per leaf
    parents     per child cell read key 8 + count 4 + moments; per parent read head 4,
                write count 4 + child count 4 + moments
    (with TB_SUBTREES, in place of cell_emit and parents:)
    blocks      read sorted keys 8; write the block-start byte 1
    block_build read sorted keys 8 + block-start byte 1 + sorted record 16 per particle;
                write key 8, depth 1, first 4, child link 8, count 4 + moments per cell
    upper       (the cells above the blocks: a few thousand, not counted)
    moments: FP64 80 B (com 32 + quad 48); mixed 44 B (com 16 + quad 24 + mass term 4)
    """
    mom = 80 if precision == "fp64" else 44
    inner = cells - leaves
    bits = -(-63 // key_passes)  # digit width of these passes
    forms = sort_forms(n, bits, index_bits)
    size = {"key64": 12, "pack64": 8, "pack32": 4, "idx": 4}
    sort = 0
    for p in range(key_passes):
        sort += ((8 if p == 0 else size[forms[p]]) + size[forms[p + 1]]) * n
    return {
        "keygen": 40 * n,
        "sort_pass": sort,
        "reorder": 46 * n,
        "cell_emit": 26 * n + 25 * cells + (4 + mom) * leaves,
        "parents": (12 + mom) * max(cells - 1, 0) + (12 + mom) * inner,
        "blocks": 9 * n,
        "block_build": 25 * n + (25 + mom) * cells,
    }


def sort_forms(n: int, bits: int, index_bits: int = 0) -> list:
    """Element format read by each radix pass, then the last pass's output, as
    the library plans them: the index needs ib = bits(n - 1) bits (or a batch's
    set-size bound, index_bits, when smaller); once the key bits not yet
    consumed (with its leading 1) fit beside it in 64 or 32 bits, key and index
    travel as one packed word."""
    ib = max(1, (n - 1).bit_length())
    if 0 < index_bits < ib:
        ib = index_bits
    passes = -(-63 // bits)
    forms = ["key64"]
    for k in range(passes):
        rem = 64 - (k + 1) * bits  # key >> consumed bits, the leading 1 at bit 63 included
        if k + 1 == passes:
            forms.append("idx")
        elif rem + ib <= 32:
            forms.append("pack32")
        elif rem + ib <= 64:
            forms.append("pack64")
        else:
            forms.append("key64")
    return forms


def method_bytes(n: int, cells: int, key_passes: int, precision: str) -> float:
    """What the method must move per build (the whole-build algorithmic bytes):
    keys 20 B, sort 8 + 24 P, gather 20, structure 8 + 25 c, moments 2 x 80 c
    (FP64) or 2 x 40 c (mixed) per particle, with c = cells / N."""
    c = cells / max(n, 1)
    mom = 160 if precision == "fp64" else 80
    return n * (56 + 24 * key_passes + (25 + mom) * c)


def traced_kernels(run, steps, tb):
    """Per-stage durations from HIP events recorded on the build stream."""
    import torch
    tb.tb_trace_enable(True)
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    trace = tb.tb_trace_read()
    tb.tb_trace_enable(False)
    return trace


def kernels_table(trace, steps, alg):
    out = {}
    for name, (launches, total_ms) in sorted(trace.items()):
        per_build_ms = total_ms / steps
        k = {"ms_per_build": round(per_build_ms, 4), "launches_per_build": launches // steps,
             "avg_launch_ms": round(total_ms / max(launches, 1), 5)}
        if alg.get(name):
            k["alg_bytes_per_build"] = alg[name]
            k["alg_GBps"] = round(alg[name] / (per_build_ms * 1e-3) / 1e9, 1)
        out[name] = k
    return out


SORT_PASS_BYTES = 24  # the method's bytes per key and radix pass: (key 8 + index 4) in and out


def roofline(trace, alg, key_passes, workload, n, counters_apply=True):
    """Roofline entry of the dominant kernel (the sort's key passes).  achieved =
    the method's algorithmic bytes of one pass (24 per key) / the mean pass
    time; design_* = what this design's element formats move (less, as the
    key narrows and is packed with its index)."""
    launches, total_ms = trace["sort_pass"]
    avg_ms = total_ms / launches
    per_launch = SORT_PASS_BYTES * n
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    design = alg["sort_pass"] / key_passes
    r = {"kernel": "k_onesweep (radix pass over the key bits, one per digit; a counted pass "
                   "includes its k_tile_count and k_tile_scan)",
         "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
         "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
         "alg_bytes_per_launch": per_launch, "avg_launch_ms": round(avg_ms, 5),
         "design_bytes_per_launch": design,
         "design_GBps": round(design / (avg_ms * 1e-3) / 1e9, 1)}
    prof = counter_traffic(workload) if counters_apply else None
    if prof is not None:
        k = prof["kernels"].get("sort_pass")
        if k:
            r["traffic"] = k["bytes_per_launch"]
            r["traffic_source"] = prof["file"]
    return r


def counter_summary(workload, ms_per_step, counters_apply=True):
    prof = counter_traffic(workload) if counters_apply else None
    if prof is None:
        return None
    tot = sum(k["bytes_per_launch"] * k["launches_per_build"] for k in prof["kernels"].values())
    return {"bytes_per_build": tot, "GBps": round(tot / (ms_per_step * 1e-3) / 1e9, 1),
            "frac": round(tot / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "source": prof["file"]}


def stream_copy(reps: int = 10, nbytes: int = 1 << 30) -> dict:
    """A plain device-to-device copy of `nbytes` (read + write), timed outside the
    build steps: the bandwidth a streaming kernel reaches on this GPU, against
    which the build's algorithmic byte rate is also quoted."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / reps
    del src, dst
    torch.cuda.empty_cache()
    gbps = 2 * nbytes / sec / 1e9
    return {"bytes_moved": 2 * nbytes, "GBps": round(gbps, 1),
            "frac_of_peak": round(gbps / HBM_PEAK_GBPS, 4)}


def time_steps(run, steps, warmup):
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def moment_error_vs(res, ref, side=1.0):
    """Max per-cell relative errors of res against ref (same tree): |dM|/M,
    max|d com|/l, max|dQ|/(M l^2), l the cell side."""
    import torch
    lvl = ref["cell_level"].to(torch.float64)
    l = side * torch.pow(2.0, -lvl)
    M = ref["com"][:, 3].to(torch.float64)
    gc, gq = res["com"].to(torch.float64), res["quad"].to(torch.float64)
    rc, rq = ref["com"].to(torch.float64), ref["quad"].to(torch.float64)
    e_m = ((gc[:, 3] - M).abs() / M).max().item()
    e_c = ((gc[:, :3] - rc[:, :3]).abs().amax(1) / l).max().item()
    e_q = ((gq - rq).abs().amax(1) / (M * l * l)).max().item()
    return {"M": e_m, "com": e_c, "quad": e_q}


def run_single(args, tb, dg, torch, np):
    t_gen = time.time()
    pos_np, mass_np, n_leaf = dg.workload(args.workload)
    n = pos_np.shape[0]
    print(f"[bench] generated {args.workload} N={n} in {time.time() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    precision = args.precision or ("mixed" if args.workload == "mixed16m" else "fp64")
    # the committed counter profiles were taken with the defaults: their sort
    # figures apply while the sort runs as profiled, the whole-build figure only
    # while every kernel does
    sort_as_profiled = not (args.sort_config or args.sort_counted or args.sort_lookback)
    build_as_profiled = (not args.subtrees and args.curve == "morton"
                         and precision == ("mixed" if args.workload == "mixed16m" else "fp64"))
    k = args.sort_config or 0
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    mass = torch.from_numpy(mass_np).to(dev)
    box = ((0.0, 0.0, 0.0), 1.0)
    b = tb.Builder(n, n_leaf, precision, k, dev, subtrees=args.subtrees,
                   counted=args.sort_counted, lookback=args.sort_lookback, curve=args.curve)
    run = lambda: b.launch(pos, mass, box)
    sec = time_steps(run, args.steps, args.warmup)
    print(f"[bench] {args.steps} builds, {sec * 1e3:.3f} ms/build", file=sys.stderr, flush=True)
    res = b.result()
    cells = res["n_cells"]
    leaves = int((res["child_ptr"][:, 0] < 0).sum().item())
    key_passes = (63 + tb.tb_sort_configs()[k][0] - 1) // tb.tb_sort_configs()[k][0]
    trace = traced_kernels(run, args.steps, tb)
    alg = kernel_bytes(n, cells, leaves, key_passes, precision)
    total_method = method_bytes(n, cells, key_passes, precision)
    line = {
        "metric": METRIC, "value": n / sec, "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 keys + f64 moments" if precision == "fp64" else "u64 keys + f32 moments",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "N": n,
                   "n_leaf": n_leaf, "precision": precision, "box": "unit cube",
                   "sort_config": list(tb.tb_sort_configs()[k]), "cells": cells,
                   "leaves": leaves,
                   "cell_build": "subtree-rooted blocks" if args.subtrees else "tiles + parents",
                   "sort_counted_all_passes": bool(args.sort_counted),
                   "sort_lookback_all_passes": bool(args.sort_lookback), "keys": args.curve},
        "roofline": roofline(trace, alg, key_passes, args.workload, n, sort_as_profiled),
        "build_method_bytes": total_method,
        "build_alg_GBps": round(total_method / sec / 1e9, 1),
        "build_alg_frac": round(total_method / sec / 1e9 / HBM_PEAK_GBPS, 4),
        "build_counter_traffic": counter_summary(args.workload, sec * 1e3,
                                                 sort_as_profiled and build_as_profiled),
        "traced_ms_per_build": round(sum(v[1] for v in trace.values()) / args.steps, 4),
        "kernels": kernels_table(trace, args.steps, alg),
    }
    if not args.no_compare:
        # the other cell build on the same data (the tree is the same either way)
        alt_b = tb.Builder(n, n_leaf, precision, k, dev, subtrees=not args.subtrees,
                           counted=args.sort_counted, lookback=args.sort_lookback,
                           curve=args.curve)
        alt_run = lambda: alt_b.launch(pos, mass, box)
        sec_alt = time_steps(alt_run, args.steps, args.warmup)
        alt = alt_b.result()
        same = all(torch.equal(res[f], alt[f]) for f in
                   ("perm", "cell_key", "cell_level", "cell_first", "cell_count", "child_ptr"))
        alt_trace = traced_kernels(alt_run, min(args.steps, 5), tb)
        line["other_cell_build"] = {
            "cell_build": "tiles + parents" if args.subtrees else "subtree-rooted blocks",
            "ms_per_step": sec_alt * 1e3, "tree_identical": bool(same),
            "kernels": kernels_table(alt_trace, min(args.steps, 5), alg)}
        del alt_b, alt
    if args.workload == "mixed16m" and not args.no_compare:
        # the FP64 path on the same data and the mixed path's error against it
        # (the FP64 path matches the FP64 oracle to 1e-12 in the parity tests)
        ref_b = tb.Builder(n, n_leaf, "fp64", k, dev)
        ref_run = lambda: ref_b.launch(pos, mass, box)
        sec64 = time_steps(ref_run, args.steps, args.warmup)
        ref = ref_b.result()
        same = all(torch.equal(res[f], ref[f]) for f in
                   ("perm", "cell_key", "cell_level", "cell_first", "cell_count", "child_ptr"))
        line["fp64_comparison"] = {
            "fp64_ms_per_step": sec64 * 1e3, "fp64_particles_per_s": n / sec64,
            "mixed_speedup": sec64 / sec, "tree_identical": bool(same),
            "max_rel_error_vs_fp64": moment_error_vs(res, ref),
            "error_measures": "per cell: |dM|/M, max|d com|/l, max|dQ|/(M l^2), l = cell side; "
                              "max over all cells"}
    return line, (pos_np, mass_np, n_leaf, None)


def run_batched(args, tb, dg, torch, np):
    from paper_2312_06102_amd import autotune
    t_gen = time.time()
    sizes = dg.batched_sizes(4096, 256, 262144, seed=4)
    pos_np, mass_np, offsets_np = dg.batched_plummer(sizes, seed=4)
    n, B, n_leaf = pos_np.shape[0], len(sizes), 16
    print(f"[bench] generated batched4096 N={n} in {time.time() - t_gen:.1f}s", file=sys.stderr,
          flush=True)
    precision = args.precision or "fp64"
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    mass = torch.from_numpy(mass_np).to(dev)
    off = torch.from_numpy(offsets_np).to(dev)
    boxes = torch.tensor([[0.0, 0.0, 0.0, 1.0]] * B, dtype=torch.float64, device=dev)
    # the largest set bounds the sort's index within a set (TB_SET_INDEX_BITS)
    set_bits = max(1, (int(np.max(sizes)) - 1).bit_length())
    # sort shape: the autotuner's choice on this batch (timed outside the steps)
    t_tune = time.time()
    if args.sort_config is None:
        k = autotune.tune(pos, mass, n_leaf, precision, set_offsets=off, boxes=boxes,
                          use_cache=False, verbose=True, set_index_bits=set_bits)
    else:
        k = args.sort_config
    tune_s = time.time() - t_tune
    bb = tb.BatchBuilder(n, B, n_leaf, precision, k, dev, set_index_bits=set_bits)
    bb.capture(pos, mass, off, boxes)
    sec = time_steps(bb.replay, args.steps, args.warmup)
    print(f"[bench] {args.steps} graph replays, {sec * 1e3:.3f} ms/batch", file=sys.stderr,
          flush=True)
    res = bb.result()
    cells = res["n_cells"]
    leaves = int((res["child_ptr"][:, 0] < 0).sum().item())
    eager = lambda: bb.launch(pos, mass, off, boxes)
    sec_eager = time_steps(eager, args.steps, 1)
    trace = traced_kernels(eager, args.steps, tb)
    bits = tb.tb_sort_configs()[k][0]
    key_passes = (63 + bits - 1) // bits
    alg = kernel_bytes(n, cells, leaves, key_passes, precision, set_bits)
    total_method = method_bytes(n, cells, key_passes, precision)
    line = {
        "metric": METRIC, "value": n / sec, "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 keys + f64 moments" if precision == "fp64" else "u64 keys + f32 moments",
        "data": "synthetic",
        "config": {"workload": "batched4096", "description": WORKLOADS["batched4096"], "N": n,
                   "sets": B, "set_size_min": int(sizes.min()), "set_size_max": int(sizes.max()),
                   "set_index_bits": set_bits,
                   "n_leaf": n_leaf, "precision": precision, "box": "unit cube per set",
                   "sort_config": list(tb.tb_sort_configs()[k]), "autotune_s": round(tune_s, 2),
                   "cells": cells, "leaves": leaves, "launch": "one HIP graph per batch"},
        "roofline": roofline(trace, alg, key_passes, "batched4096", n),
        "build_method_bytes": total_method,
        "build_alg_GBps": round(total_method / sec / 1e9, 1),
        "build_alg_frac": round(total_method / sec / 1e9 / HBM_PEAK_GBPS, 4),
        "build_counter_traffic": counter_summary("batched4096", sec * 1e3),
        "eager_batch_ms": sec_eager * 1e3,
        "traced_ms_per_build": round(sum(v[1] for v in trace.values()) / args.steps, 4),
        "kernels": kernels_table(trace, args.steps, alg),
    }
    del bb
    torch.cuda.empty_cache()
    if not args.no_sequential:
        # the same sets as 4096 sequential single-set builds on one stream, one
        # workspace and one set of outputs sized for the largest set
        nmax = int(sizes.max())
        ws_bytes = tb.tb_workspace_bytes(nmax, n_leaf, tb.TB_FP64 if precision == "fp64" else tb.TB_MIXED)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        outb = tb.TreeBuffers.allocate(nmax, n_leaf, precision, dev)
        st = outb.struct()
        flags = tb.TB_FP64 if precision == "fp64" else tb.TB_MIXED
        box = tb._box_struct(((0.0, 0.0, 0.0), 1.0))
        stream = torch.cuda.current_stream().cuda_stream
        pp, mp = pos.data_ptr(), mass.data_ptr()

        def sequential():
            for bi in range(B):
                s0, s1 = int(offsets_np[bi]), int(offsets_np[bi + 1])
                rc = tb.tb_build(pp + 12 * s0, mp + 4 * s0, s1 - s0, n_leaf, box, flags,
                                 ws.data_ptr(), ws_bytes, st, stream)
                if rc:
                    raise RuntimeError(f"tb_build failed: {rc}")
        seq_steps = max(1, min(3, args.steps))
        sec_seq = time_steps(sequential, seq_steps, 1)
        line["sequential"] = {"ms_per_batch": sec_seq * 1e3, "particles_per_s": n / sec_seq,
                              "steps": seq_steps, "graph_speedup": sec_seq / sec,
                              "what": "4096 tb_build calls on one stream, sort config 0"}
    return line, (pos_np, mass_np, n_leaf, offsets_np)


def cpu_model() -> str:
    """The host CPU's model name (first /proc/cpuinfo entry)."""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(args, data, np):
    """The CPU oracle (top-down insertion + direct FP64 moments, one thread) timed
    on this host, per stage, on the workload itself when N <= 2^24, else on a
    bounded sample; beside it the paper's own leaf-first method on one thread
    (Algorithms 1 + 2, moments from the children) on the same particles."""
    import oracle
    pos_np, mass_np, n_leaf, offsets = data
    oracle.load()
    if offsets is None:
        m = pos_np.shape[0] if args.cpu_sample is None else min(args.cpu_sample, pos_np.shape[0])
        p, w = np.ascontiguousarray(pos_np[:m]), np.ascontiguousarray(mass_np[:m])
        tc0 = time.perf_counter()
        ref = oracle.build(p, w, n_leaf)
        tc1 = time.perf_counter()
        lf = oracle.leaf_first_build(p, w, n_leaf)
        tc2 = time.perf_counter()
        if lf["n_cells"] != ref["n_cells"]:
            raise RuntimeError("leaf-first CPU reference disagrees with the oracle")
        stages = {k: round(v, 3) for k, v in ref["stage_s"].items()}
        lf_stages = {k: round(v, 3) for k, v in lf["stage_s"].items()}
        what = ("the whole workload" if m == pos_np.shape[0]
                else f"the first {m} particles of the workload")
        what += f" (N = {m}), one run"
    else:
        # whole sets from the start of the batch, about cpu_sample particles
        want = args.cpu_sample or (1 << 22)
        nb = int(np.searchsorted(offsets, want)) or 1
        m = int(offsets[nb])
        stages = dict.fromkeys(oracle.ORACLE_STAGES, 0.0)
        lf_stages = dict.fromkeys(oracle.LEAF_FIRST_STAGES, 0.0)
        tc0 = time.perf_counter()
        for b in range(nb):
            s0, s1 = int(offsets[b]), int(offsets[b + 1])
            r = oracle.build(pos_np[s0:s1], mass_np[s0:s1], n_leaf)
            for k, v in r["stage_s"].items():
                stages[k] += v
        tc1 = time.perf_counter()
        for b in range(nb):
            s0, s1 = int(offsets[b]), int(offsets[b + 1])
            r = oracle.leaf_first_build(pos_np[s0:s1], mass_np[s0:s1], n_leaf)
            for k, v in r["stage_s"].items():
                lf_stages[k] += v
        tc2 = time.perf_counter()
        stages = {k: round(v, 3) for k, v in stages.items()}
        lf_stages = {k: round(v, 3) for k, v in lf_stages.items()}
        what = f"the first {nb} sets ({m} particles) of the same batch, one build per set, one run"
    host = f"{cpu_model()}, host nproc={os.cpu_count()}"
    return {"value": m / (tc1 - tc0), "unit": "particles/s", "cores": 1, "kind": "oracle",
            "sample": f"{what}: full oracle build (FP64 keys, top-down insertion, perm, "
                      f"canonical order, direct FP64 moments per cell), {tc1 - tc0:.2f} s on "
                      f"one thread of {host}",
            "N": m, "seconds": round(tc1 - tc0, 3), "stages_s": stages, "cpu_model": cpu_model(),
            "paper_method": {
                "value": m / (tc2 - tc1), "unit": "particles/s", "cores": 1,
                "seconds": round(tc2 - tc1, 3), "stages_s": lf_stages,
                "what": "the paper's leaf-first build on one thread (keys, sort of key/index "
                        "pairs, reorder, leaves by Algorithm 1, parents by Algorithm 2 with "
                        "moments combined from the children), same particles"}}


def run_sim(args, dg, np):
    """Leapfrog steps on a Plummer sphere or an exponential disk (Sec. 3: theta
    0.75, n_leaf 10, n_crit 512), reordering every step and every tenth step."""
    from paper_2312_06102_amd.simulate import Simulation
    gen = dg.plummer_sim if args.sim == "plummer" else dg.disk_sim
    pos, vel, mass = gen(args.sim_n)
    dt = 1e-4 if args.sim == "plummer" else 3e-4
    runs = {}
    for k in (1, 10):
        sim = Simulation(pos, vel, mass, dt, n_leaf=10, theta=0.75, n_crit=512, eps=5e-4,
                         reorder_every=k)
        sim.step(max(args.warmup, 1))
        sim.synchronise()
        sim._events.clear()
        t0 = time.perf_counter()
        sim.step(args.steps)
        sim.synchronise()
        wall = time.perf_counter() - t0
        t = sim.timings()["mean_ms"]
        inter = int(sim.interactions[-1].cpu()[1])
        runs[f"reorder_every_{k}"] = {"ms_per_step": wall * 1e3 / args.steps, "phase_ms": t,
                                      "interactions_last_step": inter}
        print(f"[bench sim] k={k}: {wall * 1e3 / args.steps:.2f} ms/step {t}", file=sys.stderr,
              flush=True)
        del sim
    r1, r10 = runs["reorder_every_1"], runs["reorder_every_10"]
    build = lambda r: r["phase_ms"]["build"] + r["phase_ms"]["reorder"] * r["phase_ms"]["reorders"] / max(r["phase_ms"]["steps"], 1)
    return {
        "metric": "leapfrog N-body step with a tree rebuild every step: tree-build ms per step",
        "value": build(r10), "unit": "ms", "higher_is_better": False, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
        "config": {"workload": f"{args.sim}_sim", "N": args.sim_n, "n_leaf": 10, "theta": 0.75,
                   "n_crit": 512, "eps": 5e-4, "dt": dt, "quadrupole": True},
        "build_ms_reorder_every_step": build(r1), "build_ms_reorder_every_10": build(r10),
        "runs": runs,
    }


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gather_calibration:
        gather_calibration()
        return
    if args.summarize_trace:
        summarize_trace(args)
        return
    if args.summarize_pmc:
        summarize_pmc(args)
        return
    if args.summarize_sq:
        summarize_sq(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2312_06102_amd import datagen as dg
    from paper_2312_06102_amd import treebuild as tb

    if args.sim:
        print(json.dumps(run_sim(args, dg, np)))
        return
    if args.workload == "batched4096":
        line, data = run_batched(args, tb, dg, torch, np)
    else:
        line, data = run_single(args, tb, dg, torch, np)
    copy = stream_copy()
    copy["build_alg_frac_of_copy"] = round(line["build_alg_GBps"] / copy["GBps"], 4)
    line["stream_copy"] = copy
    if not args.no_cpu_baseline:
        if args.cpu_sample is None and data[3] is None and data[0].shape[0] > (1 << 24):
            args.cpu_sample = 1 << 24
        print("[bench] timing the CPU oracle and the CPU leaf-first reference", file=sys.stderr,
              flush=True)
        line["cpu_baseline"] = cpu_baseline(args, data, np)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
