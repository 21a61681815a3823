"""Autotuner for the radix-sort shape (digit width and tile size) of a build.

Every entry of ``tb_sort_configs()`` gives bit-identical trees; they differ in
speed, and the best one depends on the number of particles and sets.  The tuner
times each shape on the caller's own data (whole builds, HIP events on the
build stream), keeps the fastest, and remembers it per size class in a JSON
cache so that later builders of a similar size skip the timing.

    k = autotune.tune(pos, mass, n_leaf)                       # one set
    k = autotune.tune(pos, mass, n_leaf, set_offsets=offsets)  # a batch
    b = BatchBuilder(n, B, n_leaf, sort_config=k)

Size class: (device name, precision, n_leaf, round(log2 N), round(log2 B)).
"""
from __future__ import annotations

import json
import math
import os
import sys
from typing import Optional

import torch

from . import treebuild as tb

CACHE_ENV = "TREEBUILD_TUNE_CACHE"
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "treebuild_tune.json")


def cache_path() -> str:
    return os.environ.get(CACHE_ENV, DEFAULT_CACHE)


def size_class(n: int, nsets: int, n_leaf: int, precision: str, device=None) -> str:
    name = torch.cuda.get_device_name(device) if torch.cuda.is_available() else "none"
    return (f"{name}|{precision}|nl{n_leaf}|n{round(math.log2(max(n, 1)))}"
            f"|b{round(math.log2(max(nsets, 1)))}")


def _load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: dict) -> None:
    data = _load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(n: int, nsets: int, n_leaf: int, precision: str = "fp64", device=None,
           path: Optional[str] = None) -> Optional[int]:
    """The cached choice for this size class, or None."""
    e = _load_cache(path or cache_path()).get(size_class(n, nsets, n_leaf, precision, device))
    return None if e is None else int(e["sort_config"])


def time_config(k: int, pos, mass, n_leaf: int, precision: str, set_offsets=None, boxes=None,
                box=((0.0, 0.0, 0.0), 1.0), reps: int = 3, set_index_bits: int = 0) -> float:
    """Milliseconds per build with sort shape k (median of `reps` after one warm-up);
    set_index_bits: the batch's set-size bound, as the builds will use it."""
    n = pos.shape[0]
    if set_offsets is None:
        b = tb.Builder(n, n_leaf, precision, k, pos.device)
        run = lambda: b.launch(pos, mass, box)
    else:
        b = tb.BatchBuilder(n, set_offsets.shape[0] - 1, n_leaf, precision, k, pos.device,
                            set_index_bits=set_index_bits)
        run = lambda: b.launch(pos, mass, set_offsets, boxes)
    run()
    torch.cuda.synchronize()
    times = []
    s = torch.cuda.current_stream()
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        run()
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    del b
    return sorted(times)[len(times) // 2]


def tune(pos, mass, n_leaf: int, precision: str = "fp64", set_offsets=None, boxes=None,
         box=((0.0, 0.0, 0.0), 1.0), reps: int = 3, use_cache: bool = True,
         path: Optional[str] = None, verbose: bool = False, set_index_bits: int = 0) -> int:
    """Fastest sort shape for builds like this one; the result is cached.
    set_index_bits: a batch's set-size bound (TB_SET_INDEX_BITS), timed with it."""
    n = pos.shape[0]
    nsets = 1 if set_offsets is None else set_offsets.shape[0] - 1
    path = path or cache_path()
    key = size_class(n, nsets, n_leaf, precision, pos.device)
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit is not None:
            return int(hit["sort_config"])
    results = {}
    for k in range(len(tb.tb_sort_configs())):
        results[k] = time_config(k, pos, mass, n_leaf, precision, set_offsets, boxes, box, reps,
                                 set_index_bits)
        if verbose:
            print(f"[autotune] {key} config {k} {tb.tb_sort_configs()[k]}: {results[k]:.3f} ms",
                  file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    best = min(results, key=results.get)
    _store(path, key, {"sort_config": best, "shape": list(tb.tb_sort_configs()[best]),
                       "ms": {str(k): round(v, 4) for k, v in results.items()}})
    return best
