"""Project autotuner: picks, by timing on the device, the tile-pass kernel
variant per tile size and the tile size (qubits per LDS tile) per register
size n, for batched throughput, and the radix-sort shape (key bits per pass,
terms per thread) of the SPARSE engine's merge per term-capacity class.
Results are cached as JSON keyed by the device name and weight dtype, and
applied through pp_tune_set.

Probes are seeded random circuits (50% H/S/CX, 50% RX/RY/RZ) evaluated in
batches large enough to fill the GPU.  For a fixed tile size the candidates
agree bit for bit, except that the register-tile kernels (variants 3 and 4)
run a schedule ordered into register segments, which changes only rounding;
so does a changed tile size (the schedule packs the same gates differently).
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import _lib as L

VARIANT_NAMES = {0: "workgroup-per-tile", 1: "persistent-prefetch", 2: "wave-per-tile",
                 3: "register-tile", 4: "register-tile-prefetch"}
# radix-sort shapes of the SPARSE merge: (key bits per pass, terms per thread)
SORT_SHAPES = {0: (8, 8), 1: (8, 4), 2: (8, 16), 3: (7, 8), 4: (7, 16), 5: (6, 16)}
# per capacity class: the largest term capacity of the class and a probe
# circuit (qubits, gates) whose string set grows to a sizeable part of it
SORT_CLASSES = {0: (1 << 17, 16, 70), 1: (1 << 21, 20, 130), 2: (1 << 23, 20, 200)}


def _device_name():
    import torch
    return torch.cuda.get_device_name(0).replace(" ", "_").replace("/", "_")


def cache_path(dtype="f64"):
    base = os.environ.get("PAULIPROP_TUNE_CACHE")
    if base and base.endswith(".json"):
        return base
    d = base or os.path.join(os.path.expanduser("~"), ".cache", "pauliprop")
    return os.path.join(d, f"tune_{_device_name()}_{dtype}.json")


def apply(table):
    for n, b in table.get("resident_block", {}).items():
        L.tune_set(L.PP_TUNE_RESIDENT_BLOCK, int(n), int(b))
    for k, v in table.get("tile_kernel", {}).items():
        L.tune_set(L.PP_TUNE_TILE_KERNEL, int(k), int(v))
    for n, k in table.get("tile_qubits", {}).items():
        L.tune_set(L.PP_TUNE_TILE_QUBITS, int(n), int(k))
    for cls, v in table.get("sort_shape", {}).items():
        L.tune_set(L.PP_TUNE_SORT_SHAPE, int(cls), int(v))


def load_cached(dtype="f64", apply_now=True):
    p = cache_path(dtype)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        table = json.load(f)
    if apply_now:
        apply(table)
    return table


def _probe_batch(api, n, count, m, dtype, seed, tile_qubits=0):
    from . import workloads as W
    rng = np.random.default_rng(seed)
    circs = []
    for _ in range(count):
        w = W.random_circuit(rng, n, m, W.obs_z(n, [0, 1]))
        circs.append(api.Circuit.from_workload(w, dtype=dtype, engine="dense", tile_qubits=tile_qubits))
    return circs


def _time_batch(api, circs, reps=3):
    import torch
    out = torch.empty(len(circs), dtype=torch.float64, device="cuda")
    api.evaluate_batch(circs, out)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        api.evaluate_batch(circs, out)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def _count_for(n):
    # enough tiles to fill 256 CUs several times over
    return max(2, min(64, (1 << 16) // (4 ** (n - 6))))


def _sort_probe(api, cls, dtype, say):
    """A sort-merge SPARSE circuit of capacity class cls whose strings fill
    a sizeable part of the capacity (fewer gates until nothing overflows)."""
    from . import workloads as W
    cap, n, m = SORT_CLASSES[cls]
    for _ in range(8):
        w = W.random_circuit(np.random.default_rng(9300 + cls), n, m, W.obs_z(n, [0, 1]))
        c = api.Circuit.from_workload(w, dtype=dtype, engine="sparse", max_terms=cap)
        c.set_option(L.PP_OPT_SPARSE_FRAME, 0)
        c.evaluate()
        st = c.stats()
        if not st["overflow"]:
            return c, st
        c.close()
        m = m * 3 // 4
    say(f"sort class {cls}: no probe fits the capacity")
    return None, None


def tune_sort(dtype="f64", log=None, reps=3):
    """Times every radix-sort shape on one sort-merge probe per capacity class
    and applies the fastest; returns {"sort_shape": {cls: shape}, "timings":
    ...}.  Every shape must give the same <O> bit for bit."""
    import torch
    from . import api
    say = log or (lambda s: None)
    res = {"sort_shape": {}, "timings": {}}
    for cls in SORT_CLASSES:
        c, st = _sort_probe(api, cls, dtype, say)
        if c is None:
            continue
        best, times, ref = None, {}, None
        old = L.tune_get(L.PP_TUNE_SORT_SHAPE, cls)
        for v in SORT_SHAPES:
            L.tune_set(L.PP_TUNE_SORT_SHAPE, cls, v)
            ev = c.evaluate()
            torch.cuda.synchronize()
            bits = np.float64(ev.item()).view(np.uint64)
            if ref is None:
                ref = bits
            elif bits != ref:
                L.tune_set(L.PP_TUNE_SORT_SHAPE, cls, old)
                raise RuntimeError(f"sort shape {v} changed <O> in class {cls}")
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                c.evaluate()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            times[v] = float(np.median(ts))
            if best is None or times[v] < times[best]:
                best = v
        L.tune_set(L.PP_TUNE_SORT_SHAPE, cls, best)
        res["sort_shape"][str(cls)] = best
        res["timings"][str(cls)] = {"terms": int(st["final_terms"]),
                                    **{f"{SORT_SHAPES[v][0]}b{SORT_SHAPES[v][1]}i": t for v, t in times.items()}}
        say(f"sort shape class {cls} ({st['final_terms']} strings): {SORT_SHAPES[best]} "
            f"({ {SORT_SHAPES[v]: round(t * 1e3, 2) for v, t in times.items()} } ms)")
        c.close()
    return res


def tune(sizes=(8, 9, 10, 11, 12), dtype="f64", m=1200, save=True, log=None, resident=(5, 6, 7), sort=True):
    """Times every candidate and returns (and applies, and caches) the table
    {"tile_kernel": {k: variant}, "tile_qubits": {n: k},
     "resident_block": {n: threads}, "sort_shape": {class: shape},
     "timings": ...}."""
    from . import api
    say = log or (lambda s: None)
    table = {"tile_kernel": {}, "tile_qubits": {}, "resident_block": {},
             "timings": {"tile_kernel": {}, "tile_qubits": {}, "resident_block": {}},
             "device": _device_name(), "dtype": dtype, "probe_gates": m}
    # 0. threads of the LDS-resident kernel (one circuit per workgroup)
    for n in resident:
        circs = _probe_batch(api, n, 256, m, dtype, seed=8900 + n)
        best, times = None, {}
        for b in (256, 512, 1024):
            L.tune_set(L.PP_TUNE_RESIDENT_BLOCK, n, b)
            times[b] = _time_batch(api, circs)
            if best is None or times[b] < times[best]:
                best = b
        L.tune_set(L.PP_TUNE_RESIDENT_BLOCK, n, best)
        table["resident_block"][str(n)] = best
        table["timings"]["resident_block"][str(n)] = {str(b): t for b, t in times.items()}
        say(f"resident block n={n}: {best} ({ {b: round(t * 1e3, 2) for b, t in times.items()} } ms)")
        for c in circs:
            c.close()
    # 1. kernel variant per tile size k, on circuits with n = k + 3 tiled at k
    for k in (4, 5, 6, 7):
        n = k + 3
        circs = _probe_batch(api, n, _count_for(n), m, dtype, seed=9000 + k, tile_qubits=k)
        best, times = None, {}
        for v in {6: (0, 1, 2, 3, 4), 7: (0, 1)}.get(k, (0, 1, 2)):
            L.tune_set(L.PP_TUNE_TILE_KERNEL, k, v)
            times[v] = _time_batch(api, circs)
            if best is None or times[v] < times[best]:
                best = v
        L.tune_set(L.PP_TUNE_TILE_KERNEL, k, best)
        table["tile_kernel"][str(k)] = best
        table["timings"]["tile_kernel"][str(k)] = {VARIANT_NAMES[v]: t for v, t in times.items()}
        say(f"tile kernel k={k}: {VARIANT_NAMES[best]} ({ {VARIANT_NAMES[v]: round(t * 1e3, 2) for v, t in times.items()} } ms)")
        for c in circs:
            c.close()
    # 2. tile size per n
    for n in sizes:
        best, times = None, {}
        for k in (4, 5, 6, 7):
            if k >= n:
                continue
            circs = _probe_batch(api, n, _count_for(n), m, dtype, seed=9100 + n, tile_qubits=k)
            times[k] = _time_batch(api, circs)
            for c in circs:
                c.close()
            if best is None or times[k] < times[best]:
                best = k
        if best is None:
            continue
        L.tune_set(L.PP_TUNE_TILE_QUBITS, n, best)
        table["tile_qubits"][str(n)] = best
        table["timings"]["tile_qubits"][str(n)] = {str(k): t for k, t in times.items()}
        say(f"tile qubits n={n}: k={best} ({ {k: round(t * 1e3, 2) for k, t in times.items()} } ms)")
    # 3. radix-sort shape of the SPARSE merge per capacity class
    if sort:
        srt = tune_sort(dtype, log=log)
        table["sort_shape"] = srt["sort_shape"]
        table["timings"]["sort_shape"] = srt["timings"]
    if save:
        p = cache_path(dtype)
        os.makedirs(os.path.dirname(p), exist_ok=True)
        with open(p, "w") as f:
            json.dump(table, f, indent=1)
        table["cache"] = p
    return table
