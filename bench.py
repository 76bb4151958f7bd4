"""Benchmark of the Pauli-propagation hot path on one MI355X.

Default workload: 512 seeded random circuits of uneven size (n ~ U{4..10},
m log-uniform in [1k, 20k], half Clifford gates H/S/CX and half RX/RY/RZ with
theta ~ U[0, 2pi), observable Z0 Z1), all evaluated per step in batched
launches; the same 512 circuits are also timed one circuit per launch
sequence ("plain").  The metric is Pauli-term updates per second, where one
update is one live string passing one gate on the canonical schedule (merge
after every gate), counted by the GPU itself in tracked runs.

Prints ONE JSON line.  Only the cpu_baseline leg touches the CPU oracle.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "Pauli-term updates/s; circuits/s + p50/p99 latency, batched vs plain, 1 GPU"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(name):
    from paper_2502_10685_amd import workloads as W
    if name == "batch512":
        circs = W.config3()
        desc = ("512 random circuits, n~U{4..10}, m log-uniform [1k,20k], 50% H/S/CX + 50% RX/RY/RZ, "
                "theta~U[0,2pi), O=Z0Z1, seed 3")
    elif name == "deep6":
        circs = [W.config2()]
        desc = "n=6, 60,000 random gates (50% Clifford), O=sum Z_i, seed 2"
    elif name == "hea4":
        circs = [W.config1()]
        desc = "n=4, HEA 10 layers (160 gates), O=Z0, seed 1"
    elif name == "chain4":
        circs = [W.chain_zxz_circuit()]
        desc = ("n=4, the paper's timing-ansatz shape: 50 layers x (4-CX ring + 100 x RZ RX RZ on every qubit) = "
                "60,200 gates, O=Z0, seed 6")
    elif name == "hea8":
        circs = [W.config4()]
        desc = "n=8, HEA 40 layers (1,280 gates, 960 params), O=TFIM (15 terms), seed 4"
    elif name in ("rand7", "rand10", "rand12"):
        n = int(name[4:])
        circs = [W.random_circuit(10 + n, n, 6000, W.obs_z(n, [0, 1]))]
        desc = f"n={n}, 6,000 random gates (50% Clifford), O=Z0Z1, seed {10 + n}"
    else:
        raise SystemExit(f"unknown workload {name}")
    return circs, desc


def updates_of(api, w, dtype="f64"):
    """U = sum over gates of the set size entering the gate, in Heisenberg
    order (g_m first), from tracked GPU runs.  The set size never decreases
    and is at most 4^n - 1 (+1 if O contains the identity), so a tracked run
    over the last L gates that ends saturated fixes U exactly:
    U = U_last_L + (m - L) * T_max.  L doubles until saturated or L = m."""
    from paper_2502_10685_amd import workloads as W
    n, m = w.n, w.m
    ident = bool(np.any((w.obs_x == 0) & (w.obs_z == 0)))
    tmax = 4 ** n - 1 + (1 if ident else 0)
    L = min(m, 256)
    while True:
        sub = W.make_circuit(n, (w.op[m - L:], w.q0[m - L:], w.q1[m - L:], w.param[m - L:]), w.n_params,
                             (w.obs_x, w.obs_z, w.obs_c), w.theta)
        c = api.Circuit.from_workload(sub, dtype=dtype, track=True)
        c.evaluate()
        st = c.stats()
        c.close()
        if L == m:
            return st["term_updates"], st["final_terms"]
        if st["final_terms"] == tmax:
            return st["term_updates"] + (m - L) * tmax, tmax
        L = min(m, 2 * L)


def count_updates(api, circs, dtype):
    """U per circuit (structure only: U does not depend on theta)."""
    us, terms = [], []
    t0 = time.time()
    for i, w in enumerate(circs):
        u, t = updates_of(api, w, dtype)
        us.append(u)
        terms.append(t)
        if (i + 1) % 128 == 0:
            log(f"update counts {i + 1}/{len(circs)} ({time.time() - t0:.1f}s)")
    return np.array(us, dtype=np.int64), np.array(terms, dtype=np.int64)


def serve(api, lam, count, budget, max_active):
    """Poisson arrivals at rate lam (seeded) of random circuits n ~ U{4..12},
    m log-uniform in [1k, 60k]; submit at arrival time, poll completions.
    Afterwards every served value is compared bit for bit with the same
    circuit evaluated alone (the oracle leg checks them against the state
    vector)."""
    from paper_2502_10685_amd import workloads as W
    import torch
    reqs = W.config5_requests(seed=5, lam=lam, count=count)
    arrivals = np.array([a for a, _ in reqs])
    ws = [w for _, w in reqs]
    U, _ = count_updates(api, ws, "f64")
    circs = [api.Circuit.from_workload(w) for w in ws]
    srv = api.Server(mem_budget_bytes=budget, max_active=max_active)
    torch.cuda.synchronize()
    lat, done_at, vals = {}, {}, {}
    t0 = time.perf_counter()
    i = 0
    tickets = {}
    while len(done_at) < count:
        now = time.perf_counter() - t0
        while i < count and arrivals[i] <= now:
            tickets[srv.submit(circs[i])] = i
            i += 1
        for t, j in list(tickets.items()):
            r = srv.poll(t)
            if r is not None:
                vals[j], lat[j] = r
                done_at[j] = time.perf_counter() - t0
                del tickets[t]
        if i < count:
            time.sleep(max(0.0, min(5e-4, arrivals[i] - (time.perf_counter() - t0))))
        else:
            time.sleep(2e-4)
    span = max(done_at.values())
    cnt = srv.counters()
    held, peak = srv.pool_bytes()
    srv.close()
    served = np.array([vals[j] for j in range(count)])
    solo = np.empty(count)
    for j, w in enumerate(ws):
        c = api.Circuit.from_workload(w)
        solo[j] = float(c.evaluate().item())
        c.close()
    mismatch = int(np.sum(served != solo))
    lats = np.array([lat[j] for j in range(count)]) * 1e-3
    rec = {"lambda_per_s": lam, "requests": count, "span_s": span,
           "offered_updates_per_s": float(U.sum() / max(arrivals[-1], 1e-9)),
           "updates_per_s": float(U.sum() / span), "circuits_per_s": count / span,
           "latency_ms": {"p50": float(np.percentile(lats, 50)), "p99": float(np.percentile(lats, 99))},
           "term_updates": int(U.sum()), "server": cnt,
           "pool_bytes_peak": int(peak), "budget_bytes": int(budget),
           "served_vs_solo_bitwise_mismatches": mismatch,
           "n_range": [int(min(w.n for w in ws)), int(max(w.n for w in ws))]}
    return rec, ws, served


def timed_steps(fn, steps, torch):
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, np.array(lat)


TILE_KERNEL_NAMES = {0: "tile_kernel", 1: "tile_stream_kernel", 2: "tile_kernel", 3: "tile_reg_kernel",
                     4: "tile_reg_kernel"}


def measured_traffic(kernel, workload, dtype):
    """HBM bytes per launch of the dominant kernel from the committed
    FETCH_SIZE/WRITE_SIZE summary (already scaled by the copy-kernel
    calibration), or None when no summary covers this kernel and workload or
    the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if dtype != "f64" or not os.path.exists(path):
        return None
    rec = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
    src = os.path.join(ROOT, rec.get("source", ""))
    if not os.path.isfile(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec.get("source_sha256"):
        return None
    return float(rec["fetch_bytes_per_launch"]) + float(rec["write_bytes_per_launch"])


def dense_bytes(objs):
    """Algorithmic HBM bytes of one evaluation of each tiled circuit: every
    pass reads and writes each 4^n weight once."""
    total = 0
    for o in objs:
        st = o.stats()
        total += st["bytes_per_eval"]
    return total


def gradient_leg(api, torch):
    """n = 8, HEA-40, TFIM (960 parameters): the adjoint gradient (checkpoint
    every 5 layers, eager and replayed as a graph) against the
    parameter-shift gradient (pp_psr_gradient: its 1,920 shifted evaluations
    run as one parameter sweep, the combine on the device).  Returns the
    timing record and the gradients, which the oracle leg checks."""
    from paper_2502_10685_amd import workloads as W
    wc = W.config4()
    c = api.Circuit.from_workload(wc)
    ev, g_adj = c.gradient(5 * 32)
    g_psr = c.psr_gradient()
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        c.gradient(5 * 32)
    torch.cuda.synchronize()
    t_adj = (time.perf_counter() - t0) / reps
    cg = api.Circuit.from_workload(wc, use_graph=True)
    cg.gradient(5 * 32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        cg.gradient(5 * 32)
    torch.cuda.synchronize()
    t_adj_graph = (time.perf_counter() - t0) / reps
    cg.close()
    t0 = time.perf_counter()
    for _ in range(reps):
        c.psr_gradient()
    torch.cuda.synchronize()
    t_psr = (time.perf_counter() - t0) / reps
    n_psr = 2 * int(np.sum(wc.op >= 3))
    u_eval = int(count_updates(api, [wc], "f64")[0][0])
    g_adj = g_adj.cpu().numpy()
    g_psr = g_psr.cpu().numpy()
    c.close()
    rec = {"workload": "n=8 HEA-40 (1280 gates, 960 theta), TFIM, FP64",
           "adjoint_ms": t_adj * 1e3, "adjoint_graph_ms": t_adj_graph * 1e3,
           "psr_ms": t_psr * 1e3, "psr_evaluations": n_psr,
           "psr_evaluations_per_s": n_psr / t_psr,
           "psr_updates_per_s": n_psr * u_eval / t_psr,
           "adjoint_speedup_vs_psr": t_psr / t_adj,
           "max_abs_adjoint_minus_psr": float(np.max(np.abs(g_adj - g_psr)))}
    return rec, {"circuit": wc, "adjoint": g_adj, "psr": g_psr, "expval": float(ev.item())}


def sparse_leg(api, torch, engines=("frame", "graph", "sortmerge")):
    """The SPARSE engine past the dense range (n = 20, 4^n slots): a seeded
    300-gate random circuit (2.66M strings at the end) and the spread circuit
    (n = 20, RY on 5 qubits: 7,962,624 strings).  Each is timed with the
    Clifford-frame engine (the default for exact runs with n <= 31; eager and
    replayed as a captured hipGraph) and with the sort-merge engine (the
    radix sort at the tuned shape of its capacity class); both must leave the
    same <O> and the same term-update count."""
    from paper_2502_10685_amd import _lib as L
    from paper_2502_10685_amd import workloads as W
    cases = [("random n=20 m=300 seed 20", W.random_circuit(np.random.default_rng(20), 20, 300, W.obs_z(20, [0, 1]))),
             ("spread n=20 k=5", W.spread_circuit(20, 20, 5))]
    out = []
    for name, wc in cases:
        row = {"workload": name, "gates": wc.m}
        for frame, graph in ((1, False), (1, True), (0, False)):
            if (frame, graph) != (1, False) and {(1, True): "graph", (0, False): "sortmerge"}[(frame, graph)] \
                    not in engines:
                continue
            c = api.Circuit.from_workload(wc, engine="sparse", max_terms=1 << 24, use_graph=graph)
            c.set_option(L.PP_OPT_SPARSE_FRAME, frame)
            c.evaluate()
            torch.cuda.synchronize()
            reps = 5
            t0 = time.perf_counter()
            for _ in range(reps):
                ev = c.evaluate()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            st = c.stats()
            if frame and graph:
                row.update({"ms_graph": dt * 1e3, "updates_per_s_graph": st["term_updates"] / dt,
                            "expval_graph": float(ev.item())})
            elif frame:
                row.update({"engine": "clifford frame", "ms": dt * 1e3, "final_terms": int(st["final_terms"]),
                            "term_updates": int(st["term_updates"]), "passes": int(st["passes"]),
                            "updates_per_s": st["term_updates"] / dt, "overflow": bool(st["overflow"]),
                            "expval": float(ev.item())})
            else:
                cls = 2  # capacity 2^24 strings
                row["sort_merge"] = {
                    "ms": dt * 1e3, "updates_per_s": st["term_updates"] / dt, "expval": float(ev.item()),
                    "sort_shape": L.tune_get(L.PP_TUNE_SORT_SHAPE, cls),
                    "same_updates_as_frame": int(st["term_updates"]) == row["term_updates"],
                    "expval_abs_diff_vs_frame": abs(float(ev.item()) - row["expval"])}
            c.close()
        out.append(row)
    if "sortmerge" not in engines:
        return out
    # truncated propagation past the exact method's reach (approximate; the
    # dropped weight bounds the error of <O>)
    wc = W.random_circuit(np.random.default_rng(32), 32, 400, W.obs_z(32, [0, 1]))
    c = api.Circuit.from_workload(wc, engine="sparse", max_terms=1 << 24)
    c.set_truncation(1e-7, 64)
    c.evaluate()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        ev = c.evaluate()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    st = c.stats()
    out.append({"workload": "random n=32 m=400 seed 32, truncated (|c| >= 1e-7)", "gates": wc.m,
                "ms": dt * 1e3, "final_terms": int(st["final_terms"]), "term_updates": int(st["term_updates"]),
                "updates_per_s": st["term_updates"] / dt, "overflow": bool(st["overflow"]),
                "expval": float(ev.item()), "dropped_weight_bound": c.truncation_dropped()})
    c.close()
    return out


def ramp_leg(api, torch):
    """DENSE evaluations with and without the Clifford-frame ramp
    (PP_OPT_FRAME_RAMP = 6: the frame runs the gates over which the set
    stays below 4^n / 64): a random circuit (the set fills 4^n within a few
    dozen rotations) and a Clifford-heavy one (5 % rotations, the set stays
    small for most of the circuit), both n = 12."""
    from paper_2502_10685_amd import workloads as W
    rng = np.random.default_rng(12)
    gates, p = W.random_gates(rng, 12, 4000)
    ops = np.asarray(gates[0]).copy()
    rot = ops >= 3
    keep = ~rot | (rng.random(len(ops)) < 0.1)  # about 5 % rotations left
    g2 = tuple(np.asarray(a)[keep] for a in gates)
    # renumber the kept rotations' parameters
    par = np.full(len(g2[0]), -1, np.int32)
    rmask = g2[0] >= 3
    par[rmask] = np.arange(int(rmask.sum()), dtype=np.int32)
    cliff = W.make_circuit(12, (g2[0], g2[1], g2[2], par), int(rmask.sum()), W.obs_z(12, [0, 1]),
                           rng.uniform(0, 2 * np.pi, int(rmask.sum())))
    cases = [("random n=12 m=3000 seed 12", W.random_circuit(np.random.default_rng(12), 12, 3000, W.obs_z(12, [0, 1]))),
             (f"Clifford-heavy n=12 m={cliff.m} ({int(rmask.sum())} rotations)", cliff)]
    out = []
    for name, wc in cases:
        row = {"workload": name}
        for ramp in (0, 6):
            c = api.Circuit.from_workload(wc, engine="dense", frame_ramp=ramp)
            c.evaluate()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                ev = c.evaluate()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 5
            st = c.stats()
            row["ramp" if ramp else "plain"] = {"ms": dt * 1e3, "passes": int(st["passes"]), "expval": float(ev.item())}
            c.close()
        row["speedup"] = row["plain"]["ms"] / row["ramp"]["ms"]
        row["expval_abs_diff"] = abs(row["plain"]["expval"] - row["ramp"]["expval"])
        out.append(row)
    return out


def density_leg(api, torch):
    """The paper's toDM task (rho = U|0><0|U^dag, pp_density_matrix) on its
    timing shape (n = 4, 60,200 gates: CX ring + RZ RX RZ blocks) and on a
    seeded n = 10, 5,000-gate random circuit; trace and purity as checks."""
    from paper_2502_10685_amd import workloads as W
    cases = [("chain n=4 60,200 gates", W.chain_zxz_circuit()),
             ("random n=10 m=5000 seed 10", W.random_circuit(np.random.default_rng(10), 10, 5000))]
    out = []
    for name, wc in cases:
        c = api.Circuit.from_workload(wc)
        rho = c.density_matrix()
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            rho = c.density_matrix()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        tr = complex(torch.trace(rho).item())
        purity = float((rho.abs() ** 2).sum().item())
        out.append({"workload": name, "gates": wc.m, "ms": dt * 1e3, "trace_minus_1": abs(tr - 1.0),
                    "purity_minus_1": abs(purity - 1.0)})
        c.close()
    return out


def density_sweep_leg(api, torch):
    """toDM over the two sweeps of the paper's timing study (Sec. V, the
    W_chain+ZXZ ansatz at n = 2..4): #Layers = 1..1000 at #Repeats = 1, and
    #Repeats = 1..100 at #Layers = 50.  One seeded theta per point; the time
    is the mean of 5 calls after one untimed call."""
    from paper_2502_10685_amd import workloads as W
    grid = [("layers", n, L, 1) for n in (2, 3, 4) for L in (1, 10, 100, 1000)]
    grid += [("repeats", n, 50, R) for n in (2, 3, 4) for R in (1, 10, 100)]
    out = []
    for sweep, n, layers, repeats in grid:
        wc = W.chain_zxz_circuit(seed=1000 * n + layers + repeats, n=n, layers=layers, repeats=repeats)
        c = api.Circuit.from_workload(wc)
        rho = c.density_matrix()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            rho = c.density_matrix()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 5
        out.append({"sweep": sweep, "n": n, "layers": layers, "repeats": repeats, "gates": wc.m,
                    "ms": dt * 1e3, "trace_minus_1": abs(complex(torch.trace(rho).item()) - 1.0)})
        c.close()
    return out


def stabilizer_order_leg(api, torch):
    """The stabilizer order of the paper's Sec. II-B: the number of Pauli
    strings in a generator Z_j evolved forward, U_k Z_j U_k^dag, after the
    first k gates of the W_chain+ZXZ ansatz (n = 2..4, two layers of one
    repeat), the largest over j.  A tracked GPU run propagates Z_j backwards
    through the k gates in reverse order: H and CX are self-inverse, S and
    its inverse map X and Y into each other alike, and R(-t) splits the
    same strings as R(t), so the string set has the forward set's size
    (zero weights are kept)."""
    from paper_2502_10685_amd import workloads as W
    out = []
    for n in (2, 3, 4):
        wc = W.chain_zxz_circuit(seed=n, n=n, layers=2, repeats=1)
        counts = []
        for k in range(wc.m + 1):
            best = 0
            for j in range(n):
                rev = W.make_circuit(n, (np.ascontiguousarray(wc.op[:k][::-1]), np.ascontiguousarray(wc.q0[:k][::-1]),
                                         np.ascontiguousarray(wc.q1[:k][::-1]),
                                         np.ascontiguousarray(wc.param[:k][::-1])),
                                     wc.n_params, W.obs_z(n, [j]), wc.theta)
                c = api.Circuit.from_workload(rev, track=True)
                c.evaluate()
                best = max(best, int(c.stats()["final_terms"]))
                c.close()
            counts.append(best)
        out.append({"n": n, "gates": list(range(wc.m + 1)), "max_order": counts, "bound": 4 ** n - 1})
    return out


# Gates of each sampled circuit the timed oracle run propagates, per n: the
# whole circuit for n <= 6, else its last L gates (the first L a Heisenberg
# propagation meets), about 6e7 term updates each once the set is saturated
ORACLE_SUFFIX = {7: 4000, 8: 1000, 9: 400, 10: 280}


def cpu_baseline(circs, updates, checks):
    """The CPU oracle on the host's cores (one process per circuit).

    Timing: the scalar Pauli propagator on every 8th circuit of the workload
    (the whole circuit for n <= 6, else a suffix sized by ORACLE_SUFFIX),
    run across all worker processes at once: `value` is the measured
    aggregate rate.  Per-n single-process rates give an extrapolated time for
    the whole batch (labelled as such).

    Errors: every GPU result of the benchmark against the oracle's FP64 state
    vector (all batch outputs in FP64 and FP32, every served value) and the
    adjoint and parameter-shift gradients against the oracle's
    parameter-shift rule."""
    from oracle import pool
    workers = pool.default_workers()
    sample = list(range(0, len(circs), 8)) if len(circs) > 1 else [0]
    jobs = [("propagate", circs[i], ORACLE_SUFFIX.get(circs[i].n, circs[i].m)) for i in sample]
    res, wall, workers = pool.run(jobs, workers)
    done_u = sum(r["updates"] for r in res)
    busy = sum(r["seconds"] for r in res)
    per_n = {}
    for i, r in zip(sample, res):
        d = per_n.setdefault(int(circs[i].n), {"circuits": 0, "updates": 0, "seconds": 0.0})
        d["circuits"] += 1
        d["updates"] += int(r["updates"])
        d["seconds"] += r["seconds"]
    for d in per_n.values():
        d["updates_per_s_one_process"] = d["updates"] / d["seconds"] if d["seconds"] > 0 else None
    est = 0.0
    for w, u in zip(circs, updates):
        rate = per_n.get(int(w.n), {}).get("updates_per_s_one_process")
        if rate is None:  # an n the sample missed: the nearest sampled n
            near = min(per_n, key=lambda k: abs(k - int(w.n)))
            rate = per_n[near]["updates_per_s_one_process"]
        est += float(u) / rate
    out = {"value": done_u / wall, "unit": "Pauli-term updates/s", "cores": workers, "kind": "oracle",
           "host_cpus": os.cpu_count(), "cpu_model": pool.cpu_model(),
           "sample": (f"scalar Pauli propagator (C, merge after every gate), one process per circuit on "
                      f"{workers} worker processes, on every 8th circuit of the workload ({len(sample)} circuits; "
                      f"circuits with n >= 7 timed on their last {ORACLE_SUFFIX} gates): "
                      f"{done_u:.3e} updates in {wall:.1f} s wall ({busy:.1f} s summed over processes)"),
           "per_n": {str(k): per_n[k] for k in sorted(per_n)},
           "batch_seconds_extrapolated": est / workers,
           "batch_updates_per_s_extrapolated": float(np.sum(updates)) / (est / workers),
           "extrapolation": ("whole batch from the per-n one-process rates, split evenly over the worker "
                             "processes (independent circuits)")}
    # every GPU result against the oracle's state vector / parameter-shift rule
    cjobs, slots = [], []
    for i, w in enumerate(circs):
        cjobs.append(("sv", w, None))
        slots.append(("batch", i))
    for k, (ws, _) in enumerate(checks.get("served", [])):
        for j, w in enumerate(ws):
            cjobs.append(("sv", w, None))
            slots.append(("served", (k, j)))
    if "gradient" in checks:
        cjobs.append(("psr", checks["gradient"]["circuit"], None))
        slots.append(("psr", 0))
    cres, cwall, _ = pool.run(cjobs, workers)
    sv_batch = np.array([r["expval"] for (kind, _), r in zip(slots, cres) if kind == "batch"])
    errs = {"checked_on": f"{len(cjobs)} oracle runs in {cwall:.1f} s wall on {workers} processes"}
    errs["batch_fp64_max_abs_vs_statevector"] = float(np.max(np.abs(checks["batch_f64"] - sv_batch)))
    if checks.get("batch_f32") is not None:
        errs["batch_fp32_max_abs_vs_statevector"] = float(np.max(np.abs(checks["batch_f32"] - sv_batch)))
    if checks.get("batch_graph_f64") is not None:
        errs["batch_graph_fp64_max_abs_vs_statevector"] = float(np.max(np.abs(checks["batch_graph_f64"] - sv_batch)))
    if checks.get("served"):
        sv_served = {}
        for (kind, key), r in zip(slots, cres):
            if kind == "served":
                sv_served[key] = r["expval"]
        errs["served_max_abs_vs_statevector"] = [
            float(max(abs(vals[j] - sv_served[(k, j)]) for j in range(len(vals))))
            for k, (_, vals) in enumerate(checks["served"])]
        errs["served_requests_checked"] = int(sum(len(v) for _, v in checks["served"]))
    if "gradient" in checks:
        g_orc = [r["grad"] for (kind, _), r in zip(slots, cres) if kind == "psr"][0]
        g = checks["gradient"]
        errs["gradient_adjoint_max_abs_vs_oracle_psr"] = float(np.max(np.abs(g["adjoint"] - g_orc)))
        errs["gradient_psr_max_abs_vs_oracle_psr"] = float(np.max(np.abs(g["psr"] - g_orc)))
    out["errors"] = errs
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch512")
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the gradient leg")
    ap.add_argument("--no-sparse", action="store_true", help="skip the SPARSE engine leg")
    ap.add_argument("--sparse-engines", default="frame,graph,sortmerge",
                    help="parts of the SPARSE leg: the Clifford-frame engine eager (always), 'graph' (the same "
                         "replayed as a hipGraph), 'sortmerge' (the sort-merge engine and the truncated run)")
    ap.add_argument("--no-density", action="store_true", help="skip the density-matrix (toDM) leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replayed batch leg")
    ap.add_argument("--no-ramp", action="store_true", help="skip the frame-ramp leg (it runs with the SPARSE leg)")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--autotune", action="store_true",
                    help="time the tuning candidates on this device first (defaults are MI355X measurements)")
    ap.add_argument("--tune", default="",
                    help="tuning knobs, e.g. 'kernel:6=1,qubits:12=7,sort:2=3' (tile kernel variant per k, tile "
                         "qubits per n, radix-sort shape per SPARSE capacity class)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}): the library has no multi-GPU "
              "path; how it would shard is described but not implemented", file=sys.stderr)
        return 2

    import torch
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": src.numel() * 8,
                          "bytes_written": dst.numel() * 8, "launches": 3}))
        return 0

    from paper_2502_10685_amd import _lib as L
    from paper_2502_10685_amd import api

    for item in filter(None, args.tune.split(",")):
        what, rest = item.split(":")
        idx, val = rest.split("=")
        key = {"kernel": L.PP_TUNE_TILE_KERNEL, "qubits": L.PP_TUNE_TILE_QUBITS, "resblock": L.PP_TUNE_RESIDENT_BLOCK,
               "sort": L.PP_TUNE_SORT_SHAPE}
        L.tune_set(key[what], int(idx), int(val))

    tuned = None
    if args.autotune:
        from paper_2502_10685_amd import autotune
        t0 = time.time()
        tuned = autotune.tune(sizes=(8, 9, 10, 11, 12), dtype=args.dtype, save=False, log=log)
        tuned["seconds"] = time.time() - t0

    circs, desc = build_workload(args.workload)
    log(f"workload {args.workload}: {len(circs)} circuits, {sum(w.m for w in circs)} gates")
    U, T = count_updates(api, circs, args.dtype)
    u_step = int(U.sum())
    log(f"term updates per step {u_step:.4e}")

    objs = [api.Circuit.from_workload(w, dtype=args.dtype) for w in circs]
    out = torch.empty(len(objs), dtype=torch.float64, device="cuda")

    def step():
        if len(objs) == 1:
            objs[0].evaluate(out[0])
        else:
            api.evaluate_batch(objs, out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    L.profile_enable(True)
    L.profile_read()
    total_s, lat = timed_steps(step, args.steps, torch)
    prof = L.profile_read()
    L.profile_enable(False)
    gpu_vals = out.cpu().numpy().copy()
    checks = {"batch_f64": gpu_vals}  # GPU results the oracle leg checks
    value = u_step * args.steps / total_s
    log(f"batched: {total_s / args.steps * 1e3:.2f} ms/step, {value:.4e} updates/s")

    # dominant kernel and its roofline
    dom = max(prof.items(), key=lambda kv: kv[1][1]) if prof else ("none", (0, 0.0))
    dname, (dlaunch, dms) = dom
    bytes_step = dense_bytes(objs)
    if dname == "tile_pass" and dlaunch:
        alg_bytes = bytes_step * args.steps
        achieved = alg_bytes / (dms * 1e-3) / 1e9
        kname = TILE_KERNEL_NAMES.get(L.tune_get(L.PP_TUNE_TILE_KERNEL, 6), "tile_kernel")
        roof = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "traffic": measured_traffic(kname, args.workload, args.dtype),
                "launches": dlaunch, "avg_launch_us": dms * 1e3 / dlaunch,
                "alg_bytes_per_launch": alg_bytes / dlaunch}
    else:
        roof = {"kernel": dname, "bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "launches": dlaunch,
                "avg_launch_us": dms * 1e3 / max(dlaunch, 1)}
    kernels = {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in prof.items()}
    # per-gate streaming figure of merit: the HBM time a propagator that reads
    # and writes every live term (key + weight) at every gate would need,
    # relative to the measured time (48 B per update FP64, 40 B FP32)
    b_upd = 48.0 if args.dtype == "f64" else 40.0
    streaming = {"bytes_per_update": b_upd, "frac": value * b_upd / (PEAK_HBM_GBS * 1e9),
                 "note": "updates/s x bytes per update / 8 TB/s; above 1 because a tile pass carries many gates "
                         "per HBM round trip"}

    res = {"metric": METRIC, "value": value, "unit": "Pauli-term updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_s / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
           "data": "synthetic",
           "config": {"workload": f"{args.workload}: {desc}", "circuits": len(circs),
                      "gates": int(sum(w.m for w in circs)), "term_updates_per_step": u_step,
                      "engine": "dense (direct-address), LDS-resident n<=7, LDS-tiled passes n>=8"},
           "circuits_per_s": len(circs) * args.steps / total_s,
           "step_latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                               "p99": float(np.percentile(lat, 99) * 1e3)},
           "kernels": kernels, "roofline": roof, "per_gate_streaming_roofline": streaming,
           "paper_reference": {
               "figure": "4.23x faster than Qiskit 1.1.1 (toDM: full density matrix), n = 4, 60.2K gates",
               "hardware": "Intel i9-10940X @ 3.30 GHz, Python 3.11 + JAX (one CPU)",
               "comparable": False,
               "layers_sweep_s": {"n=2": {"pstabilizer": 0.157, "qiskit": 0.4578},
                                  "n=4": {"pstabilizer": 0.7789, "qiskit": 1.1158},
                                  "point": "not stated; read as the sweep's end, #Layers = 1000, #Repeats = 1"},
               "note": "the paper times toDM (the full density matrix); the density_matrix and density_sweep "
                       "fields time the same task on its gate shapes here, a different machine, so the figures "
                       "stay context"}}
    if tuned is not None:
        res["autotune"] = {"tile_kernel": tuned["tile_kernel"], "tile_qubits": tuned["tile_qubits"],
                           "resident_block": tuned["resident_block"], "sort_shape": tuned.get("sort_shape"),
                           "seconds": round(tuned["seconds"], 1)}

    if not args.no_graph and len(objs) > 1:
        # the same step captured once as a hipGraph and replayed (theta is
        # read from device memory at replay); its outputs must equal the
        # eager step's bit for bit
        for o in objs:
            o.set_option(L.PP_OPT_USE_GRAPH, 1)
        outg = torch.empty_like(out)

        def gstep():
            api.evaluate_batch(objs, outg)
        gstep()
        torch.cuda.synchronize()
        gs, glat = timed_steps(gstep, args.steps, torch)
        gv = outg.cpu().numpy()
        res["batch_graph"] = {
            "ms_per_step": gs / args.steps * 1e3, "value": u_step * args.steps / gs,
            "speedup_vs_eager": (total_s / gs), "bitwise_equal_to_eager": bool(
                np.array_equal(gv.view(np.uint64), gpu_vals.view(np.uint64))),
            "step_latency_ms": {"p50": float(np.percentile(glat, 50) * 1e3),
                                "p99": float(np.percentile(glat, 99) * 1e3)}}
        checks["batch_graph_f64"] = gv
        for o in objs:
            o.set_option(L.PP_OPT_USE_GRAPH, 0)
        log(f"graph-replayed batch: {gs / args.steps * 1e3:.2f} ms/step")

    if not args.no_plain and len(objs) > 1:
        def plain():
            for i, o in enumerate(objs):
                o.evaluate(out[i])
        plain()
        ps, plat = timed_steps(plain, 1, torch)
        res["plain"] = {"ms_per_step": ps * 1e3, "value": u_step / ps,
                        "speedup_batched_vs_plain": ps / (total_s / args.steps)}
        log(f"plain: {ps * 1e3:.2f} ms/step")

    if not args.no_fp32 and args.dtype == "f64":
        objs32 = [api.Circuit.from_workload(w, dtype="f32") for w in circs]
        out32 = torch.empty(len(objs32), dtype=torch.float64, device="cuda")

        def step32():
            if len(objs32) == 1:
                objs32[0].evaluate(out32[0])
            else:
                api.evaluate_batch(objs32, out32)
        step32()
        L.profile_enable(True)
        L.profile_read()
        s32, _ = timed_steps(step32, args.steps, torch)
        prof32 = L.profile_read()
        L.profile_enable(False)
        v32 = out32.cpu().numpy()
        checks["batch_f32"] = v32
        res["fp32"] = {"value": u_step * args.steps / s32, "ms_per_step": s32 / args.steps * 1e3,
                       "max_abs_diff_vs_fp64": float(np.max(np.abs(v32 - gpu_vals)))}
        t32 = prof32.get("tile_pass")
        if t32 and t32[0]:
            # the same kernel on FP32 weights: half the algorithmic bytes
            b32 = dense_bytes(objs32) * args.steps
            a32 = b32 / (t32[1] * 1e-3) / 1e9
            res["fp32"]["roofline"] = {
                "kernel": TILE_KERNEL_NAMES.get(L.tune_get(L.PP_TUNE_TILE_KERNEL, 6), "tile_kernel"),
                "bound": "hbm", "achieved": a32, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": a32 / PEAK_HBM_GBS,
                "launches": t32[0], "avg_launch_us": t32[1] * 1e3 / t32[0], "alg_bytes_per_launch": b32 / t32[0]}
        log(f"fp32: {s32 / args.steps * 1e3:.2f} ms/step")
        del objs32

    if not args.no_serve and args.workload == "batch512":
        res["serving"] = []
        for lam in (100.0, 1000.0):
            log(f"serving lambda={lam:.0f}/s")
            sv, sws, svals = serve(api, lam, args.serve_requests, budget=64 << 30, max_active=64)
            checks.setdefault("served", []).append((sws, svals))
            log(f"serving lambda={lam:.0f}: p50 {sv['latency_ms']['p50']:.1f} ms, p99 "
                f"{sv['latency_ms']['p99']:.1f} ms, {sv['updates_per_s']:.3e} updates/s")
            res["serving"].append(sv)

    if not args.no_grad and args.workload == "batch512":
        log("gradient: adjoint vs parameter-shift sweep")
        res["gradient"], checks["gradient"] = gradient_leg(api, torch)
        log(f"gradient: adjoint {res['gradient']['adjoint_ms']:.2f} ms, psr sweep "
            f"{res['gradient']['psr_ms']:.2f} ms")

    if not args.no_sparse and args.workload == "batch512":
        log("sparse engine: n = 20")
        res["sparse"] = sparse_leg(api, torch, tuple(args.sparse_engines.split(",")))
        for r in res["sparse"]:
            log(f"sparse {r['workload']}: {r['ms']:.2f} ms"
                + (f" ({r['ms_graph']:.2f} ms as a graph)" if "ms_graph" in r else "")
                + f", {r['final_terms']} strings, {r['updates_per_s']:.3e} updates/s")

    if not args.no_sparse and not args.no_ramp and args.workload == "batch512":
        res["frame_ramp"] = ramp_leg(api, torch)
        for r in res["frame_ramp"]:
            log(f"frame ramp {r['workload']}: {r['plain']['ms']:.2f} ms plain, {r['ramp']['ms']:.2f} ms with the ramp")

    if not args.no_density and args.workload == "batch512":
        log("density matrix (toDM)")
        res["density_matrix"] = density_leg(api, torch)
        for r in res["density_matrix"]:
            log(f"toDM {r['workload']}: {r['ms']:.3f} ms (|Tr rho - 1| {r['trace_minus_1']:.1e})")
        res["stabilizer_order"] = stabilizer_order_leg(api, torch)
        for r in res["stabilizer_order"]:
            log(f"stabilizer order n={r['n']}: {r['max_order']} (bound {r['bound']})")
        res["density_sweep"] = density_sweep_leg(api, torch)
        for sweep in ("layers", "repeats"):
            pts = [r for r in res["density_sweep"] if r["sweep"] == sweep]
            log(f"toDM #{sweep} sweep: " + ", ".join(f"n={r['n']} L={r['layers']} R={r['repeats']} {r['ms']:.3f} ms"
                                                    for r in pts))

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(circs, U, checks)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
