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
    elif name == "hea8":
        circs = [W.config4()]
        desc = "n=8, HEA 40 layers (1,280 gates, 960 params), O=TFIM (15 terms), seed 4"
    elif name in ("rand10", "rand12"):
        n = int(name[4:])
        circs = [W.random_circuit(10 + n, n, 6000, W.obs_z(n, [0, 1]))]
        desc = f"n={n}, 6,000 random gates (50% Clifford), O=Z0Z1, seed {10 + n}"
    else:
        raise SystemExit(f"unknown workload {name}")
    return circs, desc


def count_updates(api, circs, dtype):
    """U per circuit from one tracked GPU run each (structure only: U does not
    depend on theta)."""
    us, terms = [], []
    t0 = time.time()
    for i, w in enumerate(circs):
        c = api.Circuit.from_workload(w, dtype=dtype, track=True)
        c.evaluate()
        st = c.stats()
        us.append(st["term_updates"])
        terms.append(st["final_terms"])
        c.close()
        if (i + 1) % 128 == 0:
            log(f"tracked runs {i + 1}/{len(circs)} ({time.time() - t0:.1f}s)")
    return np.array(us, dtype=np.int64), np.array(terms, dtype=np.int64)


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


def dense_bytes(objs):
    """Algorithmic HBM bytes of one evaluation of each tiled circuit: every
    pass reads and writes each 4^n weight once."""
    total = 0
    for o in objs:
        st = o.stats()
        total += st["bytes_per_eval"]
    return total


def cpu_baseline(circs, gpu_vals, seconds, updates):
    """The oracle's scalar propagator on a bounded sample of the workload: every
    8th circuit whose estimated cost still fits the time budget."""
    import oracle
    done_u, spent, maxerr, names = 0, 0.0, 0.0, []
    order = list(range(0, len(circs), 8)) if len(circs) > 1 else [0]
    rate_guess = 5.0e6  # updates/s of the oracle on one core, for budgeting only
    picked = [i for i in order if updates[i] / rate_guess <= seconds]
    if not picked:
        picked = [min(order, key=lambda i: updates[i])]
    for i in picked:
        if spent > 0 and spent + updates[i] / rate_guess > seconds:
            continue
        t0 = time.perf_counter()
        r = oracle.propagate(circs[i])
        dt = time.perf_counter() - t0
        spent += dt
        done_u += r.updates
        maxerr = max(maxerr, abs(r.expval - gpu_vals[i]))
        names.append(i)
        if spent >= seconds:
            break
    return {"value": done_u / spent if spent > 0 else None, "unit": "Pauli-term updates/s",
            "cores": 1, "kind": "oracle",
            "sample": (f"scalar Pauli propagator (C, merge after every gate, 1 thread) on {len(names)} "
                       f"of the workload's circuits (every 8th that fits a {seconds:.0f}s budget: "
                       f"{names[:10]}{'...' if len(names) > 10 else ''}), "
                       f"{done_u:.3e} updates in {spent:.1f}s"),
            "max_abs_err_vs_gpu": maxerr}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch512")
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}); the multi-GPU path is a "
              "design only in this build", file=sys.stderr)
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
    value = u_step * args.steps / total_s
    log(f"batched: {total_s / args.steps * 1e3:.2f} ms/step, {value:.4e} updates/s")

    # dominant kernel and its roofline
    dom = max(prof.items(), key=lambda kv: kv[1][1]) if prof else ("none", (0, 0.0))
    dname, (dlaunch, dms) = dom
    bytes_step = dense_bytes(objs)
    if dname == "tile_pass" and dlaunch:
        alg_bytes = bytes_step * args.steps
        achieved = alg_bytes / (dms * 1e-3) / 1e9
        roof = {"kernel": "tile_kernel", "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "launches": dlaunch, "avg_launch_us": dms * 1e3 / dlaunch,
                "alg_bytes_per_launch": alg_bytes / dlaunch}
    else:
        roof = {"kernel": dname, "bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "launches": dlaunch,
                "avg_launch_us": dms * 1e3 / max(dlaunch, 1)}
    kernels = {k: {"launches": v[0], "ms_per_step": v[1] / args.steps} for k, v in prof.items()}

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
           "kernels": kernels, "roofline": roof}

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
        s32, _ = timed_steps(step32, args.steps, torch)
        v32 = out32.cpu().numpy()
        res["fp32"] = {"value": u_step * args.steps / s32, "ms_per_step": s32 / args.steps * 1e3,
                       "max_abs_diff_vs_fp64": float(np.max(np.abs(v32 - gpu_vals)))}
        log(f"fp32: {s32 / args.steps * 1e3:.2f} ms/step")
        del objs32

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(circs, gpu_vals, args.cpu_seconds, U)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
