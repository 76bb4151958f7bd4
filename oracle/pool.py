"""Oracle jobs across host cores -- TEST INFRASTRUCTURE ONLY.

Runs the oracle's functions on many independent circuits at once, one job per
worker process (processes started fresh, so a parent that has opened the GPU
is not copied into them).  Used by the benchmark's CPU-baseline leg to time
the scalar propagator on all host cores and to check every GPU result
against the state vector.  Nothing here is reached from the GPU library.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import time
from concurrent.futures import ProcessPoolExecutor


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def default_workers(cap: int = 16) -> int:
    """Worker processes: the host's cores, at most `cap`."""
    return max(1, min(cap, os.cpu_count() or 1))


def _suffix(circ, L):
    """The circuit's last L gates (the first L a Heisenberg propagation meets)."""
    from paper_2502_10685_amd import workloads as W
    m = circ.m
    L = min(L, m)
    return W.make_circuit(circ.n, (circ.op[m - L:], circ.q0[m - L:], circ.q1[m - L:], circ.param[m - L:]),
                          circ.n_params, (circ.obs_x, circ.obs_z, circ.obs_c), circ.theta)


def _job(kind, circ, arg):
    import oracle
    t0 = time.perf_counter()
    if kind == "propagate":  # timed scalar propagation of the last `arg` gates
        r = oracle.propagate(_suffix(circ, arg))
        return {"updates": r.updates, "seconds": time.perf_counter() - t0, "expval": r.expval,
                "gates": min(arg, circ.m), "n": circ.n}
    if kind == "sv":  # <O> from the FP64 state vector
        return {"expval": oracle.expval_sv(circ), "seconds": time.perf_counter() - t0}
    if kind == "psr":  # parameter-shift gradient on the state vector
        return {"grad": oracle.psr_gradient(circ), "seconds": time.perf_counter() - t0}
    raise ValueError(kind)


def run(jobs, workers=None):
    """jobs: list of (kind, circuit, arg).  Returns (results in job order,
    wall seconds, workers used)."""
    workers = workers or default_workers()
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        futs = [ex.submit(_job, k, c, a) for k, c, a in jobs]
        out = [f.result() for f in futs]
    return out, time.perf_counter() - t0, workers
